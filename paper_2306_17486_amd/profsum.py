"""Summaries of rocprofv3 runs of bench.py, for the profiles/ folder.

  python -m paper_2306_17486_amd.profsum --trace DIR [--fetch DIR --write DIR] [--copy-mib S]
      [--out-md FILE] [--traffic-dir DIR] [--workload TAG]

DIR is a rocprofv3 output directory (-d); the CSV files under it are found by
name (kernel_stats.csv from --kernel-trace --stats, counter_collection.csv
from --pmc).  Kernels are grouped into the classes the library's own event
timing uses (hh_profile_begin).  With the two counter runs, HBM traffic per
dispatch is FETCH_SIZE and WRITE_SIZE (KiB) scaled by what the same counters
read for the plain copy of --copy-mib MiB that bench.py --copy-mib makes
first; per class it is written as <class>_<workload>_traffic.txt files
(key: value lines, with the hash of the class's kernel sources) that bench.py
reports while those sources are unchanged."""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import re
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))

# kernel name prefix -> class (the library's kernel classes)
CLASS_OF = [
    ("k_conv_mfma", "conv"), ("k_conv_t2", "conv"), ("k_conv_in", "conv"), ("k_conv_dma", "conv"),
    ("k_ib_fused", "conv"), ("k_pointwise", "conv"), ("k_depthwise", "conv"), ("k_explicit", "net_other"),
    ("k_conv_out", "net_other"), ("k_implicit", "net_other"), ("k_sumsq", "net_other"),
    ("k_scales", "net_other"), ("k_prolong_x0", "net_other"),
    ("k_op_dots", "op_dots"), ("k_ortho", "ortho"),
    ("k_arnoldi_col", "small"), ("k_givens", "small"), ("k_cycle_begin", "small"),
    ("k_residual64", "restart"), ("k_xupdate", "restart"),
    ("k_vc_down", "vc_down"), ("k_vc_up", "vc_up"),
    # once per medium: coefficients and the coarsest operator's factorisation
    ("k_coef", "setup"), ("k_blkinv", "setup"), ("k_cf_", "setup"), ("k_pf_", "setup"), ("k_tstore", "setup"),
    ("k_cr_tfill", "setup"), ("k_cr_level_prod", "setup"),
    ("k_cr_", "vc_coarse"), ("k_coarse", "vc_coarse"), ("k_cg_", "vc_coarse"),
]

# kernel sources of each class (their hash marks which build the counters saw)
CLASS_SOURCES = {
    "conv": ("net_conv.hip", "net_light.hip", "net.h", "hh_internal.h"),
    "op_dots": ("krylov.hip", "hh_internal.h"),
    "ortho": ("krylov.hip", "hh_internal.h"),
    "vc_down": ("mg.hip", "hh_internal.h"),
    "vc_up": ("mg.hip", "hh_internal.h"),
}


def class_of(name: str) -> str:
    if name.startswith("k_conv_mfma") and re.search(r", true(, \d+)?>$", name.rstrip()):
        return "net_other"  # the projection layer (launched in the library's network-other scope)
    for p, c in CLASS_OF:
        if name.startswith(p):
            return c
    return "other"


def source_sha(cls: str) -> str | None:
    files = CLASS_SOURCES.get(cls)
    if not files:
        return None
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _find(d: str, pattern: str) -> list[str]:
    return sorted(glob.glob(os.path.join(d, "**", pattern), recursive=True))


def _short(name: str) -> str:
    name = re.sub(r"\(.*$", "", name)  # drop the argument list
    name = name.replace("void ", "").replace("hh::", "")
    return name


def read_stats(d: str):
    rows = []
    for f in _find(d, "*kernel_stats.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                rows.append((_short(r["Name"]), int(r["Calls"]), float(r["TotalDurationNs"]) / 1e6,
                             float(r["AverageNs"]) / 1e3))
    return rows


def read_counters(d: str, counter: str):
    """({kernel: (dispatches, summed value)}, {kernel: largest single-dispatch value}) of one counter."""
    acc = defaultdict(lambda: [0, 0.0])
    mx = defaultdict(float)
    for f in _find(d, "*counter_collection.csv"):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                k = _short(r["Kernel_Name"])
                v = float(r["Counter_Value"])
                acc[k][0] += 1
                acc[k][1] += v
                mx[k] = max(mx[k], v)
    return {k: tuple(v) for k, v in acc.items()}, dict(mx)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-mib", type=float, default=256.0)
    ap.add_argument("--out-md")
    ap.add_argument("--traffic-dir")
    ap.add_argument("--workload", default="cnn_mg_1024_64rhs")
    ap.add_argument("--top", type=int, default=40)
    ap.add_argument("--active-rhs", type=int, default=64,
                    help="right-hand sides active in every launch of the counter runs (bench.py --max-iters 30 "
                         "stops before any of the 64 converges)")
    a = ap.parse_args()
    lines = []
    stats = read_stats(a.trace)
    total = sum(r[2] for r in stats)
    lines.append("Kernel trace (rocprofv3 --kernel-trace --stats), top kernels:")
    lines.append(f"{'kernel':60s} {'class':10s} {'calls':>7s} {'total ms':>10s} {'avg us':>10s} {'%':>6s}")
    for name, calls, ms, avg in sorted(stats, key=lambda r: -r[2])[:a.top]:
        lines.append(f"{name[:60]:60s} {class_of(name):10s} {calls:7d} {ms:10.2f} {avg:10.1f} {100 * ms / total:6.2f}")
    lines.append(f"(all kernels: {total:.1f} ms)")
    by_cls = defaultdict(lambda: [0, 0.0])
    for name, calls, ms, avg in stats:
        by_cls[class_of(name)][0] += calls
        by_cls[class_of(name)][1] += ms
    lines.append("")
    lines.append("Per class (summed kernel time over the whole run):")
    for c, (calls, ms) in sorted(by_cls.items(), key=lambda kv: -kv[1][1]):
        lines.append(f"  {c:10s} {calls:7d} dispatches {ms:10.2f} ms")
    if a.fetch and a.write:
        fe, fe_max = read_counters(a.fetch, "FETCH_SIZE")
        wr, wr_max = read_counters(a.write, "WRITE_SIZE")
        # the plain copy of --copy-mib MiB is the largest single copy dispatch
        copy = [k for k in fe if "copy" in k.lower()]
        ref_bytes = a.copy_mib * 1024.0  # KiB
        big = max(copy, key=lambda k: fe_max[k]) if copy else None
        rs = ws = 1.0
        if big and big in wr:
            rs = ref_bytes / fe_max[big]
            ws = ref_bytes / wr_max[big]
            lines.append("")
            lines.append(f"Plain copy of {a.copy_mib:g} MiB ({big}, its largest dispatch): FETCH {fe_max[big]:.0f} "
                         f"KiB, WRITE {wr_max[big]:.0f} KiB -> bytes = FETCH x {rs:.3f}, WRITE x {ws:.3f}")
        lines.append("")
        lines.append("HBM traffic per dispatch (scaled FETCH_SIZE / WRITE_SIZE, MiB):")
        cls_tr = defaultdict(lambda: [0, 0.0, 0.0])
        for k in sorted(fe, key=lambda k: -fe[k][1]):
            if k not in wr:
                continue
            n = fe[k][0]
            rd = fe[k][1] * rs / n / 1024.0
            wt = wr[k][1] * ws / wr[k][0] / 1024.0
            lines.append(f"  {k[:58]:58s} n={n:5d} read {rd:10.2f} write {wt:10.2f}")
            c = class_of(k)
            cls_tr[c][0] += n
            cls_tr[c][1] += fe[k][1] * rs * 1024.0
            cls_tr[c][2] += wr[k][1] * ws * 1024.0 * n / wr[k][0]
        # the convolution class is reported per network application (all its
        # convolution kernels over the active right-hand sides): one implicit-
        # layer dispatch per application
        apps = sum(v[0] for k, v in fe.items() if k.startswith("k_implicit"))
        if a.traffic_dir:
            os.makedirs(a.traffic_dir, exist_ok=True)
            for c, (n, rb, wb) in cls_tr.items():
                sha = source_sha(c)
                if sha is None or n == 0 or c == "vc_coarse":  # the coarse solve: many kernels per V-cycle
                    continue
                unit = "dispatch"
                if c == "conv":
                    if apps == 0:
                        continue
                    n, unit = apps, "network application"
                path = os.path.join(a.traffic_dir, f"{c}_{a.workload}_traffic.txt")
                with open(path, "w") as fh:
                    fh.write(f"# HBM traffic of the {c} kernel class, rocprofv3 FETCH_SIZE and WRITE_SIZE\n")
                    fh.write(f"# (one --pmc run each), scaled by a plain {a.copy_mib:g} MiB copy's readings;\n")
                    fh.write("# per launch unit of the class (below), averaged over the counter runs\n")
                    fh.write(f"class: {c}\n")
                    fh.write(f"unit: {unit}\n")
                    fh.write(f"units: {n}\n")
                    fh.write(f"read_bytes_per_launch: {rb / n:.0f}\n")
                    fh.write(f"write_bytes_per_launch: {wb / n:.0f}\n")
                    fh.write(f"traffic_bytes_per_launch: {(rb + wb) / n:.0f}\n")
                    fh.write(f"active_rhs: {a.active_rhs}\n")
                    fh.write(f"traffic_bytes_per_rhs: {(rb + wb) / n / a.active_rhs:.0f}\n")
                    fh.write(f"read_scale: {rs:.4f}\nwrite_scale: {ws:.4f}\n")
                    fh.write(f"source_sha256_16: {sha}\n")
    text = "\n".join(lines) + "\n"
    if a.out_md:
        with open(a.out_md, "w") as fh:
            fh.write(text)
    print(text)


if __name__ == "__main__":
    main()
