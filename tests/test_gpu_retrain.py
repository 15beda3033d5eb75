"""Solve-time re-training on an out-of-distribution medium (Sec. 5.4): pairs
generated on the half-size medium by the library, a few epochs of the
library's own training step, then the network at the full size."""
import os
import sys

import numpy as np
import pytest
import torch

from paper_2306_17486_amd import inputs

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NET_FILE = os.path.join(ROOT, "paper_2306_17486_amd", "weights", "net_ms128_256_512.bin")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.timeout(300)
def test_retrain_on_half_size_medium():
    from paper_2306_17486_amd import hh, retrain
    ctx = hh.Context(0)
    kappa = inputs.salt_slowness(256, 3)
    before = hh.Net.load(ctx, NET_FILE)
    net = hh.Net.load(ctx, NET_FILE)
    p0 = net.get_params()
    rep = retrain.retrain(ctx, net, kappa, npairs=60, epochs=8, batch=30, lr=1e-4, seed=3)
    _say(f"epoch losses {[round(v, 3) for v in rep['epoch_loss']]}")
    assert rep["half_size"] == 128
    assert np.all(np.isfinite(rep["epoch_loss"]))
    # the loss on the medium's own pairs falls, and the parameters moved
    assert rep["epoch_loss"][-1] < rep["epoch_loss"][0]
    assert not np.array_equal(net.get_params(), p0)
    its = retrain.iterations(ctx, kappa, {"before": before, "after": net}, nsrc=2)
    _say(f"iterations at 256^2: {its}")
    assert its["before_converged"] == 2 and its["after_converged"] == 2
    # fine-tuning on the medium does not cost iterations on it (measured at 1024^2:
    # 1-5% fewer with the implicit network, 4-7% with the explicit one)
    assert np.mean(its["after"]) <= 1.1 * np.mean(its["before"])
    assert np.mean(its["after"]) <= 0.5 * np.mean(its["mg"])
    before.close()
    net.close()
    ctx.close()
