"""Host logic of the training driver: the multiscale schedule (Sec. 5.3) and
the learning-rate drop."""
from paper_2306_17486_amd import train


def test_schedule_follows_the_16_to_10_weighting():
    s = train.schedule(2000, 100)
    assert len(s) == 20
    assert s.count(128) == 12 and s.count(256) == 8
    # the sizes alternate: never more than two blocks of the small grid in a row
    assert all(not (s[i] == s[i + 1] == s[i + 2] == 128) for i in range(len(s) - 2))
    assert s[0] == 128


def test_learning_rate_drops_tenfold_for_the_last_quarter():
    lr = [train.learning_rate(i, 2000, 1e-3) for i in range(2000)]
    assert lr[0] == lr[1499] == 1e-3
    assert lr[1500] == lr[1999] == 1e-4


def test_training_media_alternate_families():
    assert [train.family_of(j) for j in range(4)] == ["grf", "layered", "grf", "layered"]


def test_three_size_schedule_follows_the_16_10_4_epoch_lengths():
    s = train.schedule(3000, 100, sizes=(128, 256, 512))
    assert (s.count(128), s.count(256), s.count(512)) == (16, 10, 4)


def test_gradient_clip_threshold_follows_the_median():
    c = train.GradClip(2.0, window=5, warmup=3)
    assert c.threshold() == 0.0
    for v in (1.0, 3.0, 2.0):
        c.record(v)
    assert c.threshold() == 4.0
    for v in (100.0, 2.0, 2.0, 2.0):
        c.record(v)
    assert c.threshold() == 4.0  # one outlier does not move the median
    assert train.GradClip(0.0, warmup=0).threshold() == 0.0
