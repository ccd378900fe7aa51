"""The seeded input generators (no GPU)."""
import numpy as np

from paper_2105_12764_amd import synth


def test_service_stream_is_seeded_and_has_the_stated_mix():
    a = synth.service_requests(4000, seed=5000)
    b = synth.service_requests(4000, seed=5000)
    assert a == b
    sides = np.array([r[0] for r in a], dtype=np.float64)
    f32 = np.mean([r[1] == np.float32 for r in a])
    rec = np.mean([r[2] for r in a])
    gaps = np.array([r[3] for r in a])
    assert abs(f32 - 0.75) < 0.03 and abs(rec - 0.5) < 0.03
    assert abs(gaps.mean() - 1.0) < 0.05
    assert sides.min() >= 17 and sides.max() <= 513 and np.all(sides == np.rint(sides))
    # log-uniform integer side: mean of log(side) at the midpoint of the range,
    # and about a quarter of the sides below exp(quarter point)
    assert abs(np.log(sides).mean() - 0.5 * (np.log(17) + np.log(513))) < 0.05
    q = np.exp(np.log(17) + 0.25 * (np.log(513) - np.log(17)))
    assert abs(np.mean(sides < q) - 0.25) < 0.03
    assert len(np.unique(sides)) > 300
