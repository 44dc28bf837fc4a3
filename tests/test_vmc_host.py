"""Host-side schedule of the VMC optimisation loop (no GPU)."""
import math

import pytest

pytest.importorskip("torch")
from paper_2011_07125_amd import vmc  # noqa: E402


def test_learning_rate_schedule():
    assert vmc.learning_rate(0) == 0.05
    assert math.isclose(vmc.learning_rate(10000), 0.025)
    assert math.isclose(vmc.learning_rate(30000, rate=0.1, delay=1e4, decay=2.0), 0.1 / 16)
    lrs = [vmc.learning_rate(t) for t in range(0, 100000, 5000)]
    assert all(a > b for a, b in zip(lrs, lrs[1:]))


def test_adapt_width_moves_towards_target_and_stays_bounded():
    assert math.isclose(vmc.adapt_width(0.1, 0.9), 0.11)
    assert math.isclose(vmc.adapt_width(0.1, 0.1), 0.1 / 1.1)
    assert vmc.adapt_width(0.1, 0.5) == 0.1
    w = 1.0
    for _ in range(200):
        w = vmc.adapt_width(w, 1.0)
    assert w == 10.0
    for _ in range(400):
        w = vmc.adapt_width(w, 0.0)
    assert w == 1e-3
