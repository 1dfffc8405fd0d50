"""Host logic of the learned-rank form (no GPU): the modelled cost of rank
doubling and the calibration of the network's output shift."""
from __future__ import annotations

import math

import numpy as np
import pytest

pytest.importorskip("torch")

from paper_2104_05877_amd import learned as L  # noqa: E402


def test_modelled_cost_counts_doubling_attempts():
    """From 100 to a label of 300: attempts at 100, 200, 400; a censored
    label runs to the cap; a start above the label is one attempt."""
    c0 = 32.0
    assert L.modelled_cost(100, 300, 1024, c0) == (100 + c0) + (200 + c0) + (400 + c0)
    assert L.modelled_cost(300, None, 1024, c0) == (300 + c0) + (600 + c0) + (1024 + c0)
    assert L.modelled_cost(900, 50, 1024, c0) == 900 + c0
    assert L.rank_of(10.5, 0.0, 1024) == 1024 and L.rank_of(-3.0, 0.0, 1024) == 1


def test_calibration_shift_minimises_modelled_cost():
    """The calibrated shift is the grid point of least modelled cost, and a
    network that always under-predicts by 2x is shifted up by about one."""
    labels = [100, 200, 300, None, 50, 700]
    y = [math.log2(k / 2) if k is not None else 9.0 for k in labels]
    d = L.calibrate_shift(y, labels, L.RANK_CAP)
    assert 0.9 <= d <= 1.1, d
    costs = {round(g, 2): sum(L.modelled_cost(L.rank_of(v, g, L.RANK_CAP), lab, L.RANK_CAP)
                              for v, lab in zip(y, labels)) for g in np.arange(-1.0, 2.0001, 0.05)}
    assert costs[round(d, 2)] == min(costs.values())
