"""Host logic of the surrogate's gate (no GPU): the threshold is the largest
uncertainty at which every calibration set at or below it reaches the IoU
target, -inf when even the most certain set misses it."""
import numpy as np

from paper_1709_08018_amd import surrogate as S


def _check(unc, iou, target):
    tau = S.gate_threshold(np.array(unc), np.array(iou), target)
    unc, iou = np.array(unc), np.array(iou)
    # every calibration set at or below tau reaches the target ...
    assert (iou[unc <= tau] >= target).all()
    # ... and tau is the largest such value among the calibration uncertainties
    higher = np.sort(unc[unc > tau])
    if len(higher):
        assert (iou[unc <= higher[0]] < target).any()
    return tau


def test_threshold_stops_at_the_first_failing_set():
    assert _check([0.1, 0.2, 0.3, 0.4], [0.99, 0.97, 0.90, 0.99], 0.95) == 0.2


def test_threshold_takes_every_set_when_all_pass():
    assert _check([0.3, 0.1, 0.2], [0.96, 0.99, 0.97], 0.95) == 0.3


def test_threshold_is_minus_infinity_when_the_most_certain_fails():
    assert _check([0.1, 0.2], [0.5, 0.99], 0.95) == -np.inf


def test_threshold_with_ties_and_random_cases():
    rng = np.random.default_rng(1)
    for _ in range(200):
        n = int(rng.integers(1, 30))
        unc = np.round(rng.random(n), 1)        # ties
        iou = rng.random(n)
        _check(unc, iou, float(rng.random()))
