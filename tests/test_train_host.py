"""Host logic of the training loop: the patience-based learning-rate schedule."""
import pytest

from paper_2602_17601_amd.train import PatienceScheduler


def test_patience_scheduler_halves_after_a_plateau_and_respects_the_floor():
    s = PatienceScheduler(1e-2, factor=0.5, patience=2, threshold=0.0, min_lr=3e-3)
    assert s.step(1.0) == 1e-2          # improvement
    assert s.step(0.5) == 1e-2          # improvement
    assert s.step(0.6) == 1e-2          # 1 bad epoch
    assert s.step(0.55) == 1e-2         # 2 bad epochs
    assert s.step(0.7) == 5e-3          # 3rd bad epoch > patience: halve, counter reset
    assert s.step(0.4) == 5e-3          # improvement
    for _ in range(3):
        lr = s.step(0.9)
    assert lr == 3e-3                   # halving stops at min_lr


def test_patience_scheduler_threshold_is_relative():
    s = PatienceScheduler(1.0, factor=0.1, patience=0, threshold=0.1)
    s.step(1.0)
    assert s.step(0.95) == pytest.approx(0.1)  # less than 10% better counts as no improvement


def test_patience_scheduler_rejects_bad_settings():
    with pytest.raises(ValueError):
        PatienceScheduler(1.0, factor=1.5)
