"""Host logic of the training loop (no GPU): the ADC thresholds are the
paper's, the learning-rate schedule and the view cycle."""
import math
from types import SimpleNamespace

import pytest

from paper_2409_06765_amd.train import GaussianTrainer, TrainConfig


def test_adc_thresholds_are_the_papers():
    c = TrainConfig()
    assert (c.grad_threshold, c.scale_threshold, c.prune_opacity) == (2e-4, 0.01, 0.005)
    assert c.strategy == "adc" and c.split_shrink == 1.6


def test_means_learning_rate_decays_exponentially():
    c = TrainConfig(lr_means=1.6e-4, lr_means_final=1.6e-6, lr_decay_steps=30_000)
    tr = SimpleNamespace(cfg=c, extent=2.0)
    lr = lambda t: GaussianTrainer.lr_means(tr, t)
    assert lr(0) == pytest.approx(2.0 * 1.6e-4, rel=1e-12)
    assert lr(30_000) == pytest.approx(2.0 * 1.6e-6, rel=1e-12)
    assert lr(60_000) == pytest.approx(2.0 * 1.6e-6, rel=1e-12)
    assert lr(15_000) == pytest.approx(2.0 * math.sqrt(1.6e-4 * 1.6e-6), rel=1e-12)   # geometric midpoint


@pytest.mark.parametrize("k", [1, 2, 3])
def test_views_cycle_through_every_training_view(k):
    tr = SimpleNamespace(cfg=TrainConfig(views_per_step=k), V=5)
    seen = [v for t in range(1, 6) for v in GaussianTrainer.views_of(tr, t)]
    assert seen == [i % 5 for i in range(5 * k)]


def test_unknown_strategy_is_rejected():
    with pytest.raises(ValueError):
        GaussianTrainer({}, {}, None, TrainConfig(strategy="other"))
