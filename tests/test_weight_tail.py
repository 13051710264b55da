"""The weight-tail diagnostic (mcubes_weight_tail_shape, host only): the
Hill estimate of the generalised Pareto shape of the upper tail of a log2
weight histogram.  Pinned against samples whose tail shape is known in
closed form: Pareto(alpha) weights have shape 1/alpha; exponential and
half-normal weights have shape 0 (light tails, where the Hill estimate over
the top 3 sqrt N of N samples is small and positive); equal weights give
half a bin.  The library is loaded, no GPU is used."""
import math

import numpy as np
import pytest

import paper_2302_05730_amd as mc

BINS = 4096


def _hist(w):
    w = np.asarray(w, dtype=np.float64)
    w = w[w > 0]
    b = np.floor(np.log2(w) * 8.0)
    b = np.clip(b, -2048, 2047).astype(np.int64) + 2048
    return np.bincount(b, minlength=BINS).astype(np.uint32)


@pytest.mark.parametrize("alpha", [1.2, 1.6, 2.5, 4.0])
def test_pareto_tails_give_one_over_alpha(alpha):
    rng = np.random.default_rng(int(alpha * 10))
    n = 1 << 21
    w = (1.0 - rng.random(n)) ** (-1.0 / alpha)  # Pareto with x_min 1
    shape, k = mc.mcubes_weight_tail_shape(_hist(w))
    assert k >= 3 * math.sqrt(n) - 1
    # Hill over ~4300 order statistics: sd ~ xi / sqrt(k) ~ 0.015; binning <= 0.04
    assert shape == pytest.approx(1.0 / alpha, abs=0.06)


def test_scale_does_not_matter():
    rng = np.random.default_rng(3)
    w = (1.0 - rng.random(1 << 20)) ** (-1.0 / 1.5)
    a, _ = mc.mcubes_weight_tail_shape(_hist(w))
    b, _ = mc.mcubes_weight_tail_shape(_hist(w * 2.0 ** 20))
    assert a == pytest.approx(b, abs=1e-12)  # a power-of-two scale shifts whole bins


@pytest.mark.parametrize("kind", ["exponential", "halfnormal"])
def test_light_tails_stay_well_below_one_half(kind):
    rng = np.random.default_rng(5)
    n = 1 << 21
    w = rng.exponential(size=n) if kind == "exponential" else np.abs(rng.normal(size=n))
    shape, _ = mc.mcubes_weight_tail_shape(_hist(w))
    assert 0.0 < shape < 0.2


def test_equal_weights_and_too_few():
    h = np.zeros(BINS, dtype=np.uint32)
    h[2048] = 1000
    shape, k = mc.mcubes_weight_tail_shape(h)
    assert shape == pytest.approx(0.5 * math.log(2.0) / 8.0)
    assert k == 1000
    h[2048] = 99
    shape, k = mc.mcubes_weight_tail_shape(h)
    assert math.isnan(shape) and k == 0
    with pytest.raises(ValueError):
        mc.mcubes_weight_tail_shape(np.zeros(10))
