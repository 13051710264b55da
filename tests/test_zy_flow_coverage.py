"""Coverage of the learned proposal's error bars over seeds (a statistical
test of the whole pipeline).  It sits in a file of its own, collected after
the deterministic GPU parity tests, so that a rare miss, which a correct
error bar also produces now and then, does not stop those from running."""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2302_05730_amd as m
    m.lib()
    return m


def _say(*a):
    print(*a, flush=True, file=sys.stderr)


def test_flow_pipeline_error_bars_cover_the_integral(mc):
    """Coverage over seeds, the error model of m-Cubes (the error is the
    standard deviation of the estimate): sixteen pipelines with the default
    recipe on the mixture at 2^22 samples per iteration, run to a relative
    error of 1e-3 (at least four flow iterations).  The same seed trains a
    different flow on every run (the FP64 histogram atomics of the warm-up
    add in hardware order), so the sixteen pulls are independent draws and
    the criterion is a statistical one, set by the binomial distribution:
      * asked: at least 12 of 16 within 2 sigma, at most one beyond 3 sigma,
        and every run the pipeline calls converged within 2e-3 of the
        integral;
      * an exactly Gaussian error (95.4% within 2 sigma, 99.73% within 3)
        fails this with probability 0.14%; the measured coverage of the
        default recipe at this size (about 90% and 99%: the weights' heavy
        tail leaves the median run slightly low) fails it with about 3%;
        error bars 2 times too small fail it with 86%, 1.5 times too small
        with 29%.
    (Eight seeds with 7 of 8 within 2 sigma and all within 3 fail an exactly
    Gaussian error 6.9% of the time, and this recipe 25%.)  Runs the
    pipeline refuses to call converged (heavy weight tail with disagreeing
    iterations) still count in the pulls: their error bars must cover too.
    The absolute bound holds for the converged ones only: a run that ends
    unconverged after every iteration has reported that its estimate is
    not settled, with an error bar to match (one such run measured 2.2e-3
    off with a claimed 2.5e-3)."""
    pr = workloads.mixture_6d(ncall=1 << 22)
    pulls, devs = [], []  # devs: converged runs only
    for seed in range(101, 117):
        fl = mc.Flow(workloads.flow_init(7))
        res, rep = fl.integrate(pr.family, pr.params, pr.ncall, 50, 1e-3, seed,
                                mc.mcubes_default_options(nbins=500))
        dev = res["estimate"] - 1.0
        pull = dev / res["error"]
        _say(f"seed {seed}: {res['estimate']:.6f} +- {res['error']:.2e} (pull {pull:+.2f}), "
             f"{res['iterations']} flow iterations, chi2/dof {res['chi2_dof']:.2f}, "
             f"tail {rep['tail_shape']:.3f}, converged {res['converged']}, "
             f"used {rep['used_flow']}")
        assert rep["used_flow"] == 1 and res["iterations"] >= 4
        pulls.append(pull)
        if res["converged"]:
            devs.append(abs(dev))
    pulls = np.abs(np.array(pulls))
    assert np.sum(pulls <= 2.0) >= 12, pulls
    assert np.sum(pulls > 3.0) <= 1, pulls
    assert not devs or max(devs) <= 2e-3, devs
