"""Helpers of the GPU parity tests: run one V-Sample iteration of the HIP
library through the C interface, run the same iteration in the oracle, and
compare them to the stated tolerances.

Tolerances (FP64):
  * bins and, for integrands without cancellation, I_t: 1e-12 relative.  Each
    sample's weight is bit-identical for integrands without libm calls and
    within a few ulp for exp/cos (both libraries are faithfully rounded), and
    every bin is a sum of positive terms, so only the summation order differs.
  * I_t of the oscillatory family (positive and negative terms): 1e-12 of the
    RMS sample weight sqrt(sum w^2 / N), the scale of the sum's rounding.
  * var_t: sum over cubes of (w1 - w0)^2 / 2 (p = 2).  A relative perturbation
    delta of every w moves var_t by at most 2 delta sqrt(Q / (2 sum var_c))
    relative (Cauchy-Schwarz), Q = sum w^2, so the tolerance is
    max(1e-12, 16 eps sqrt(Q / (2 var_t p m^2))) with eps = 2^-53; for
    integrands without libm calls delta is 0 and the tolerance is 1e-12.
  * refined grid edges: 1e-12 relative + 1e-15 absolute.
"""
import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle

EPS = 2.0**-53
LIBM_FAMILIES = {0, 3, 4, 5, 7}  # cos or exp inside the integrand


def host_threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def oracle_iteration_parallel(family, params, dim, nb, ncall, seed, it, grid, threads=None,
                              stream=0):
    """The oracle's iteration, split over contiguous cube ranges run in threads
    (the C oracle releases the GIL); partial sums are combined with fsum.
    `stream` is the Philox stream word (the integrand's index in a batch)."""
    g, m, p, n = oracle.plan(dim, ncall)
    threads = threads or host_threads()
    chunks = min(threads * 4, max(1, m))
    cut = [m * k // chunks for k in range(chunks + 1)]
    with ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(lambda ab: oracle.sample_range(family, params, dim, nb, g, m, p, seed,
                                                           it, grid, ab[0], ab[1], stream),
                            zip(cut[:-1], cut[1:])))
    s = math.fsum(x[0] for x in parts)
    v = math.fsum(x[1] for x in parts)
    bins = np.zeros((dim, nb))
    for x in parts:
        bins += x[2]
    I, var = oracle.estimates(m, p, s, v)
    return I, var, bins


def gpu_iteration(plan, it, grid_np, with_bins=True):
    """One V-Sample + reduce on the GPU for a given grid -> (I_t, var_t, bins)
    (bins None when V-Sample runs without bin sums)."""
    import torch
    import paper_2302_05730_amd as mc
    info = plan.info
    dim, nb = info["dim"], info["nbins"]
    d_grid = torch.from_numpy(np.ascontiguousarray(grid_np, dtype=np.float64).ravel()).cuda()
    d_bins = torch.empty(info["bins_len"], dtype=torch.float64, device="cuda")
    d_part = torch.empty(info["partials_len"], dtype=torch.float64, device="cuda")
    d_est = torch.empty(2, dtype=torch.float64, device="cuda")
    mc.mcubes_fill(d_bins, 0.0)
    mc.mcubes_vsample(plan, it, d_grid, d_bins if with_bins else None, d_part)
    mc.mcubes_reduce(plan, d_part, d_est)
    torch.cuda.synchronize()
    est = d_est.cpu().numpy()
    bins = d_bins.cpu().numpy().reshape(dim, nb) if with_bins else None
    return float(est[0]), float(est[1]), bins


def gpu_refine(plan, grid_np, bins_np):
    import torch
    import paper_2302_05730_amd as mc
    info = plan.info
    d_grid = torch.from_numpy(np.ascontiguousarray(grid_np, dtype=np.float64).ravel()).cuda()
    d_bins = torch.from_numpy(np.ascontiguousarray(bins_np, dtype=np.float64).ravel()).cuda()
    d_out = torch.empty_like(d_grid)
    mc.mcubes_refine(plan, d_grid, d_bins, d_out)
    torch.cuda.synchronize()
    return d_out.cpu().numpy().reshape(info["dim"], info["nbins"] + 1)


def var_tolerance(family, var, bins, m, p):
    if family not in LIBM_FAMILIES or var <= 0:
        return 1e-12
    Q = float(bins[0].sum())
    return max(1e-12, 16 * EPS * math.sqrt(Q / (2 * var * p * m * m)))


def assert_iteration_close(family, got, ref, m, p, what=""):
    gI, gV, gB = got
    rI, rV, rB = ref
    n = m * p
    assert np.all(np.isfinite(gB)) and math.isfinite(gI) and math.isfinite(gV), what
    # bins: positive sums, elementwise 1e-12 relative (zero bins exactly zero)
    diff = np.abs(gB - rB)
    assert np.all(diff <= 1e-12 * np.abs(rB) + 1e-300), \
        f"{what}: bins max rel diff {np.max(diff / np.maximum(np.abs(rB), 1e-300)):.3e}"
    if family == 0:
        scale = max(abs(rI), math.sqrt(float(rB[0].sum()) / n))
    else:
        scale = abs(rI)
    assert abs(gI - rI) <= 1e-12 * scale + 1e-300, f"{what}: I {gI!r} vs {rI!r}"
    tol = var_tolerance(family, rV, rB, m, p)
    assert abs(gV - rV) <= tol * abs(rV) + 1e-300, f"{what}: var {gV!r} vs {rV!r} (tol {tol:.2e})"


def random_grid(rng, dim, nb, shape=1.5):
    g = np.zeros((dim, nb + 1))
    for j in range(dim):
        w = rng.gamma(shape, size=nb)
        g[j, 1:] = np.cumsum(w) / w.sum()
        g[j, -1] = 1.0
    return g
