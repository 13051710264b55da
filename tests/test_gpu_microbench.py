"""The integrand microbenchmark kernel evaluates the same families as
V-Sample; on points from a table its per-thread sums must match the
oracle's integrand summed in the same order."""
import numpy as np
import pytest

import oracle
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


@pytest.mark.parametrize("k", range(1, 8))
@pytest.mark.parametrize("dim", [1, 5, 8, 10])
def test_integrand_kernel_matches_oracle(mc, k, dim):
    import torch
    fam, params = workloads.paper_integrand(k, dim)
    rng = np.random.default_rng(k * 100 + dim)
    npts, calls, blocks, block = 37, 50, 2, 64
    pts = rng.uniform(0, 1, (npts, dim))
    d_pts = torch.from_numpy(pts).cuda()
    out = torch.empty(blocks * block, dtype=torch.float64, device="cuda")
    mc.mcubes_microbench(mc.MCUBES_MB_INTEGRAND, out, blocks, block, calls, fam, params, dim,
                         d_pts, npts)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    fvals = np.array([oracle.integrand(fam, params, p) for p in pts])
    for tid in range(blocks * block):
        q = (tid * 7919) % npts
        s = 0.0
        for _ in range(calls):
            s += fvals[q]
            q = 0 if q + 1 == npts else q + 1
        if fam in (1, 2, 6):  # no libm call: bit-identical
            assert got[tid] == s, (tid, got[tid], s)
        else:
            assert abs(got[tid] - s) <= 1e-13 * max(abs(s), np.abs(fvals).sum()), (tid, got[tid], s)


def test_microbench_kinds_run(mc):
    import torch
    out = torch.empty(128, dtype=torch.float64, device="cuda")
    for kind in range(1, 8):
        mc.mcubes_microbench(kind, out, 2, 64, 16, dim=8)
        torch.cuda.synchronize()
        assert torch.isfinite(out).all()
    with pytest.raises(mc.MCubesError):
        mc.mcubes_microbench(9, out, 2, 64, 16)
