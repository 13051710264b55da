"""GPU parity of the learned proposal (the flow kernels, FP32) against the FP64
flow oracle, the export of an iteration's samples, and what training buys.

Tolerances.  The GPU evaluates the flow in FP32 (2^-24 relative per
operation) and the oracle in FP64.  The network sums 96 + 64 + 64 products
per output and the spline turns an error d in a raw output into at most a
few d in the CDF and the log-density, so per coordinate and layer the
transformed value moves by ~1e-6 and the log-density by ~1e-5; over four
layers and six coordinates: |dz| <= 2e-5, |d log q| <= 2e-4 per sample,
and the mean of |d log q| an order below that.  The weights of the
flow-mapped iteration inherit |dw/w| <= |d log q| + |grad log f| |dx|.
Gradients: each component against the oracle to 1e-3 of the largest
component (FP32 accumulation over the batch and the layers).

The BF16 matrix-core path is compared with the oracle evaluating the network
the same way (weights and product inputs rounded to bfloat16, biases FP32):
a product input within the FP32-versus-FP64 difference of a rounding
boundary may round the other way on the two sides (one bfloat16 ulp, 2^-8
relative, moving the spline outputs by ~1e-3), so 99% of the samples must
agree to |d log q| <= 2e-3, |dx| <= 2e-4 and all of them to ten times that.
The BF16 training gradient is compared component by component with the
oracle's BF16 gradient (same rounded operands)."""
import math
import sys

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


def _say(*a):
    print(*a, flush=True, file=sys.stderr)


def _f32(theta):
    """parameters as the GPU holds them (FP32), widened back"""
    return np.asarray(theta, dtype=np.float32).astype(np.float64)


def _cube_multiplier(m, g):
    """V-Sample's visiting order: the multiplier nearest below 0.618 m that is
    coprime to g (the definition the library documents for work items)."""
    mult = max(1, int(math.floor(m * 0.6180339887498949)))
    while math.gcd(mult, g) != 1:
        mult += 1
    return mult % m if m > 1 else 0


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("seed,out_scale", [(1, 0.3), (2, 0.8)])
def test_density_and_sample_match_oracle(mc, seed, out_scale):
    import torch
    theta = _f32(workloads.flow_random(seed, out_scale=out_scale))
    fl = mc.Flow(theta)
    rng = np.random.default_rng(seed)
    n = 2048
    pts = rng.uniform(0.0, 1.0, (n, 6))
    d_in = _dev(pts)
    d_out = torch.empty(n * 6, dtype=torch.float64, device="cuda")
    d_lq = torch.empty(n, dtype=torch.float64, device="cuda")
    for direction in ("density", "sample"):
        getattr(fl, direction)(d_in, n, d_out, d_lq)
        torch.cuda.synchronize()
        out = d_out.cpu().numpy().reshape(n, 6)
        lq = d_lq.cpu().numpy()
        fn = oracle.flow_density if direction == "density" else oracle.flow_sample
        ref = [fn(theta, p) for p in pts]
        dz = np.abs(out - np.array([r[0] for r in ref]))
        dl = np.abs(lq - np.array([r[1] for r in ref]))
        _say(f"{direction}: max |dz| {dz.max():.2e}, max |dlogq| {dl.max():.2e}, "
             f"mean {dl.mean():.2e}")
        assert dz.max() <= 2e-5, direction
        assert dl.max() <= 2e-4 and dl.mean() <= 2e-5, direction


def test_identity_flow_is_exact(mc):
    import torch
    fl = mc.Flow(workloads.flow_init(5))
    rng = np.random.default_rng(3)
    n = 1000
    pts = np.asarray(rng.uniform(0, 1, (n, 6)), dtype=np.float32).astype(np.float64)
    d_out = torch.empty(n * 6, dtype=torch.float64, device="cuda")
    d_lq = torch.empty(n, dtype=torch.float64, device="cuda")
    fl.sample(_dev(pts), n, d_out, d_lq)
    torch.cuda.synchronize()
    assert np.abs(d_out.cpu().numpy().reshape(n, 6) - pts).max() <= 2e-7
    assert np.abs(d_lq.cpu().numpy()).max() <= 1e-6


@pytest.mark.parametrize("seed,out_scale", [(3, 0.3), (8, 0.8)])
def test_bf16_sampling_matches_oracle(mc, seed, out_scale):
    import torch
    theta = _f32(workloads.flow_random(seed, out_scale=out_scale))
    fl = mc.Flow(theta)
    rng = np.random.default_rng(seed)
    n = 4000  # 62.5 waves: a partial last wave
    z = np.asarray(rng.uniform(0.0, 1.0, (n, 6)), dtype=np.float32).astype(np.float64)
    d_x = torch.empty(n * 6, dtype=torch.float64, device="cuda")
    d_lq = torch.empty(n, dtype=torch.float64, device="cuda")
    fl.sample(_dev(z), n, d_x, d_lq, precision=mc.MCUBES_BF16)
    torch.cuda.synchronize()
    x = d_x.cpu().numpy().reshape(n, 6)
    lq = d_lq.cpu().numpy()
    ref = [oracle.flow_sample(theta, zz, bf16=True) for zz in z]
    dx = np.abs(x - np.array([r[0] for r in ref])).max(axis=1)
    dl = np.abs(lq - np.array([r[1] for r in ref]))
    tight = (dx <= 2e-4) & (dl <= 2e-3)
    _say(f"bf16 sample: max |dx| {dx.max():.2e}, max |dlogq| {dl.max():.2e}, "
         f"tight fraction {tight.mean():.4f}")
    assert tight.mean() >= 0.99
    assert dx.max() <= 2e-3 and dl.max() <= 2e-2
    # and it is a different computation from the FP32 path (the rounding shows)
    d_x32 = torch.empty_like(d_x)
    d_lq32 = torch.empty_like(d_lq)
    fl.sample(_dev(z), n, d_x32, d_lq32, precision=mc.MCUBES_FP32)
    torch.cuda.synchronize()
    assert np.abs(d_lq32.cpu().numpy() - lq).max() > 1e-6


def test_loss_gradient_and_adam_match_oracle(mc):
    import torch
    theta = _f32(workloads.flow_random(4, out_scale=0.4))
    fl = mc.Flow(theta)
    rng = np.random.default_rng(11)
    n = 700  # several workgroups and a ragged tail
    xs = rng.uniform(0.02, 0.98, (n, 6))
    ws = rng.uniform(0.1, 3.0, n)
    d_grad = torch.zeros(mc.MCUBES_FLOW_PARAMS, dtype=torch.float64, device="cuda")
    d_loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    fl.loss_grad(_dev(xs), _dev(ws), n, d_grad, d_loss)
    torch.cuda.synchronize()
    g = d_grad.cpu().numpy()
    loss_ref, g_ref = oracle.flow_loss_grad(theta, xs, ws)
    assert float(d_loss.cpu()[0]) == pytest.approx(loss_ref, rel=1e-5, abs=1e-6)
    scale = np.abs(g_ref).max()
    err = np.abs(g - g_ref)
    _say(f"gradient: max err {err.max():.2e} of scale {scale:.2e}")
    assert err.max() <= 1e-3 * scale
    # cosine similarity close to one, no component with the wrong sign among the large ones
    assert g @ g_ref / (np.linalg.norm(g) * np.linalg.norm(g_ref)) > 1 - 1e-6
    big = np.abs(g_ref) > 1e-2 * scale
    assert np.all(np.sign(g[big]) == np.sign(g_ref[big]))
    # one Adam step from the kept gradient
    fl.adam_step(1e-3)
    torch.cuda.synchronize()
    t_gpu = np.array(fl.params())
    t_ref, _, _ = oracle.flow_adam(theta, np.zeros_like(theta), np.zeros_like(theta),
                                   _f32(g), 1, lr=1e-3)
    assert np.abs(t_gpu - t_ref).max() <= 1e-6


@pytest.mark.parametrize("n", [4000, 3999])
def test_bf16_loss_gradient_matches_the_bf16_oracle(mc, n):
    """The matrix-core form of the training pass against the oracle's BF16
    mode, which rounds the same operands to bfloat16 (weights, the one-blob
    encoding, h1 and h2, the spline-parameter deltas and the deltas after
    each ReLU) and sums their products exactly.  What is left between the
    two is FP32 arithmetic on the GPU (splines, accumulation, the one-blob
    recurrence; relative ~1e-6 per term) and what it decides:
      * rounding flips: a value within that distance of a bfloat16 rounding
        boundary lands on the other side and moves by one bfloat16 ulp
        (2^-8 relative), with probability ~2^8 times the distance: a
        component's error stays within 1e-3 of the sum of its terms'
        magnitudes A_i (grad_abs); asked of 99.5% of the components
        (measured: 99.8% and 99.9%);
      * decision flips: a ReLU pre-activation or a spline-bin position within
        the FP32 accumulation error (~1e-5 of its terms) of the boundary
        takes the other branch, which switches one sample's term of every
        component it feeds on or off.  That term is a share of A_i: the
        largest seen is 4% (a W1 entry of a bump far from most samples,
        where a few samples carry A_i); every component must stay within
        0.1 A_i.
    Mistakes that move a whole parameter block do not hide in either
    allowance: each of the 24 blocks must agree in relative L2 to 1e-2 (a
    block off by 2x reads 1.0; measured at most 3.5e-3), and the BF16
    oracle must be at least ten times closer than the FP64 gradient.
    n = 4000: many waves and a ragged last one, rows read 16 bytes at a
    time; n = 3999: rows not 16-byte aligned (read element by element) and
    a ragged last 16-sample step."""
    import torch
    theta = _f32(workloads.flow_random(4, out_scale=0.4))
    fl = mc.Flow(theta)
    rng = np.random.default_rng(12)
    xs = rng.uniform(0.02, 0.98, (n, 6))
    ws = rng.uniform(0.1, 3.0, n)
    d_grad = torch.zeros(mc.MCUBES_FLOW_PARAMS, dtype=torch.float64, device="cuda")
    d_loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    fl.loss_grad(_dev(xs), _dev(ws), n, d_grad, d_loss, precision=mc.MCUBES_BF16)
    torch.cuda.synchronize()
    g = d_grad.cpu().numpy()
    loss = float(d_loss.cpu()[0])
    loss16, g16, A = oracle.flow_loss_grad(theta, xs, ws, bf16=True, with_abs=True)
    loss64, g64 = oracle.flow_loss_grad(theta, xs, ws)
    err = np.abs(g - g16)
    gmax = np.abs(g16).max()
    ratio = err / (A + 1e-300)
    rel16 = np.linalg.norm(g - g16) / np.linalg.norm(g16)
    rel64 = np.linalg.norm(g - g64) / np.linalg.norm(g64)
    _say(f"bf16 loss {loss} vs bf16 oracle {loss16} (fp64 {loss64}); err/A median "
         f"{np.median(ratio):.2e} p99 {np.percentile(ratio, 99):.2e} max {ratio.max():.2e}; "
         f"rel L2 vs bf16 oracle {rel16:.2e}, vs fp64 oracle {rel64:.2e}")
    assert loss == pytest.approx(loss16, rel=1e-5)
    rounding = err <= 1e-3 * A + 1e-6 * gmax
    assert np.mean(rounding) >= 0.995, np.mean(rounding)
    assert np.all(err <= 0.1 * A + 1e-6 * gmax), np.argmax(err / (A + 1e-300))
    lp = oracle.FLOW_LAYER_PARAMS
    i, h, o = oracle.FLOW_IN, oracle.FLOW_HID, oracle.FLOW_OUT
    bounds = np.cumsum([0, i * h, h, h * h, h, h * o, o])
    for l in range(4):
        for a, b in zip(bounds[:-1], bounds[1:]):
            blk = slice(l * lp + a, l * lp + b)
            rel = np.linalg.norm(g[blk] - g16[blk]) / np.linalg.norm(g16[blk])
            assert rel < 1e-2, (l, a, rel)
    assert rel16 < 0.1 * rel64


def test_flow_iteration_weight_tail(mc):
    """The weight histogram of a flow-mapped iteration feeds the tail
    diagnostic, in FP32 and BF16.  The identity flow (uniform proposal) on
    the additive integrand (weights sum x in (0, 6), flat at the top) reads
    as a light tail; on a peaked 6-D Gaussian (a = 5) the few samples near
    the peak carry weights spread over a factor of ~15 above the tail's
    threshold, which reads as heavy (the estimate for uniform sampling of
    exp(-25 |x - u|^2) over the top 0.6% is 0.67), as it should: there a
    handful of weights decides the estimate.  The tail count is
    min(N/5, 3 sqrt N) or a little more (whole bins)."""
    import torch
    opts = mc.mcubes_default_options(nbins=50)
    fl = mc.Flow(workloads.flow_init(7))
    d_est = torch.zeros(2, dtype=torch.float64, device="cuda")
    gauss = [5.0] * 6 + [0.4, 0.5, 0.6, 0.45, 0.55, 0.5]
    for family, params, lo, hi in ((workloads.ADDITION, None, 0.0, 0.2),
                                   (workloads.GAUSSIAN, gauss, 0.5, 0.9)):
        plan = mc.mcubes_plan_create(family, params, 6, 1 << 18, 3, opts)
        n = plan.info["samples_per_iter"]
        for prec in (mc.MCUBES_FP32, mc.MCUBES_BF16):
            fl.vsample(plan, 2, d_est, precision=prec)
            shape, k = fl.weight_tail()
            _say(f"family {family} precision {prec}: tail shape {shape:.3f} over {k} of {n}")
            assert k >= min(n // 5, int(3 * math.sqrt(n)))
            assert lo < shape < hi


def test_bf16_draw_follows_the_fp32_draw(mc):
    """Training samples drawn on the matrix cores use the same counters as
    the FP32 draw: the same z, mapped with BF16 products, so the points agree
    to the BF16 sampling tolerance (99% within 2e-3, all within 2e-2) and
    the weights f/q of a smooth integrand to a few 1e-3 (99% within 1e-2
    relative); the ragged tail of a wave is drawn as well."""
    import torch
    theta = _f32(workloads.flow_random(5, out_scale=0.3))
    fl = mc.Flow(theta)
    params = [2.0] * 6 + [0.4, 0.5, 0.6, 0.45, 0.55, 0.5]
    plan = mc.mcubes_plan_create(workloads.GAUSSIAN, params, 6, 1 << 16, 9,
                                 mc.mcubes_default_options(nbins=50))
    n = 5000
    out = {}
    for prec in (mc.MCUBES_FP32, mc.MCUBES_BF16):
        d_x = torch.zeros(n * 6, dtype=torch.float64, device="cuda")
        d_w = torch.zeros(n, dtype=torch.float64, device="cuda")
        fl.draw(plan, 77, n, d_x, d_w, precision=prec)
        torch.cuda.synchronize()
        out[prec] = (d_x.cpu().numpy().reshape(n, 6), d_w.cpu().numpy())
    (x32, w32), (x16, w16) = out[mc.MCUBES_FP32], out[mc.MCUBES_BF16]
    dx = np.abs(x16 - x32).max(axis=1)
    dw = np.abs(w16 / w32 - 1.0)
    _say(f"bf16 draw: |dx| 99% {np.quantile(dx, 0.99):.1e} max {dx.max():.1e}; "
         f"|dw/w| 99% {np.quantile(dw, 0.99):.1e}")
    assert np.all(w32 > 0) and np.all(w16 > 0)
    assert np.quantile(dx, 0.99) <= 2e-3 and dx.max() <= 2e-2
    assert np.quantile(dw, 0.99) <= 1e-2


def test_sample_export_is_the_iterations_own_samples(mc):
    """The exported samples of an iteration: every weight and point of a few
    cubes against the oracle's own map (bitwise), and the sum of all weights
    against the iteration's estimate from V-Sample."""
    import torch
    from parity_util import random_grid
    pr = workloads.mixture_6d(ncall=40000)
    nb = 50
    plan = mc.mcubes_plan_create(pr.family, pr.params, 6, pr.ncall, 21,
                                 mc.mcubes_default_options(nbins=nb))
    info = plan.info
    g, m, p = info["cube_side"], info["ncubes"], info["samples_per_cube"]
    grid = random_grid(np.random.default_rng(1), 6, nb)
    d_grid = _dev(grid.ravel())
    rows = m * p
    d_x = torch.empty(rows * 6, dtype=torch.float64, device="cuda")
    d_w = torch.empty(rows, dtype=torch.float64, device="cuda")
    mc.mcubes_vsample_dump(plan, 3, d_grid, 0, m, d_x, d_w)
    torch.cuda.synchronize()
    xs = d_x.cpu().numpy().reshape(rows, 6)
    ws = d_w.cpu().numpy()
    from parity_util import gpu_iteration
    I, V, _ = gpu_iteration(plan, 3, grid)
    assert math.fsum(ws) / rows == pytest.approx(I, rel=1e-12)
    key = [21 & 0xffffffff, 21 >> 32]
    # work item w holds cube (w mult) mod m; the rows cover every cube once
    mult = _cube_multiplier(m, g)
    cubes = [(w * mult) % m for w in range(m)]
    assert sorted(cubes) == list(range(m))
    for w in (0, 1, m // 3, m - 1):
        c = cubes[w]
        digits = [(c // g**j) % g for j in range(6)]
        for k in range(p):
            z = []
            for b in range(2):
                r = oracle.philox4x32_10([c, 0, k * 2 + b, 3], key)
                z += [(digits[4 * b + q] + oracle.uniform(r[q])) * (nb / g)
                      for q in range(4) if 4 * b + q < 6]
            x, J, _ = oracle.map_point(grid, np.array(z))
            row = w * p + k
            assert np.array_equal(xs[row], x), (c, k)
            assert ws[row] == pytest.approx(oracle.integrand(pr.family, pr.params, x) * J,
                                            rel=1e-14)


def test_flow_iteration_matches_oracle(mc):
    import torch
    theta = _f32(workloads.flow_random(6, out_scale=0.5))
    fl = mc.Flow(theta)
    params = [4.0] * 6 + [0.45, 0.5, 0.55, 0.5, 0.4, 0.6]
    plan = mc.mcubes_plan_create(workloads.GAUSSIAN, params, 6, 20000, 77,
                                 mc.mcubes_default_options(nbins=10, stream_id=3))
    info = plan.info
    g, m, p = info["cube_side"], info["ncubes"], info["samples_per_cube"]
    d_est = torch.empty(2, dtype=torch.float64, device="cuda")
    for it in (0, 5):
        fl.vsample(plan, it, d_est)
        torch.cuda.synchronize()
        I, V = d_est.cpu().tolist()
        s, v = oracle.flow_proposal_range(theta, workloads.GAUSSIAN, params, g, m, p, 77,
                                          0x80000003, it, 0, m)
        rI, rV = oracle.estimates(m, p, s, v)
        _say(f"flow iteration {it}: {I!r} vs {rI!r}; var {V!r} vs {rV!r}")
        assert I == pytest.approx(rI, rel=2e-4)
        assert V == pytest.approx(rV, rel=2e-3)
        # the matrix-core form against the oracle with bfloat16 rounding
        fl.vsample(plan, it, d_est, precision=mc.MCUBES_BF16)
        torch.cuda.synchronize()
        I16, V16 = d_est.cpu().tolist()
        s, v = oracle.flow_proposal_range(theta, workloads.GAUSSIAN, params, g, m, p, 77,
                                          0x80000003, it, 0, m, bf16=True)
        bI, bV = oracle.estimates(m, p, s, v)
        _say(f"bf16 flow iteration {it}: {I16!r} vs {bI!r}; var {V16!r} vs {bV!r}")
        assert I16 == pytest.approx(bI, rel=2e-3)
        assert V16 == pytest.approx(bV, rel=2e-2)


def test_training_reduces_the_loss(mc):
    """Training on an iteration's exported samples lowers the weighted
    negative log-likelihood; refining on the flow's own samples (weights f/q)
    narrows the spread of log w (the robust measure: a few extreme weights
    decide the effective sample size (sum w)^2 / (n sum w^2), which must
    still rise; a single weight of 1e4 among 2^21 samples caps it at 2%)."""
    import torch
    pr = workloads.mixture_6d(ncall=1 << 22)
    plan = mc.mcubes_plan_create(pr.family, pr.params, 6, pr.ncall, 5,
                                 mc.mcubes_default_options(nbins=500))
    bufs = mc.Buffers(plan)
    mc.mcubes_init_grid(plan, bufs.grid[0])
    for t in range(8):
        mc.mcubes_iteration(plan, t, bufs.grid[t & 1], bufs.grid[(t + 1) & 1], bufs.bins,
                            bufs.partials, bufs.est, bufs.state, 0.0)
    p = plan.info["samples_per_cube"]
    rows = 1 << 20
    n = 1 << 21
    d_x = torch.empty(n * 6, dtype=torch.float64, device="cuda")
    d_w = torch.empty(n, dtype=torch.float64, device="cuda")
    mc.mcubes_vsample_dump(plan, 7, bufs.grid[1], 0, rows // p, d_x, d_w)
    fl = mc.Flow(workloads.flow_init(7))
    losses = fl.train(d_x, d_w, rows, 10, 32768, 2e-3)
    _say(f"losses {losses}")
    assert losses[-1] < losses[0] - 2.0

    def stats(k):
        fl.draw(plan, 300 + k, n, d_x, d_w)
        w = d_w.cpu().numpy()
        return float(w.sum() ** 2 / (w ** 2).sum() / n), float(np.log(w[w > 0]).std())
    ess0, sd0 = stats(0)
    for r in range(4):
        fl.draw(plan, 400 + r, n, d_x, d_w)
        fl.train(d_x, d_w, n, 2, 32768, 1e-3)
    ess1, sd1 = stats(1)
    _say(f"effective sample fraction {ess0:.4f} -> {ess1:.4f}; sd of log w {sd0:.3f} -> {sd1:.3f}")
    assert sd1 < sd0 / 1.5 and ess1 > ess0


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
def test_training_call_equals_its_steps(mc, precision):
    """mcubes_flow_train ends each BF16 step with one launch that sums the
    slices, takes the Adam step and writes the new parameters straight into
    the packed fragments (no repack before the next step).  It must leave
    exactly the parameters of the same minibatches taken one call at a time,
    mcubes_flow_loss_grad (which repacks) then mcubes_flow_adam_step, bit for
    bit, over two epochs with a ragged last minibatch."""
    import torch
    prec = mc.MCUBES_BF16 if precision == "bf16" else mc.MCUBES_FP32
    n, batch, epochs, lr = 3 * 8192 + 1000, 8192, 2, 1e-3
    rng = np.random.default_rng(11)
    x = _dev(rng.uniform(0.02, 0.98, (n, 6)))
    w = _dev(rng.uniform(0.1, 3.0, n))
    theta0 = workloads.flow_random(5, out_scale=0.4)
    whole = mc.Flow(theta0)
    whole.train(x.view(-1), w, n, epochs, batch, lr, precision=prec)
    steps = mc.Flow(theta0)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(epochs):
        for b0 in range(0, n, batch):
            nb = min(batch, n - b0)
            steps.loss_grad(x.view(-1)[6 * b0:6 * (b0 + nb)], w[b0:b0 + nb], nb, None, loss,
                            precision=prec)
            steps.adam_step(lr)
    torch.cuda.synchronize()
    a = np.asarray(whole.params(), dtype=np.float64)
    b = np.asarray(steps.params(), dtype=np.float64)
    assert np.any(a != np.asarray(theta0, dtype=np.float32))
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    # other calls in between (BF16 sampling packs the forward fragments
    # itself), then one more epoch each way
    z = _dev(rng.uniform(0.0, 1.0, (4096, 6)))
    xs = torch.empty(4096 * 6, dtype=torch.float64, device="cuda")
    lq = torch.empty(4096, dtype=torch.float64, device="cuda")
    for fl in (whole, steps):
        fl.sample(z.view(-1), 4096, xs, lq, precision=mc.MCUBES_BF16)
    whole.train(x.view(-1), w, n, 1, batch, lr, precision=prec)
    for b0 in range(0, n, batch):
        nb = min(batch, n - b0)
        steps.loss_grad(x.view(-1)[6 * b0:6 * (b0 + nb)], w[b0:b0 + nb], nb, None, loss,
                        precision=prec)
        steps.adam_step(lr)
    torch.cuda.synchronize()
    a = np.asarray(whole.params(), dtype=np.float64)
    b = np.asarray(steps.params(), dtype=np.float64)
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_flow_combine_matches_oracle(mc):
    """The equal-weight combination of flow-mapped iterations, fed one
    iteration at a time through the C-ABI, against the oracle on every
    prefix: the same FP64 sums in the same order, so 1e-14 relative (one
    zero-variance iteration, which adds nothing to chi2).  The error is the
    larger of the within-iteration and the scatter estimate; the scatter
    wins on some prefixes and loses on others here.  Converged only from
    the third iteration on (min_iters = 3)."""
    import torch
    rng = np.random.default_rng(21)
    T = 12
    I = 1.0 + 0.01 * rng.standard_normal(T)
    V = (1e-4 * rng.lognormal(0.0, 1.0, T)) ** 2
    V[4] = 0.0
    d_est = torch.empty(2, dtype=torch.float64, device="cuda")
    d_state = torch.zeros(mc.MCUBES_STATE_LEN, dtype=torch.float64, device="cuda")
    for t in range(T):
        d_est.copy_(torch.tensor([I[t], V[t]], dtype=torch.float64))
        mc.mcubes_flow_combine(t, d_est, d_state, 2e-5, min_iters=3)
        st = d_state.cpu().numpy()
        Ibar, sigma, chi2, dof = oracle.flow_combine(I[:t + 1], V[:t + 1])
        assert st[0] == pytest.approx(Ibar, rel=1e-14)
        assert st[1] == pytest.approx(sigma, rel=1e-14)
        assert st[2] == pytest.approx(chi2, rel=1e-13, abs=1e-300)
        assert (st[3], st[4], st[6]) == (dof, t + 1, 0.0)
        assert st[5] == (1.0 if t + 1 >= 3 and sigma <= 2e-5 * abs(Ibar) else 0.0)
        assert (st[8 + 2 * t], st[9 + 2 * t]) == (I[t], V[t])
    _say(f"flow combine of {T} iterations: {st[0]!r} +- {st[1]:.3e}, chi2/dof {st[2]:.3f}, "
         f"converged {st[5]}")


def _shuffle_multiplier(n):
    """The documented rule: floor(n (sqrt(5)-1)/2) with its lowest bit set,
    stepped by two (mod n) until coprime to n."""
    if n <= 2:
        return 1
    a = (int(n * 0.6180339887498949) | 1) % n
    while math.gcd(a, n) != 1:
        a = (a + 2) % n
    return a


@pytest.mark.parametrize("n", [1, 2, 7, 100003, 1 << 20])
def test_flow_shuffle_is_the_documented_permutation(mc, n):
    import torch
    i = torch.arange(n, dtype=torch.float64, device="cuda")
    x = (i[:, None] + torch.arange(6, dtype=torch.float64, device="cuda")[None, :] / 8).reshape(-1)
    w = i.clone()
    xo = torch.full_like(x, -1.0)
    wo = torch.full_like(w, -1.0)
    mc.mcubes_flow_shuffle(x, w, n, xo, wo)
    torch.cuda.synchronize()
    src = wo.cpu().numpy().astype(np.int64)
    a = _shuffle_multiplier(n)
    assert np.array_equal(src, (np.arange(n, dtype=np.int64) * a) % n)
    assert np.array_equal(np.sort(src), np.arange(n))
    # each row moves whole: x row j is still (src + k/8)
    xr = xo.view(n, 6).cpu().numpy()
    assert np.array_equal(xr, src[:, None] + np.arange(6)[None, :] / 8)
    if n >= 1 << 16:
        # every run of 4096 consecutive outputs draws evenly from the input
        lo = (src < n // 2).reshape(-1)[: (n // 4096) * 4096].reshape(-1, 4096).mean(1)
        assert lo.min() > 0.45 and lo.max() < 0.55


def test_anchored_rounds_recover_a_lost_peak(mc):
    """A flow trained only on the samples of one peak of the correlated
    mixture gives about half the integral.  Its own draws rarely reach the
    other peak, so self-training repairs it slowly if at all; the anchored
    rounds (the first two, by default) also train on the warm-up samples,
    which cover both peaks, and bring the estimate back to the integral."""
    import torch
    pr = workloads.mixture_6d(ncall=1 << 22)
    opts = mc.mcubes_default_options(nbins=500)
    plan = mc.mcubes_plan_create(pr.family, pr.params, 6, pr.ncall, 5, opts)
    B = mc.Buffers(plan)
    p = plan.info["samples_per_cube"]
    mc.mcubes_init_grid(plan, B.grid[0])
    per_it = 1 << 17
    x = torch.empty(8 * per_it * p * 6, dtype=torch.float64, device="cuda")
    w = torch.empty(8 * per_it * p, dtype=torch.float64, device="cuda")
    for t in range(8):
        mc.mcubes_iteration(plan, t, B.grid[t & 1], B.grid[(t + 1) & 1], B.bins, B.partials,
                            B.est, B.state, 0.0)
        r0 = t * per_it * p
        mc.mcubes_vsample_dump(plan, t, B.grid[t & 1], 0, per_it, x[6 * r0:], w[r0:])
    rows = x.view(-1, 6)
    low = rows.mean(1) < 0.5
    xl = rows[low].reshape(-1).contiguous()
    wl = w[low].contiguous()
    nl = int(wl.numel())
    xs, ws = torch.empty_like(xl), torch.empty_like(wl)
    mc.mcubes_flow_shuffle(xl, wl, nl, xs, ws)
    base = mc.Flow(workloads.flow_init(7))
    base.train(xs, ws, nl, 10, 65536, 4e-3)
    est = torch.empty(2, dtype=torch.float64, device="cuda")
    base.vsample(plan, 100, est, precision=mc.MCUBES_BF16)
    torch.cuda.synchronize()
    lost = est[0].item()
    theta = base.params()
    _say(f"one-peak flow: {lost}")
    assert abs(lost - 0.5) < 0.1
    out = {}
    for anc in (1, 0):
        fl = mc.Flow(theta)
        kw = {} if anc else {"anchor_rounds": 0}
        res, rep = fl.integrate(pr.family, pr.params, pr.ncall, 4, 0.0, 5, opts, epochs=0, **kw)
        out[anc] = res["estimate"]
        _say(f"anchor {anc}: {res['estimate']} +- {res['error']:.2e}, used {rep['used_flow']}, "
             f"tail {rep['tail_shape']:.2f}")
    # recovered (measured 0.9987 to 1.0002) against lost (about 0.5)
    assert abs(out[1] - 1.0) < 5e-3
    # Without the anchor the result is left to chance (measured 0.51 to
    # 0.79): the few draws the flow still makes near the lost peak can
    # bring back part of it, so it is reported, not asserted.


def test_flow_pipeline_beats_plain_mcubes_on_the_mixture(mc):
    """The whole pipeline with its default recipe on the correlated mixture
    (6-D, 2^22 samples per iteration; integral 1 to 1.6e-10).  The separable
    VEGAS map cannot follow the correlated peaks: after the warm-up its
    estimate is off by several percent.  Four flow-mapped iterations, on
    the BF16 matrix cores and in FP32, land at least ten times closer, with
    a per-iteration variance typically ten thousand times below the plain
    method's.  Whether the error bars cover the integral is a statement
    over seeds (tests/test_zy_flow_coverage.py)."""
    pr = workloads.mixture_6d(ncall=1 << 22)
    for prec in (mc.MCUBES_BF16, mc.MCUBES_FP32):
        fl = mc.Flow(workloads.flow_init(7))
        res, rep = fl.integrate(pr.family, pr.params, pr.ncall, 4, 0.0, 11,
                                mc.mcubes_default_options(nbins=500), precision=prec)
        _say(f"precision {prec}: plain {rep['plain_estimate']} +- {rep['plain_error']:.2e} "
             f"(chi2 {rep['plain_chi2_dof']:.2f}); flow {res['estimate']} +- {res['error']:.2e}; "
             f"vars {rep['last_plain_var']:.2e} -> {rep['first_flow_var']:.2e}; "
             f"ms warmup {rep['warmup_ms']:.1f} train {rep['train_ms']:.1f} "
             f"flow {rep['flow_ms']:.1f}")
        _say(f"weight tail shape {rep['tail_shape']:.3f}")
        assert rep["used_flow"] == 1 and res["iterations"] == 4
        assert math.isfinite(rep["tail_shape"])
        dev = abs(res["estimate"] - 1.0)
        assert dev < abs(rep["plain_estimate"] - 1.0) / 10
        # typically 1e4 times lower; one of the rare weights of 1e4 adds
        # (1e4 / 2^22)^2 ~ 6e-6 to a single iteration's variance
        assert rep["first_flow_var"] < rep["last_plain_var"] / 10


def test_pipeline_falls_back_to_plain_when_the_flow_loses(mc):
    """With no training at all (epochs and rounds 0) the identity flow is the
    uniform proposal, whose first iteration loses to the warmed-up VEGAS map:
    the judge drops it and the remaining iterations continue the plain
    method from the warm-up's grid, which is what the plain method alone
    gives for the same warm-up plus iterations."""
    pr = workloads.mixture_6d(ncall=1 << 20)
    fl = mc.Flow(workloads.flow_init(7))
    opts = mc.mcubes_default_options(nbins=500)
    res, rep = fl.integrate(pr.family, pr.params, pr.ncall, 4, 0.0, 11, opts,
                            epochs=0, rounds=0, tail_rounds=0, warmup_iters=6)
    assert rep["used_flow"] == 0 and rep["first_flow_var"] > rep["last_plain_var"]
    # 6 warm-up iterations, the dropped flow iteration, 3 plain ones
    plain = mc.mcubes_integrate(pr.family, pr.params, 6, pr.ncall, 9, 0.0, 11, opts)
    _say(f"fallback {res['estimate']} +- {res['error']}; plain {plain['estimate']} +- "
         f"{plain['error']}")
    # the same kernels on the same counters; the bin histograms are flushed
    # with FP64 atomics in no fixed order, and the refinement amplifies those
    # last-bit differences over the nine iterations (measured 3.4e-12)
    assert res["estimate"] == pytest.approx(plain["estimate"], rel=1e-9)
    assert res["error"] == pytest.approx(plain["error"], rel=1e-8)
