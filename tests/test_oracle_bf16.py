"""Pins of the flow oracle's BF16 mode: the bfloat16 rounding itself, the
conditioner, sampling and the flow-mapped iteration with bfloat16 operands,
and the loss gradient with the operands of every matrix product rounded.

Each pin rests on something independent of the oracle's C code:
  * the rounding against torch's float32 -> bfloat16 conversion and
    against the definition of rounding to nearest, ties to even, checked
    value by value in exact arithmetic;
  * the conditioner against a numpy re-statement that rounds with torch;
  * the gradients (FP64 and BF16 modes) against torch autograd (CPU, FP64)
    of a separately written flow, whose rounding points are custom
    autograd functions: forward values rounded (weights, the encoding,
    hidden activations) or the gradient flowing back rounded (the deltas
    entering each matrix product).
"""
import fractions

import numpy as np
import pytest
import torch

import oracle
import workloads


def _bf16_torch(v):
    return torch.tensor(np.asarray(v, dtype=np.float32)).to(torch.bfloat16).to(
        torch.float64).numpy()


def _f32_from_bits(bits):
    return np.asarray(bits, dtype=np.uint32).view(np.float32).astype(np.float64)


# ------------------------------------------------------------ the rounding
def _rounding_inputs():
    rng = np.random.default_rng(2024)
    parts = []
    # random finite float32 bit patterns of both signs (all exponents)
    b = rng.integers(0, 2**32, 60000, dtype=np.uint64).astype(np.uint32)
    b = b[(b & 0x7f800000) != 0x7f800000]
    parts.append(b)
    # exact ties: low 16 bits 0x8000, kept last bit even and odd
    hi = rng.integers(0, 0x7f7f, 8000, dtype=np.uint64).astype(np.uint32) << 16
    parts.append(hi | 0x8000)
    parts.append((hi | 0x10000 | 0x8000) & 0x7fffffff)
    # one below and one above a tie
    parts.append(hi | 0x7fff)
    parts.append(hi | 0x8001)
    # near powers of two (just below: mantissa all ones; just above)
    e = np.arange(1, 254, dtype=np.uint32) << 23
    for m in (0x7fffff, 0x7f8000, 0x7f7fff, 0x000001, 0x008000, 0x018000):
        parts.append(((e - 0x800000) | m) & 0x7fffffff if m >= 0x7f0000 else e | m)
    # subnormals (exponent field 0), including ties there
    parts.append(rng.integers(1, 0x800000, 8000, dtype=np.uint64).astype(np.uint32))
    parts.append((rng.integers(0, 0x80, 500, dtype=np.uint64).astype(np.uint32) << 16) | 0x8000)
    # the largest magnitudes: some round to the largest bfloat16, some overflow
    parts.append(np.arange(0x7f7f0000, 0x7f800000, 7, dtype=np.uint32))
    allb = np.concatenate(parts).astype(np.uint32)
    signs = (rng.integers(0, 2, len(allb)).astype(np.uint32) << 31)
    return np.concatenate([allb, allb ^ signs, np.array([0, 0x80000000], dtype=np.uint32)])


def test_bf16_rounding_matches_torch():
    bits = _rounding_inputs()
    assert len(bits) >= 100000
    v = _f32_from_bits(bits)
    ours = oracle.bf16_round(v)
    ref = _bf16_torch(v)
    same = (ours == ref) | (np.isnan(ours) & np.isnan(ref))
    assert same.all(), v[~same][:5]
    # signed zeros survive, overflow goes to infinity with the sign
    assert np.array_equal(np.signbit(ours), np.signbit(v))
    assert np.isinf(oracle.bf16_round([3.4e38, -3.4e38])).all()
    assert oracle.bf16_round([3.39e38])[0] == float.fromhex("0x1.fep+127")


def test_bf16_rounding_is_round_to_nearest_even_by_definition():
    """Exact arithmetic (fractions): the result is a bfloat16 value (8
    significant bits, or a subnormal multiple of 2^-133), no bfloat16 value
    lies strictly nearer, and a tie picks an even last bit."""
    bits = _rounding_inputs()[::23]
    v = _f32_from_bits(bits)
    ours = oracle.bf16_round(v)
    for x, r in zip(v, ours):
        if np.isinf(r):
            # rounds to infinity only from at or above max + half an ulp
            assert abs(fractions.Fraction(x)) >= fractions.Fraction(2**128 - 2**119)
            continue
        rb = np.array([r], dtype=np.float32).view(np.uint32)[0]
        assert rb & 0xffff == 0  # representable in bfloat16
        lo = (rb - 0x10000) if (rb & 0x7fffffff) else None
        up = rb + 0x10000
        d = abs(fractions.Fraction(x) - fractions.Fraction(float(r)))
        for nb in (lo, up):
            if nb is None or (nb & 0x7f800000) == 0x7f800000:
                continue
            other = float(np.array([nb], dtype=np.uint32).view(np.float32)[0])
            if np.sign(other) != np.sign(r) and r != 0:
                continue
            dn = abs(fractions.Fraction(x) - fractions.Fraction(other))
            assert d <= dn, (x, r, other)
            if d == dn:
                assert (rb >> 16) & 1 == 0, (x, r)


# --------------------------------------------------------- the conditioner
def _layer(theta, l):
    lp = oracle.FLOW_LAYER_PARAMS
    return theta[l * lp:(l + 1) * lp]


def _split(P):
    i, h, o = oracle.FLOW_IN, oracle.FLOW_HID, oracle.FLOW_OUT
    W1 = P[:i * h].reshape(i, h)
    b1 = P[i * h:i * h + h]
    off = i * h + h
    W2 = P[off:off + h * h].reshape(h, h)
    b2 = P[off + h * h:off + h * h + h]
    off += h * h + h
    W3 = P[off:off + h * o].reshape(h, o)
    b3 = P[off + h * o:off + h * o + o]
    return W1, b1, W2, b2, W3, b3


def _blobs(ua):
    k = (np.arange(oracle.FLOW_BLOBS) + 0.5) / oracle.FLOW_BLOBS
    t = (np.asarray(ua)[:, None] - k[None, :]) * oracle.FLOW_BLOBS
    return np.exp(-0.5 * t * t).ravel()


@pytest.mark.parametrize("seed", range(4))
def test_bf16_conditioner_against_numpy(seed):
    theta = workloads.flow_random(30 + seed, out_scale=0.5)
    rng = np.random.default_rng(seed)
    for l in range(4):
        W1, b1, W2, b2, W3, b3 = _split(_layer(theta, l))
        for ua in rng.uniform(0, 1, (6, 3)):
            e = _bf16_torch(_blobs(ua))
            h1 = _bf16_torch(np.maximum(e @ _bf16_torch(W1.ravel()).reshape(W1.shape)
                                        + b1.astype(np.float32), 0.0))
            h2 = _bf16_torch(np.maximum(h1 @ _bf16_torch(W2.ravel()).reshape(W2.shape)
                                        + b2.astype(np.float32), 0.0))
            out = h2 @ _bf16_torch(W3.ravel()).reshape(W3.shape) + b3.astype(np.float32)
            got = oracle.flow_conditioner(_layer(theta, l), ua, bf16=True)
            np.testing.assert_allclose(got, out, rtol=1e-12, atol=1e-14)
            # and the rounding shows against the FP64 conditioner
            full = oracle.flow_conditioner(_layer(theta, l), ua, bf16=False)
            assert np.abs(full - got).max() > 1e-5


@pytest.mark.parametrize("seed", range(3))
def test_bf16_sample_and_density_are_inverse(seed):
    """The BF16 conditioner depends only on the kept coordinates, so the
    BF16 flow is still an exact bijection: sampling inverts the density
    direction and both give the same log q."""
    theta = workloads.flow_random(40 + seed, out_scale=0.6)
    for x in np.random.default_rng(seed).uniform(0.01, 0.99, (20, 6)):
        z, lq = oracle.flow_density(theta, x, bf16=True)
        x2, lq2 = oracle.flow_sample(theta, z, bf16=True)
        np.testing.assert_allclose(x2, x, atol=1e-12)
        assert lq2 == pytest.approx(lq, abs=1e-11)
        z64, lq64 = oracle.flow_density(theta, x, bf16=False)
        assert abs(lq64 - lq) > 1e-7  # a different map


def test_bf16_identity_flow_iteration_is_plain_mcubes():
    """A zero output layer is the identity in BF16 too (the rounded zero is
    zero), so the flow-mapped iteration equals plain m-Cubes on the uniform
    grid with the flow's stream word."""
    theta = workloads.flow_init(3)
    prob = workloads.mixture_6d()
    g, m, p, _ = oracle.plan(6, 4000)
    stream = 0x80000000
    s_flow, v_flow = oracle.flow_proposal_range(theta, prob.family, prob.params, g, m, p, 5,
                                                stream, 2, 0, m, bf16=True)
    s_pl, v_pl, _ = oracle.sample_range(prob.family, prob.params, 6, 50, g, m, p, 5, 2,
                                        oracle.uniform_grid(6, 50), 0, m, stream=stream)
    assert s_flow == pytest.approx(s_pl, rel=1e-13)
    assert v_flow == pytest.approx(v_pl, rel=1e-11)


def test_bf16_flow_iteration_is_the_mean_of_f_over_q():
    """The BF16 flow-mapped iteration over a few cubes, recomputed sample by
    sample from the oracle's own Philox stream and BF16 sampling: the cube
    sums are f(x)/q(x) at x = flow(z), z_j = (c_j + u_j)/g."""
    theta = workloads.flow_random(9, out_scale=0.5)
    prob = workloads.mixture_6d()
    g, m, p, _ = 3, 3**6, 2, None
    seed, stream, it = 11, 0x80000000, 1
    S = V = 0.0
    for c in range(0, 17):
        digits = [(c // g**j) % g for j in range(6)]
        ws = []
        for k in range(p):
            z = np.zeros(6)
            for b in range(2):
                r = oracle.philox4x32_10([c, stream, k * 2 + b, it], [seed, 0])
                for l in range(4):
                    if 4 * b + l < 6:
                        z[4 * b + l] = (digits[4 * b + l] + oracle.uniform(r[l])) / g
            x, lq = oracle.flow_sample(theta, z, bf16=True)
            ws.append(oracle.integrand(prob.family, prob.params, x) / np.exp(lq))
        S += sum(ws)
        V += (ws[1] - ws[0]) ** 2 / 2.0
    s, v = oracle.flow_proposal_range(theta, prob.family, prob.params, g, m, p, seed, stream, it,
                                      0, 17, bf16=True)
    assert s == pytest.approx(S, rel=1e-12)
    assert v == pytest.approx(V, rel=1e-9)


# ------------------------------------------------ the gradient, by autograd
class _RoundFwd(torch.autograd.Function):
    """Value rounded to bfloat16; the gradient passes unchanged."""
    @staticmethod
    def forward(ctx, x):
        return x.float().to(torch.bfloat16).double()

    @staticmethod
    def backward(ctx, g):
        return g


class _RoundBwd(torch.autograd.Function):
    """Value unchanged; the gradient flowing back is rounded to bfloat16."""
    @staticmethod
    def forward(ctx, x):
        return x.clone()

    @staticmethod
    def backward(ctx, g):
        return g.float().to(torch.bfloat16).double()


_A = [[0, 1, 2], [3, 4, 5], [0, 2, 4], [1, 3, 5]]
_B = [[3, 4, 5], [0, 1, 2], [1, 3, 5], [0, 2, 4]]


def _spline_fwd(raw, u):
    """Piecewise-quadratic CDF and its density (rows: samples)."""
    nb = oracle.FLOW_BINS
    wr, vr = raw[:, :nb], raw[:, nb:]
    W = torch.softmax(wr, dim=1)
    E = torch.exp(vr - vr.max(dim=1, keepdim=True).values.detach())
    Z = (0.5 * (E[:, :-1] + E[:, 1:]) * W).sum(dim=1, keepdim=True)
    V = E / Z
    zero = torch.zeros_like(u)[:, None]
    X = torch.cat([zero, torch.cumsum(W, dim=1)], dim=1)
    Acum = torch.cat([zero, torch.cumsum(0.5 * (V[:, :-1] + V[:, 1:]) * W, dim=1)], dim=1)
    b = (X[:, 1:nb].detach() <= u.detach()[:, None]).sum(dim=1, keepdim=True)
    Xb, Wb, Ab = X.gather(1, b), W.gather(1, b), Acum.gather(1, b)
    Vb, Vb1 = V.gather(1, b), V.gather(1, b + 1)
    a = ((u[:, None] - Xb) / Wb).clamp(0.0, 1.0)
    dV = Vb1 - Vb
    y = Ab + Wb * (a * Vb + 0.5 * a * a * dV)
    pdf = Vb + a * dV
    return y[:, 0], pdf[:, 0]


def _torch_loss(theta, xs, ws, bf16):
    rf = _RoundFwd.apply if bf16 else (lambda t: t)
    rb = _RoundBwd.apply if bf16 else (lambda t: t)
    f32 = (lambda t: t.float().double()) if bf16 else (lambda t: t)
    lp = oracle.FLOW_LAYER_PARAMS
    u = [xs[:, j] for j in range(6)]
    lq = torch.zeros(xs.shape[0], dtype=torch.float64)
    k = (torch.arange(oracle.FLOW_BLOBS, dtype=torch.float64) + 0.5) / oracle.FLOW_BLOBS
    for l in range(4):
        W1, b1, W2, b2, W3, b3 = _split(theta[l * lp:(l + 1) * lp])
        ua = torch.stack([u[j] for j in _A[l]], dim=1)
        t = (ua[:, :, None] - k) * oracle.FLOW_BLOBS
        e = rf(torch.exp(-0.5 * t * t).reshape(xs.shape[0], -1))
        h1 = rf(torch.relu(rb(e @ rf(W1) + f32(b1))))
        h2 = rf(torch.relu(rb(h1 @ rf(W2) + f32(b2))))
        out = rb(h2 @ rf(W3) + f32(b3))
        for tt, j in enumerate(_B[l]):
            y, pdf = _spline_fwd(out[:, tt * oracle.FLOW_RAW:(tt + 1) * oracle.FLOW_RAW], u[j])
            u[j] = y
            lq = lq + torch.log(pdf)
    return -(ws * lq).sum() / ws.sum()


@pytest.mark.parametrize("bf16", [False, True])
def test_loss_gradient_against_autograd(bf16):
    theta = workloads.flow_random(21, out_scale=0.5)
    rng = np.random.default_rng(5)
    n = 48
    xs = rng.uniform(0.02, 0.98, (n, 6))
    ws = rng.uniform(0.1, 3.0, n)
    loss, grad, gabs = oracle.flow_loss_grad(theta, xs, ws, bf16=bf16, with_abs=True)
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    tl = _torch_loss(th, torch.tensor(xs), torch.tensor(ws), bf16)
    tl.backward()
    g_ref = th.grad.numpy()
    assert loss == pytest.approx(tl.item(), rel=1e-12)
    # Per component, against the scale of the terms it sums.  A term that is
    # itself the result of cancellation (a delta far below the values it came
    # from) carries a relative error well above 2^-53, in FP64 up to ~1e-10;
    # in BF16 mode such a term, when it sits that close to a rounding
    # boundary, can round to the neighbouring bfloat16 value on one side only.
    # Nearly every component agrees to the last bits; none beyond those two.
    err = np.abs(grad - g_ref)
    gmax = np.abs(g_ref).max()
    close = err <= 1e-12 * gabs + 1e-16 * gmax
    assert close.mean() >= 0.99
    rtol = 1e-6 if bf16 else 1e-9
    assert np.all(err <= rtol * gabs + 1e-14 * gmax), np.argmax(err / (gabs + 1e-300))
    assert np.all(np.abs(grad) <= gabs * (1 + 1e-12))
    # every block of the layout carries weight (no block vanishes or stays zero)
    lp = oracle.FLOW_LAYER_PARAMS
    i, h, o = oracle.FLOW_IN, oracle.FLOW_HID, oracle.FLOW_OUT
    bounds = np.cumsum([0, i * h, h, h * h, h, h * o, o])
    for l in range(4):
        for a, b in zip(bounds[:-1], bounds[1:]):
            blk = slice(l * lp + a, l * lp + b)
            assert np.linalg.norm(g_ref[blk]) > 0
            rel = np.linalg.norm(grad[blk] - g_ref[blk]) / np.linalg.norm(g_ref[blk])
            assert rel < (1e-6 if bf16 else 1e-10)


def test_bf16_gradient_differs_from_fp64_by_the_rounding():
    """BF16 mode is a perturbation of the FP64 gradient of the size the
    rounding predicts (a few 2^-9 relative per operand), not another
    function: close in direction, not identical."""
    theta = workloads.flow_random(4, out_scale=0.4)
    rng = np.random.default_rng(12)
    xs = rng.uniform(0.02, 0.98, (200, 6))
    ws = rng.uniform(0.1, 3.0, 200)
    _, g64 = oracle.flow_loss_grad(theta, xs, ws)
    _, g16 = oracle.flow_loss_grad(theta, xs, ws, bf16=True)
    rel = np.linalg.norm(g16 - g64) / np.linalg.norm(g64)
    assert 1e-4 < rel < 5e-2
