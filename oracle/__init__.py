"""CPU oracle of the m-Cubes integrator -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports or calls it.

The arithmetic lives in ``mcubes_oracle.c`` and ``flow_oracle.c`` (plain
single-threaded FP64 C, built by ``oracle/build.py``); this module only
marshals numpy arrays.  Integrand family ids follow the order of eqs. 1-6 of
the paper, then the addition integrand of §5.3 and the correlated Gaussian
mixture used with the learned proposal.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

OSCILLATORY, PRODUCT_PEAK, CORNER_PEAK, GAUSSIAN, C0, DISCONTINUOUS, ADDITION, MIXTURE = range(8)
FAMILY_NAMES = ["oscillatory", "product_peak", "corner_peak", "gaussian", "c0",
                "discontinuous", "addition", "mixture"]

# flow constants (flow_oracle.h)
FLOW_D, FLOW_LAYERS, FLOW_NA, FLOW_NB, FLOW_BLOBS = 6, 4, 3, 3, 32
FLOW_IN, FLOW_HID, FLOW_BINS = FLOW_NA * FLOW_BLOBS, 64, 16
FLOW_RAW = 2 * FLOW_BINS + 1
FLOW_OUT = FLOW_NB * FLOW_RAW
FLOW_LAYER_PARAMS = (FLOW_IN * FLOW_HID + FLOW_HID + FLOW_HID * FLOW_HID + FLOW_HID
                     + FLOW_HID * FLOW_OUT + FLOW_OUT)
FLOW_PARAMS = FLOW_LAYERS * FLOW_LAYER_PARAMS

_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_ip = ctypes.POINTER(ctypes.c_int)


def lib():
    """Load liboracle.so (building it first if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _build
        _build.build()
    L = ctypes.CDLL(LIB_PATH)
    L.mco_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    L.mco_philox4x32_10.restype = None
    L.mco_uniform.argtypes = [ctypes.c_uint32]
    L.mco_uniform.restype = ctypes.c_double
    L.mco_plan.argtypes = [ctypes.c_int, ctypes.c_int64, _i64p]
    L.mco_plan.restype = ctypes.c_int
    L.mco_integrand.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp]
    L.mco_integrand.restype = ctypes.c_double
    L.mco_map.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _ip]
    L.mco_map.restype = ctypes.c_double
    L.mco_sample_range.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int,
                                   ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                   ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, _dp,
                                   ctypes.c_int64, ctypes.c_int64, _dp, _dp]
    L.mco_sample_range.restype = ctypes.c_int
    L.mco_estimates.argtypes = [ctypes.c_int64, ctypes.c_int64, _dp, _dp]
    L.mco_estimates.restype = None
    L.mco_refine.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, _dp, _dp]
    L.mco_refine.restype = ctypes.c_int
    L.mco_combine.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_int, _dp]
    L.mco_combine.restype = ctypes.c_int
    L.mco_integrate.argtypes = [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int64, ctypes.c_int,
                                ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int,
                                ctypes.c_double, ctypes.c_int, ctypes.c_int, _dp, _i64p, _dp, _dp,
                                _dp]
    L.mco_integrate.restype = ctypes.c_int
    L.mcf_param_count.argtypes = []
    L.mcf_param_count.restype = ctypes.c_int
    L.mcf_masks.argtypes = [ctypes.c_int, _ip, _ip]
    L.mcf_masks.restype = None
    for fn in (L.mcf_spline_forward, L.mcf_spline_inverse):
        fn.argtypes = [_dp, ctypes.c_double, _dp, _dp]
        fn.restype = ctypes.c_int
    L.mcf_conditioner.argtypes = [_dp, _dp, ctypes.c_int, _dp]
    L.mcf_conditioner.restype = None
    for fn in (L.mcf_density, L.mcf_sample):
        fn.argtypes = [_dp, _dp, ctypes.c_int, _dp, _dp]
        fn.restype = None
    L.mcf_loss_grad.argtypes = [_dp, ctypes.c_int64, _dp, _dp, _dp]
    L.mcf_loss_grad.restype = ctypes.c_double
    L.mcf_loss_grad_ex.argtypes = [_dp, ctypes.c_int64, _dp, _dp, ctypes.c_int, _dp, _dp]
    L.mcf_loss_grad_ex.restype = ctypes.c_double
    L.mcf_bf16_array.argtypes = [_dp, ctypes.c_int64, _dp]
    L.mcf_bf16_array.restype = None
    L.mcf_adam.argtypes = [_dp, _dp, _dp, _dp, ctypes.c_int64, ctypes.c_int, ctypes.c_double,
                           ctypes.c_double, ctypes.c_double, ctypes.c_double]
    L.mcf_adam.restype = None
    L.mcf_proposal_range.argtypes = [_dp, ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int64,
                                     ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
                                     ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int64,
                                     ctypes.c_int64, _dp]
    L.mcf_proposal_range.restype = ctypes.c_int
    L.mcf_combine_equal.argtypes = [ctypes.c_int, _dp, _dp, _dp]
    L.mcf_combine_equal.restype = ctypes.c_int
    _lib = L
    return L


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def philox4x32_10(counter, key):
    """Philox4x32-10 of one 4-word counter under a 2-word key -> 4 uint32."""
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xffffffff for v in counter])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xffffffff for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().mco_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def uniform(r):
    return lib().mco_uniform(int(r) & 0xffffffff)


def plan(dim, ncall):
    """(g, m, p, N) of the stratification rule; raises on invalid input."""
    out = (ctypes.c_int64 * 4)()
    if lib().mco_plan(int(dim), int(ncall), out) != 0:
        raise ValueError(f"invalid plan arguments dim={dim} ncall={ncall}")
    return tuple(int(v) for v in out)


def integrand(family, params, x):
    x, xp = _d(x)
    params, pp = _d(params)
    return lib().mco_integrand(int(family), len(x), pp, xp)


def uniform_grid(dim, nb):
    e = np.arange(nb + 1, dtype=np.float64) / float(nb)
    return np.tile(e, (dim, 1))


def map_point(grid, z):
    """Map a point given in bin units (z = y * nb) through the grid -> (x, J, bins)."""
    grid, gp = _d(grid)
    dim, nbp1 = grid.shape
    z, zp = _d(z)
    x = np.zeros(dim)
    bins = (ctypes.c_int * dim)()
    J = lib().mco_map(dim, nbp1 - 1, gp, zp, x.ctypes.data_as(_dp), bins)
    return x, J, np.array(list(bins), dtype=np.int64)


def sample_range(family, params, dim, nb, g, m, p, seed, iteration, grid, c_begin, c_end,
                 stream=0):
    """Sums over cubes [c_begin, c_end): (sum S_c, sum var_c, bins[dim, nb])."""
    grid, gp = _d(grid)
    params, pp = _d(params if params is not None else np.zeros(2 * dim))
    sums = np.zeros(2)
    bins = np.zeros((dim, nb))
    rc = lib().mco_sample_range(int(family), int(dim), pp, int(nb), int(g), int(m), int(p),
                                int(seed), int(stream), int(iteration), gp, int(c_begin),
                                int(c_end), sums.ctypes.data_as(_dp), bins.ctypes.data_as(_dp))
    if rc != 0:
        raise ValueError(f"mco_sample_range failed rc={rc}")
    return float(sums[0]), float(sums[1]), bins


def estimates(m, p, sum_s, sum_v):
    s = np.array([sum_s, sum_v])
    e = np.zeros(2)
    lib().mco_estimates(int(m), int(p), s.ctypes.data_as(_dp), e.ctypes.data_as(_dp))
    return float(e[0]), float(e[1])


def iteration(family, params, dim, nb, ncall, seed, it, grid, stream=0):
    """One full iteration -> (I_t, var_t, bins[dim, nb])."""
    g, m, p, _ = plan(dim, ncall)
    s, v, bins = sample_range(family, params, dim, nb, g, m, p, seed, it, grid, 0, m, stream)
    I, var = estimates(m, p, s, v)
    return I, var, bins


def refine(grid, bins, alpha=1.5):
    grid, gp = _d(grid)
    bins, bp = _d(bins)
    dim, nbp1 = grid.shape
    out = np.zeros_like(grid)
    rc = lib().mco_refine(dim, nbp1 - 1, float(alpha), gp, bp, out.ctypes.data_as(_dp))
    if rc != 0:
        raise ValueError("mco_refine failed")
    return out


def combine(I, var, skip=0):
    """-> (Ibar, sigma, chi2_dof, dof)."""
    I, ip = _d(I)
    var, vp = _d(var)
    out = np.zeros(3)
    dof = lib().mco_combine(len(I), ip, vp, int(skip), out.ctypes.data_as(_dp))
    return float(out[0]), float(out[1]), float(out[2]), int(dof)


def integrate(family, params, dim, ncall, itmax, rel_tol, seed, nb=500, alpha=1.5,
              adapt_iters=None, skip=0, stream=0):
    """Whole integrator -> dict with estimate, error, chi2_dof, trace and final grid.
    `stream` is the second Philox counter word (the integrand's index in a batch)."""
    if adapt_iters is None:
        adapt_iters = itmax
    params, pp = _d(params if params is not None else np.zeros(2 * dim))
    res = np.zeros(3)
    info = np.zeros(7, dtype=np.int64)
    grid = np.zeros((dim, nb + 1))
    tI = np.zeros(itmax)
    tV = np.zeros(itmax)
    rc = lib().mco_integrate(int(family), int(dim), pp, int(ncall), int(itmax), float(rel_tol),
                             int(seed), int(stream), int(nb), float(alpha), int(adapt_iters),
                             int(skip),
                             res.ctypes.data_as(_dp), info.ctypes.data_as(_i64p),
                             grid.ctypes.data_as(_dp), tI.ctypes.data_as(_dp),
                             tV.ctypes.data_as(_dp))
    n = int(info[0])
    return {"rc": rc, "estimate": float(res[0]), "error": float(res[1]),
            "chi2_dof": float(res[2]), "iterations": n, "dof": int(info[1]),
            "g": int(info[2]), "m": int(info[3]), "p": int(info[4]), "n": int(info[5]),
            "converged": bool(info[6]), "grid": grid, "trace_I": tI[:n], "trace_var": tV[:n]}


# ---------------------------------------------------------------------------
# learned proposal (flow_oracle.c)
# ---------------------------------------------------------------------------
def flow_masks(layer):
    a = (ctypes.c_int * FLOW_NA)()
    b = (ctypes.c_int * FLOW_NB)()
    lib().mcf_masks(int(layer), a, b)
    return list(a), list(b)


def spline_forward(raw, u):
    """-> (y, pdf, bin) of the piecewise-quadratic CDF with raw parameters raw[33]."""
    raw, rp = _d(raw)
    y, pdf = ctypes.c_double(), ctypes.c_double()
    b = lib().mcf_spline_forward(rp, float(u), ctypes.byref(y), ctypes.byref(pdf))
    return y.value, pdf.value, b


def spline_inverse(raw, y):
    """-> (u, pdf, bin): the inverse CDF."""
    raw, rp = _d(raw)
    u, pdf = ctypes.c_double(), ctypes.c_double()
    b = lib().mcf_spline_inverse(rp, float(y), ctypes.byref(u), ctypes.byref(pdf))
    return u.value, pdf.value, b


def flow_conditioner(layer_params, ua, bf16=False):
    lp, lpp = _d(layer_params)
    ua, up = _d(ua)
    out = np.zeros(FLOW_OUT)
    lib().mcf_conditioner(lpp, up, int(bool(bf16)), out.ctypes.data_as(_dp))
    return out


def flow_density(theta, x, bf16=False):
    """x -> (z, log q(x))."""
    theta, tp = _d(theta)
    x, xp = _d(x)
    z = np.zeros(FLOW_D)
    lq = ctypes.c_double()
    lib().mcf_density(tp, xp, int(bool(bf16)), z.ctypes.data_as(_dp), ctypes.byref(lq))
    return z, lq.value


def flow_sample(theta, z, bf16=False):
    """z -> (x, log q(x))."""
    theta, tp = _d(theta)
    z, zp = _d(z)
    x = np.zeros(FLOW_D)
    lq = ctypes.c_double()
    lib().mcf_sample(tp, zp, int(bool(bf16)), x.ctypes.data_as(_dp), ctypes.byref(lq))
    return x, lq.value


def bf16_round(v):
    """Values rounded to bfloat16 (nearest, ties to even, through FP32), as FP64."""
    v, vp = _d(np.asarray(v, dtype=np.float64).ravel())
    out = np.zeros_like(v)
    lib().mcf_bf16_array(vp, len(v), out.ctypes.data_as(_dp))
    return out


def flow_loss_grad(theta, xs, ws, bf16=False, with_abs=False):
    """-> (loss, grad), or (loss, grad, grad_abs) with `with_abs`: weighted
    negative log-likelihood and its gradient; bf16 rounds the operands of
    every matrix product as a BF16 matrix unit does; grad_abs holds, per
    parameter, the sum of the absolute values of its gradient's terms."""
    theta, tp = _d(theta)
    xs, xp = _d(np.asarray(xs).reshape(-1, FLOW_D))
    ws, wp = _d(ws)
    grad = np.zeros(FLOW_PARAMS)
    gabs = np.zeros(FLOW_PARAMS) if with_abs else None
    loss = lib().mcf_loss_grad_ex(tp, len(ws), xp, wp, int(bool(bf16)), grad.ctypes.data_as(_dp),
                                  gabs.ctypes.data_as(_dp) if with_abs else None)
    return (loss, grad, gabs) if with_abs else (loss, grad)


def flow_adam(theta, m, v, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step; returns new (theta, m, v) arrays."""
    theta = np.array(theta, dtype=np.float64)
    m = np.array(m, dtype=np.float64)
    v = np.array(v, dtype=np.float64)
    grad, gp = _d(grad)
    lib().mcf_adam(theta.ctypes.data_as(_dp), m.ctypes.data_as(_dp), v.ctypes.data_as(_dp), gp,
                   len(theta), int(step), float(lr), float(beta1), float(beta2), float(eps))
    return theta, m, v


def flow_proposal_range(theta, family, params, g, m, p, seed, stream, iteration, c_begin, c_end,
                        bf16=False):
    """Sums (sum S_c, sum var_c) over cubes [c_begin, c_end) of one iteration
    that samples through the flow."""
    theta, tp = _d(theta)
    params, pp = _d(params)
    sums = np.zeros(2)
    rc = lib().mcf_proposal_range(tp, int(bool(bf16)), int(family), pp, int(g), int(m), int(p),
                                  int(seed), int(stream) & 0xffffffff, int(iteration),
                                  int(c_begin), int(c_end), sums.ctypes.data_as(_dp))
    if rc != 0:
        raise ValueError("mcf_proposal_range failed")
    return float(sums[0]), float(sums[1])


def flow_combine(I, var):
    """Equal-weight combination of flow-mapped iterations -> (Ibar, sigma,
    chi2_dof, dof)."""
    I, ip = _d(I)
    var, vp = _d(var)
    out = np.zeros(3)
    dof = lib().mcf_combine_equal(len(I), ip, vp, out.ctypes.data_as(_dp))
    return float(out[0]), float(out[1]), float(out[2]), int(dof)
