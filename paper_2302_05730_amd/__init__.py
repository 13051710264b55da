"""Python binding of libmcubes, the MI355X (gfx950) m-Cubes integrator.

Argument marshalling only: every entry point forwards to the C function of the
same name declared in include/mcubes.h, and all arithmetic runs in the HIP
kernels of the library.  Device buffers are PyTorch tensors (float64, on the
GPU, contiguous) or raw device addresses; streams default to PyTorch's current
stream.  There is no CPU fallback: if libmcubes.so is missing, importing
anything that needs it raises.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmcubes.so")

MCUBES_MAX_DIM = 10
MCUBES_MAX_BINS = 500
MCUBES_STATE_HEADER = 8
MCUBES_MAX_ITERATIONS = 1024
MCUBES_STATE_LEN = MCUBES_STATE_HEADER + 2 * MCUBES_MAX_ITERATIONS

MCUBES_OK, MCUBES_NOT_CONVERGED = 0, 1
MCUBES_E_ARG, MCUBES_E_INTEGRAND, MCUBES_E_NONFINITE, MCUBES_E_DEVICE, MCUBES_E_ALLOC = (
    -1, -2, -3, -4, -5)
(MCUBES_OSCILLATORY, MCUBES_PRODUCT_PEAK, MCUBES_CORNER_PEAK, MCUBES_GAUSSIAN, MCUBES_C0,
 MCUBES_DISCONTINUOUS, MCUBES_ADDITION, MCUBES_MIXTURE) = range(8)
MCUBES_FP64, MCUBES_FP32, MCUBES_BF16 = 0, 1, 2
MCUBES_FLOW_DIM, MCUBES_FLOW_PARAMS = 6, 67212
(MCUBES_MB_INTEGRAND, MCUBES_MB_PHILOX, MCUBES_MB_EXP64, MCUBES_MB_COS64, MCUBES_MB_POW64,
 MCUBES_MB_EXP32, MCUBES_MB_COS32, MCUBES_MB_POW32) = range(8)


class MCubesError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"mcubes error {code}: {message}")
        self.code = code


class mcubes_options(ctypes.Structure):
    _fields_ = [("nbins", ctypes.c_int32), ("adapt_iters", ctypes.c_int32),
                ("skip", ctypes.c_int32), ("block_size", ctypes.c_int32),
                ("blocks", ctypes.c_int32), ("stream_id", ctypes.c_uint32),
                ("precision", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("stream", ctypes.c_void_p)]


class mcubes_result(ctypes.Structure):
    _fields_ = [("estimate", ctypes.c_double), ("error", ctypes.c_double),
                ("chi2_dof", ctypes.c_double), ("iterations", ctypes.c_int32),
                ("dof", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("status", ctypes.c_int32), ("cube_side", ctypes.c_int64),
                ("ncubes", ctypes.c_int64), ("samples_per_cube", ctypes.c_int64),
                ("samples_per_iter", ctypes.c_int64), ("kernel_ms", ctypes.c_double)]


class mcubes_plan_info(ctypes.Structure):
    _fields_ = [("family", ctypes.c_int32), ("dim", ctypes.c_int32), ("nbins", ctypes.c_int32),
                ("block_size", ctypes.c_int32), ("blocks", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("cube_side", ctypes.c_int64),
                ("ncubes", ctypes.c_int64), ("samples_per_cube", ctypes.c_int64),
                ("samples_per_iter", ctypes.c_int64), ("grid_len", ctypes.c_int64),
                ("bins_len", ctypes.c_int64), ("partials_len", ctypes.c_int64),
                ("state_len", ctypes.c_int64)]


class mcubes_flow_options(ctypes.Structure):
    _fields_ = [("warmup_iters", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("train_items", ctypes.c_int64), ("epochs", ctypes.c_int32),
                ("rounds", ctypes.c_int32), ("round_samples", ctypes.c_int64),
                ("round_epochs", ctypes.c_int32), ("tail_rounds", ctypes.c_int32),
                ("batch", ctypes.c_int64), ("lr", ctypes.c_double), ("round_lr", ctypes.c_double),
                ("tail_power", ctypes.c_double), ("tail_lr", ctypes.c_double),
                ("train_precision", ctypes.c_int32), ("anchor_rounds", ctypes.c_int32),
                ("min_iters", ctypes.c_int32)]


class mcubes_flow_report(ctypes.Structure):
    _fields_ = [("warmup_ms", ctypes.c_double), ("train_ms", ctypes.c_double),
                ("flow_ms", ctypes.c_double), ("total_ms", ctypes.c_double),
                ("plain_estimate", ctypes.c_double), ("plain_error", ctypes.c_double),
                ("plain_chi2_dof", ctypes.c_double), ("last_plain_var", ctypes.c_double),
                ("first_flow_var", ctypes.c_double), ("final_loss", ctypes.c_double),
                ("flow_iterations", ctypes.c_int32), ("used_flow", ctypes.c_int32),
                ("tail_shape", ctypes.c_double)]


class mcubes_batch_item(ctypes.Structure):
    _fields_ = [("family", ctypes.c_int32), ("dim", ctypes.c_int32), ("ncall", ctypes.c_int64),
                ("params", ctypes.c_double * (2 * MCUBES_MAX_DIM))]


class mcubes_batch_info(ctypes.Structure):
    _fields_ = [("items", ctypes.c_int32), ("classes", ctypes.c_int32),
                ("tiles", ctypes.c_int32), ("launches", ctypes.c_int32),
                ("nbins", ctypes.c_int32), ("tuned", ctypes.c_int32),
                ("streams", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("grids_len", ctypes.c_int64), ("samples_per_iter", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("last_iterations", ctypes.c_int32),
                ("last_replans", ctypes.c_int32), ("last_samples", ctypes.c_int64),
                ("last_ms", ctypes.c_double)]


class mcubes_batch_class(ctypes.Structure):
    _fields_ = [("family", ctypes.c_int32), ("dim", ctypes.c_int32), ("p2", ctypes.c_int32),
                ("items", ctypes.c_int32), ("block_size", ctypes.c_int32),
                ("shares", ctypes.c_int32), ("tiles", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int32), ("samples", ctypes.c_int64),
                ("tuned_ms", ctypes.c_double), ("default_ms", ctypes.c_double)]


_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p
_lib = None

# name -> (restype, argtypes), mirroring include/mcubes.h
_SIGNATURES = {
    "mcubes_default_options": (None, [ctypes.POINTER(mcubes_options)]),
    "mcubes_last_error": (ctypes.c_char_p, []),
    "mcubes_plan_sizes": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64,
                                         ctypes.POINTER(ctypes.c_int64)]),
    "mcubes_integrate": (ctypes.c_int, [ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int64,
                                        ctypes.c_int, ctypes.c_double, ctypes.c_uint64,
                                        ctypes.POINTER(mcubes_options),
                                        ctypes.POINTER(mcubes_result), _dp, _dp]),
    "mcubes_integrate_noalloc": (ctypes.c_int, [ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int64,
                                                ctypes.c_int, ctypes.c_double, ctypes.c_uint64,
                                                ctypes.POINTER(mcubes_options),
                                                ctypes.POINTER(mcubes_result), _dp, _dp]),
    "mcubes_plan_create": (ctypes.c_int, [ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int64,
                                          ctypes.c_uint64, ctypes.POINTER(mcubes_options),
                                          ctypes.POINTER(_vp)]),
    "mcubes_plan_get_info": (ctypes.c_int, [_vp, ctypes.POINTER(mcubes_plan_info)]),
    "mcubes_plan_destroy": (None, [_vp]),
    "mcubes_init_grid": (ctypes.c_int, [_vp, _vp, _vp]),
    "mcubes_fill": (ctypes.c_int, [_vp, ctypes.c_int64, ctypes.c_double, _vp]),
    "mcubes_vsample": (ctypes.c_int, [_vp, ctypes.c_uint32, _vp, _vp, _vp, _vp]),
    "mcubes_reduce": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "mcubes_combine": (ctypes.c_int, [_vp, ctypes.c_uint32, _vp, _vp, ctypes.c_double, _vp]),
    "mcubes_refine": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "mcubes_iteration": (ctypes.c_int, [_vp, ctypes.c_uint32, _vp, _vp, _vp, _vp, _vp, _vp,
                                        ctypes.c_double, _vp]),
    "mcubes_iterate": (ctypes.c_int, [_vp, _dp, ctypes.c_uint32, _dp, _dp, _dp, _dp]),
    "mcubes_microbench": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, _vp,
                                         ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_int,
                                         _vp, _vp]),
    "mcubes_batch_create": (ctypes.c_int, [ctypes.POINTER(mcubes_batch_item), ctypes.c_int,
                                           ctypes.c_uint64, ctypes.POINTER(mcubes_options),
                                           ctypes.POINTER(_vp)]),
    "mcubes_batch_destroy": (None, [_vp]),
    "mcubes_batch_get_info": (ctypes.c_int, [_vp, ctypes.POINTER(mcubes_batch_info)]),
    "mcubes_batch_get_class": (ctypes.c_int, [_vp, ctypes.c_int,
                                              ctypes.POINTER(mcubes_batch_class)]),
    "mcubes_batch_configure_class": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int,
                                                    ctypes.c_int]),
    "mcubes_batch_autotune": (ctypes.c_int, [_vp]),
    "mcubes_batch_set_streams": (ctypes.c_int, [_vp, ctypes.c_int]),
    "mcubes_batch_step": (ctypes.c_int, [_vp, ctypes.c_uint32, _dp, _dp]),
    "mcubes_flow_create": (ctypes.c_int, [_dp, ctypes.POINTER(_vp)]),
    "mcubes_flow_destroy": (None, [_vp]),
    "mcubes_flow_get_params": (ctypes.c_int, [_vp, _dp]),
    "mcubes_flow_set_params": (ctypes.c_int, [_vp, _dp]),
    "mcubes_flow_density": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_int64, _vp, _vp, _vp]),
    "mcubes_flow_sample": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_int64, _vp, _vp, _vp]),
    "mcubes_flow_loss_grad": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, ctypes.c_int64, _vp,
                                             _vp, _vp]),
    "mcubes_flow_adam_step": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_double, ctypes.c_double, _vp]),
    "mcubes_flow_train": (ctypes.c_int, [_vp, ctypes.c_int, _vp, _vp, ctypes.c_int64,
                                         ctypes.c_int, ctypes.c_int64, ctypes.c_double, _dp, _vp]),
    "mcubes_vsample_dump": (ctypes.c_int, [_vp, ctypes.c_uint32, _vp, ctypes.c_int64,
                                           ctypes.c_int64, _vp, _vp, _vp]),
    "mcubes_flow_vsample": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_uint32, _vp, _vp]),
    "mcubes_flow_combine": (ctypes.c_int, [ctypes.c_uint32, _vp, _vp, ctypes.c_double,
                                           ctypes.c_int, _vp]),
    "mcubes_flow_shuffle": (ctypes.c_int, [_vp, _vp, ctypes.c_int64, _vp, _vp, _vp]),
    "mcubes_flow_draw": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_uint32, ctypes.c_int64,
                                        _vp, _vp, _vp]),
    "mcubes_default_flow_options": (None, [ctypes.POINTER(mcubes_flow_options)]),
    "mcubes_weight_tail_shape": (ctypes.c_int, [_vp, _dp, ctypes.POINTER(ctypes.c_int64)]),
    "mcubes_flow_weight_tail": (ctypes.c_int, [_vp, _dp, ctypes.POINTER(ctypes.c_int64)]),
    "mcubes_flow_integrate": (ctypes.c_int, [_vp, ctypes.c_int, _dp, ctypes.c_int64, ctypes.c_int,
                                             ctypes.c_double, ctypes.c_uint64,
                                             ctypes.POINTER(mcubes_options),
                                             ctypes.POINTER(mcubes_flow_options),
                                             ctypes.POINTER(mcubes_result),
                                             ctypes.POINTER(mcubes_flow_report)]),
    "mcubes_batch_integrate": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                              ctypes.POINTER(mcubes_result), _dp, _dp]),
}


def lib():
    """The loaded libmcubes.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python paper_2302_05730_amd/build.py` (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def mcubes_last_error():
    return lib().mcubes_last_error().decode()


def _check(rc, allow=(MCUBES_OK,)):
    if rc not in allow:
        raise MCubesError(rc, mcubes_last_error())
    return rc


def _dev(t, n=None, name="buffer"):
    """Device address of a float64 tensor (or a raw int address)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    import torch
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 GPU tensor")
    if n is not None and t.numel() < n:
        raise ValueError(f"{name} needs {n} elements, has {t.numel()}")
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _params(params, dim):
    if params is None:
        return None, None
    arr = (ctypes.c_double * (2 * dim))(*[float(v) for v in list(params)[:2 * dim]])
    return arr, ctypes.cast(arr, _dp)


def mcubes_default_options(**overrides):
    opt = mcubes_options()
    lib().mcubes_default_options(ctypes.byref(opt))
    for k, v in overrides.items():
        setattr(opt, k, v)
    return opt


def mcubes_plan_sizes(dim, ncall):
    out = (ctypes.c_int64 * 4)()
    _check(lib().mcubes_plan_sizes(int(dim), int(ncall), out))
    return tuple(int(v) for v in out)


def mcubes_integrate(family, params, dim, ncall, itmax, rel_tol, seed, options=None,
                     grid=True, trace=True):
    """Whole integrator.  Returns a dict with the mcubes_result fields plus the
    final grid (list of dim rows) and the per-iteration (I_t, var_t) trace."""
    return _integrate("mcubes_integrate", family, params, dim, ncall, itmax, rel_tol, seed,
                      options, grid, trace)


def mcubes_integrate_noalloc(family, params, dim, ncall, itmax, rel_tol, seed, options=None,
                             grid=True, trace=True):
    """mcubes_integrate on the library's static device scratch (no device
    allocation); same return value."""
    return _integrate("mcubes_integrate_noalloc", family, params, dim, ncall, itmax, rel_tol,
                      seed, options, grid, trace)


def _integrate(name, family, params, dim, ncall, itmax, rel_tol, seed, options, grid, trace):
    keep, pp = _params(params, dim)
    opt = options if options is not None else mcubes_default_options()
    res = mcubes_result()
    nb = opt.nbins
    g_buf = (ctypes.c_double * (dim * (nb + 1)))() if grid else None
    t_buf = (ctypes.c_double * (2 * itmax))() if trace else None
    rc = getattr(lib(), name)(int(family), pp, int(dim), int(ncall), int(itmax), float(rel_tol),
            int(seed) & (2**64 - 1), ctypes.byref(opt), ctypes.byref(res),
            ctypes.cast(g_buf, _dp) if grid else None,
            ctypes.cast(t_buf, _dp) if trace else None)
    _check(rc, allow=(MCUBES_OK, MCUBES_NOT_CONVERGED))
    out = {f: getattr(res, f) for f, _ in mcubes_result._fields_}
    out["converged"] = bool(out["converged"])
    n = res.iterations
    if grid:
        out["grid"] = [list(g_buf[j * (nb + 1):(j + 1) * (nb + 1)]) for j in range(dim)]
    if trace:
        out["trace_I"] = [t_buf[2 * t] for t in range(n)]
        out["trace_var"] = [t_buf[2 * t + 1] for t in range(n)]
    return out


class Plan:
    """Owns an mcubes_plan*; destroyed with the object."""

    def __init__(self, handle):
        self.handle = handle
        self.info = mcubes_plan_get_info(self)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.mcubes_plan_destroy(self.handle)
            self.handle = None


def mcubes_plan_create(family, params, dim, ncall, seed, options=None):
    keep, pp = _params(params, dim)
    opt = options if options is not None else mcubes_default_options()
    h = _vp()
    _check(lib().mcubes_plan_create(int(family), pp, int(dim), int(ncall),
                                    int(seed) & (2**64 - 1), ctypes.byref(opt), ctypes.byref(h)))
    return Plan(h)


def mcubes_plan_get_info(plan):
    info = mcubes_plan_info()
    _check(lib().mcubes_plan_get_info(plan.handle, ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in mcubes_plan_info._fields_}


def mcubes_plan_destroy(plan):
    if plan.handle:
        lib().mcubes_plan_destroy(plan.handle)
        plan.handle = None


def mcubes_init_grid(plan, d_grid, stream=None):
    _check(lib().mcubes_init_grid(plan.handle, _dev(d_grid, plan.info["grid_len"], "grid"),
                                  _stream(stream)))


def mcubes_fill(d, value, n=None, stream=None):
    n = d.numel() if n is None else n
    _check(lib().mcubes_fill(_dev(d, n), int(n), float(value), _stream(stream)))


def mcubes_vsample(plan, iteration, d_grid, d_bins, d_partials, stream=None):
    i = plan.info
    _check(lib().mcubes_vsample(plan.handle, int(iteration), _dev(d_grid, i["grid_len"], "grid"),
                                _dev(d_bins, i["bins_len"], "bins"),  # None: no bin sums
                                _dev(d_partials, i["partials_len"], "partials"),
                                _stream(stream)))


def mcubes_reduce(plan, d_partials, d_est, stream=None):
    i = plan.info
    _check(lib().mcubes_reduce(plan.handle, _dev(d_partials, i["partials_len"], "partials"),
                               _dev(d_est, 2, "est"), _stream(stream)))


def mcubes_combine(plan, iteration, d_est, d_state, rel_tol, stream=None):
    _check(lib().mcubes_combine(plan.handle, int(iteration), _dev(d_est, 2, "est"),
                                _dev(d_state, MCUBES_STATE_LEN, "state"), float(rel_tol),
                                _stream(stream)))


def mcubes_flow_combine(iteration, d_est, d_state, rel_tol, min_iters=1, stream=None):
    _check(lib().mcubes_flow_combine(int(iteration), _dev(d_est, 2, "est"),
                                     _dev(d_state, MCUBES_STATE_LEN, "state"), float(rel_tol),
                                     int(min_iters), _stream(stream)))


def mcubes_flow_shuffle(d_x, d_w, n, d_x_out, d_w_out, stream=None):
    _check(lib().mcubes_flow_shuffle(_dev(d_x, 6 * n, "x"), _dev(d_w, n, "w"), int(n),
                                     _dev(d_x_out, 6 * n, "x_out"), _dev(d_w_out, n, "w_out"),
                                     _stream(stream)))


def mcubes_refine(plan, d_grid, d_bins, d_grid_out, stream=None):
    i = plan.info
    _check(lib().mcubes_refine(plan.handle, _dev(d_grid, i["grid_len"], "grid"),
                               _dev(d_bins, i["bins_len"], "bins"),
                               _dev(d_grid_out, i["grid_len"], "grid_out"), _stream(stream)))


def mcubes_iteration(plan, iteration, d_grid, d_grid_out, d_bins, d_partials, d_est, d_state,
                     rel_tol, stream=None):
    i = plan.info
    _check(lib().mcubes_iteration(plan.handle, int(iteration),
                                  _dev(d_grid, i["grid_len"], "grid"),
                                  _dev(d_grid_out, i["grid_len"], "grid_out"),
                                  _dev(d_bins, i["bins_len"], "bins"),
                                  _dev(d_partials, i["partials_len"], "partials"),
                                  _dev(d_est, 2, "est"), _dev(d_state, MCUBES_STATE_LEN, "state"),
                                  float(rel_tol), _stream(stream)))


def mcubes_iterate(plan, grid_in, iteration, bins=True, refine=True):
    """One iteration on host arrays: grid_in (dim x (nbins+1)) -> (I_t, var_t,
    bins or None, refined grid or None)."""
    import numpy as np
    i = plan.info
    g = np.ascontiguousarray(grid_in, dtype=np.float64).reshape(-1)
    if g.size != i["grid_len"]:
        raise ValueError(f"grid_in holds {g.size} values, the plan needs {i['grid_len']}")
    I_t, var_t = ctypes.c_double(), ctypes.c_double()
    b = np.zeros(i["bins_len"]) if bins else None
    go = np.zeros(i["grid_len"]) if refine else None
    ptr = lambda a: a.ctypes.data_as(_dp) if a is not None else None  # noqa: E731
    _check(lib().mcubes_iterate(plan.handle, ptr(g), int(iteration), ctypes.byref(I_t),
                                ctypes.byref(var_t), ptr(b), ptr(go)))
    shape_b, shape_g = (i["dim"], i["nbins"]), (i["dim"], i["nbins"] + 1)
    return (I_t.value, var_t.value, b.reshape(shape_b) if bins else None,
            go.reshape(shape_g) if refine else None)


def mcubes_microbench(kind, d_out, blocks, block, calls_per_thread, family=0, params=None, dim=1,
                      d_points=None, npts=0, stream=None):
    keep, pp = _params(params, dim)
    _check(lib().mcubes_microbench(int(kind), int(family), pp, int(dim),
                                   _dev(d_points, npts * dim, "points") if d_points is not None
                                   else None, int(npts), int(calls_per_thread), int(blocks),
                                   int(block), _dev(d_out, blocks * block, "out"), _stream(stream)))


class Buffers:
    """Device buffers (torch float64 tensors) sized for a plan's step API."""

    def __init__(self, plan, device="cuda"):
        import torch
        i = plan.info
        z = lambda n: torch.zeros(int(n), dtype=torch.float64, device=device)  # noqa: E731
        self.grid = [z(i["grid_len"]), z(i["grid_len"])]
        self.bins = z(i["bins_len"])
        self.partials = z(i["partials_len"])
        self.est = z(2)
        self.state = z(MCUBES_STATE_LEN)


class Batch:
    """Owns an mcubes_batch* (the batched form); destroyed with the object.

    items: sequence of (family, dim, ncall, params) with params the 2*dim
    values [a..., u...] (None for the addition integrand)."""

    def __init__(self, items, seed, options=None):
        n = len(items)
        arr = (mcubes_batch_item * max(n, 1))()
        for i, (family, dim, ncall, params) in enumerate(items):
            arr[i].family = int(family)
            arr[i].dim = int(dim)
            arr[i].ncall = int(ncall)
            if params is not None:
                for q, v in enumerate(list(params)[:2 * int(dim)]):
                    arr[i].params[q] = float(v)
        opt = options if options is not None else mcubes_default_options()
        h = _vp()
        _check(lib().mcubes_batch_create(arr, int(n), int(seed) & (2**64 - 1), ctypes.byref(opt),
                                         ctypes.byref(h)))
        self.handle = h
        self.n = n
        self.dims = [int(it[1]) for it in items]
        self.nbins = opt.nbins

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.mcubes_batch_destroy(self.handle)
            self.handle = None

    def destroy(self):
        if self.handle:
            lib().mcubes_batch_destroy(self.handle)
            self.handle = None

    def info(self):
        info = mcubes_batch_info()
        _check(lib().mcubes_batch_get_info(self.handle, ctypes.byref(info)))
        return {f: getattr(info, f) for f, _ in mcubes_batch_info._fields_}

    def classes(self):
        out = []
        for k in range(self.info()["classes"]):
            c = mcubes_batch_class()
            _check(lib().mcubes_batch_get_class(self.handle, k, ctypes.byref(c)))
            out.append({f: getattr(c, f) for f, _ in mcubes_batch_class._fields_})
        return out

    def configure_class(self, k, block_size, shares):
        _check(lib().mcubes_batch_configure_class(self.handle, int(k), int(block_size),
                                                  int(shares)))

    def autotune(self):
        _check(lib().mcubes_batch_autotune(self.handle))

    def set_streams(self, streams):
        _check(lib().mcubes_batch_set_streams(self.handle, int(streams)))

    def step(self, iteration, grids):
        """One iteration from the given grids (one dim x (nbins+1) array-like
        per integrand) -> (list of (I_t, var_t), list of refined grids)."""
        import numpy as np
        nb1 = self.nbins + 1
        rows = []
        for i, (g, d) in enumerate(zip(grids, self.dims)):
            a = np.asarray(g, dtype=np.float64)
            if a.shape != (d, nb1):
                raise ValueError(f"grid {i} must have shape {(d, nb1)}, got {a.shape}")
            rows.append(a.ravel())
        if len(rows) != self.n:
            raise ValueError(f"{self.n} grids needed, got {len(rows)}")
        buf = np.ascontiguousarray(np.concatenate(rows))
        est = np.zeros(2 * self.n)
        _check(lib().mcubes_batch_step(self.handle, int(iteration), buf.ctypes.data_as(_dp),
                                       est.ctypes.data_as(_dp)))
        out_grids, off = [], 0
        for d in self.dims:
            out_grids.append(buf[off:off + d * nb1].reshape(d, nb1).copy())
            off += d * nb1
        return [(float(est[2 * i]), float(est[2 * i + 1])) for i in range(self.n)], out_grids

    def integrate(self, itmax, rel_tol, use_graph=True, grids=False, traces=False):
        """Runs the batch; returns (status, list of per-integrand dicts).  Each
        dict holds the mcubes_result fields, plus 'grid' (dim rows) and
        'trace_I' / 'trace_var' when asked for."""
        n = self.n
        res = (mcubes_result * n)()
        glen = self.info()["grids_len"]
        g_buf = (ctypes.c_double * glen)() if grids else None
        t_buf = (ctypes.c_double * (n * 2 * itmax))() if traces else None
        rc = lib().mcubes_batch_integrate(self.handle, int(itmax), float(rel_tol),
                                          1 if use_graph else 0, res,
                                          ctypes.cast(g_buf, _dp) if grids else None,
                                          ctypes.cast(t_buf, _dp) if traces else None)
        _check(rc, allow=(MCUBES_OK, MCUBES_NOT_CONVERGED, MCUBES_E_NONFINITE))
        out = []
        off = 0
        nb1 = self.nbins + 1
        for i in range(n):
            r = {f: getattr(res[i], f) for f, _ in mcubes_result._fields_}
            r["converged"] = bool(r["converged"])
            d = self.dims[i]
            if grids:
                r["grid"] = [list(g_buf[off + j * nb1:off + (j + 1) * nb1]) for j in range(d)]
            off += d * nb1
            if traces:
                it = r["iterations"]
                row = t_buf[i * 2 * itmax:(i + 1) * 2 * itmax]
                r["trace_I"] = [row[2 * t] for t in range(it)]
                r["trace_var"] = [row[2 * t + 1] for t in range(it)]
            out.append(r)
        return rc, out


class Flow:
    """Owns an mcubes_flow* (the learned proposal); destroyed with the object.
    theta: MCUBES_FLOW_PARAMS initial parameters (host)."""

    def __init__(self, theta):
        arr = (ctypes.c_double * MCUBES_FLOW_PARAMS)(*[float(v) for v in theta])
        h = _vp()
        _check(lib().mcubes_flow_create(arr, ctypes.byref(h)))
        self.handle = h

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.mcubes_flow_destroy(self.handle)
            self.handle = None

    def params(self):
        buf = (ctypes.c_double * MCUBES_FLOW_PARAMS)()
        _check(lib().mcubes_flow_get_params(self.handle, buf))
        return list(buf)

    def set_params(self, theta):
        arr = (ctypes.c_double * MCUBES_FLOW_PARAMS)(*[float(v) for v in theta])
        _check(lib().mcubes_flow_set_params(self.handle, arr))

    def density(self, d_x, n, d_z, d_logq, precision=MCUBES_FP32, stream=None):
        _check(lib().mcubes_flow_density(self.handle, int(precision), _dev(d_x, 6 * n, "x"),
                                         int(n), _dev(d_z, 6 * n, "z"),
                                         _dev(d_logq, n, "logq"), _stream(stream)))

    def sample(self, d_z, n, d_x, d_logq, precision=MCUBES_FP32, stream=None):
        _check(lib().mcubes_flow_sample(self.handle, int(precision), _dev(d_z, 6 * n, "z"),
                                        int(n), _dev(d_x, 6 * n, "x"),
                                        _dev(d_logq, n, "logq"), _stream(stream)))

    def loss_grad(self, d_x, d_w, n, d_grad, d_loss, stream=None, precision=MCUBES_FP32):
        _check(lib().mcubes_flow_loss_grad(self.handle, int(precision), _dev(d_x, 6 * n, "x"),
                                           _dev(d_w, n, "w"), int(n),
                                           _dev(d_grad, MCUBES_FLOW_PARAMS, "grad")
                                           if d_grad is not None else None,
                                           _dev(d_loss, 1, "loss"), _stream(stream)))

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check(lib().mcubes_flow_adam_step(self.handle, float(lr), float(beta1), float(beta2),
                                           float(eps), _stream(stream)))

    def train(self, d_x, d_w, n, epochs, batch, lr, stream=None, precision=MCUBES_BF16):
        losses = (ctypes.c_double * max(int(epochs), 1))()
        _check(lib().mcubes_flow_train(self.handle, int(precision), _dev(d_x, 6 * n, "x"),
                                       _dev(d_w, n, "w"), int(n), int(epochs), int(batch),
                                       float(lr), losses, _stream(stream)))
        return list(losses)[:int(epochs)]

    def draw(self, plan, iteration, n, d_x, d_w, stream=None, precision=MCUBES_BF16):
        _check(lib().mcubes_flow_draw(self.handle, int(precision), plan.handle, int(iteration),
                                      int(n), _dev(d_x, 6 * n, "x"), _dev(d_w, n, "w"),
                                      _stream(stream)))

    def integrate(self, family, params, ncall, itmax, rel_tol, seed, options=None, **flow_opts):
        """The whole learned-proposal pipeline (mcubes_flow_integrate) ->
        (result dict, report dict)."""
        keep, pp = _params(params, MCUBES_FLOW_DIM)
        fo = mcubes_flow_options()
        lib().mcubes_default_flow_options(ctypes.byref(fo))
        for k, v in flow_opts.items():
            setattr(fo, k, v)
        opt = options if options is not None else mcubes_default_options()
        res = mcubes_result()
        rep = mcubes_flow_report()
        rc = lib().mcubes_flow_integrate(self.handle, int(family), pp, int(ncall), int(itmax),
                                         float(rel_tol), int(seed) & (2**64 - 1),
                                         ctypes.byref(opt), ctypes.byref(fo), ctypes.byref(res),
                                         ctypes.byref(rep))
        _check(rc, allow=(MCUBES_OK, MCUBES_NOT_CONVERGED))
        out = {f: getattr(res, f) for f, _ in mcubes_result._fields_}
        out["converged"] = bool(out["converged"])
        return out, {f: getattr(rep, f) for f, _ in mcubes_flow_report._fields_}

    def weight_tail(self):
        """(shape, tail count) of the last flow iteration's weights."""
        shape = ctypes.c_double()
        k = ctypes.c_int64()
        _check(lib().mcubes_flow_weight_tail(self.handle, ctypes.byref(shape), ctypes.byref(k)))
        return shape.value, k.value

    def vsample(self, plan, iteration, d_est, precision=MCUBES_FP32, stream=None):
        _check(lib().mcubes_flow_vsample(self.handle, int(precision), plan.handle,
                                         int(iteration), _dev(d_est, 2, "est"),
                                         _stream(stream)))


MCUBES_WTAIL_BINS = 4096


def mcubes_weight_tail_shape(hist):
    """(shape, tail count) of a MCUBES_WTAIL_BINS-bin log2 weight histogram
    (host only; shape is NaN below 100 counted weights)."""
    import numpy as np
    h = np.ascontiguousarray(hist, dtype=np.uint32)
    if h.shape != (MCUBES_WTAIL_BINS,):
        raise ValueError(f"the histogram needs {MCUBES_WTAIL_BINS} bins")
    shape = ctypes.c_double()
    k = ctypes.c_int64()
    _check(lib().mcubes_weight_tail_shape(h.ctypes.data_as(_vp), ctypes.byref(shape),
                                          ctypes.byref(k)))
    return shape.value, k.value


def mcubes_vsample_dump(plan, iteration, d_grid, w_begin, count, d_x, d_w, stream=None):
    i = plan.info
    rows = count * i["samples_per_cube"]
    _check(lib().mcubes_vsample_dump(plan.handle, int(iteration),
                                     _dev(d_grid, i["grid_len"], "grid"), int(w_begin),
                                     int(count), _dev(d_x, rows * i["dim"], "x"),
                                     _dev(d_w, rows, "w"), _stream(stream)))
