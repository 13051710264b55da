"""One signature table for the boundary calls that both libraries export:
libmcubes.so (the HIP path) as mcubes_<name> and liboracle.so (the CPU
reference) as mcubes_oracle_<name>.  The option and result records are
declared here with the field order of include/mcubes.h; both libraries'
own declarations are checked against that layout by a compiled probe
(test_abi_mirror.py).  Tests load both libraries through this table and
call them identically."""
import ctypes

import numpy as np


class Options(ctypes.Structure):
    _fields_ = [("nbins", ctypes.c_int32), ("adapt_iters", ctypes.c_int32),
                ("skip", ctypes.c_int32), ("block_size", ctypes.c_int32),
                ("blocks", ctypes.c_int32), ("stream_id", ctypes.c_uint32),
                ("precision", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("stream", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("estimate", ctypes.c_double), ("error", ctypes.c_double),
                ("chi2_dof", ctypes.c_double), ("iterations", ctypes.c_int32),
                ("dof", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("status", ctypes.c_int32), ("cube_side", ctypes.c_int64),
                ("ncubes", ctypes.c_int64), ("samples_per_cube", ctypes.c_int64),
                ("samples_per_iter", ctypes.c_int64), ("kernel_ms", ctypes.c_double)]


_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p

# name (after the prefix) -> (restype, argtypes)
TABLE = {
    "integrate": (ctypes.c_int, [ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_uint64, ctypes.POINTER(Options),
                                 ctypes.POINTER(Result), _dp, _dp]),
    "plan_create": (ctypes.c_int, [ctypes.c_int, _dp, ctypes.c_int, ctypes.c_int64,
                                   ctypes.c_uint64, ctypes.POINTER(Options),
                                   ctypes.POINTER(_vp)]),
    "plan_destroy": (None, [_vp]),
    "iterate": (ctypes.c_int, [_vp, _dp, ctypes.c_uint32, _dp, _dp, _dp, _dp]),
}

PREFIX = {"gpu": "mcubes_", "oracle": "mcubes_oracle_"}


class Side:
    """The four calls of one library, bound through TABLE."""

    def __init__(self, path, prefix):
        self.lib = ctypes.CDLL(path)
        self.fn = {}
        for name, (res, args) in TABLE.items():
            f = getattr(self.lib, prefix + name)
            f.restype = res
            f.argtypes = args
            self.fn[name] = f

    def integrate(self, family, params, dim, ncall, itmax, rel_tol, seed, opt):
        p = None if params is None else np.ascontiguousarray(params, dtype=np.float64)
        res = Result()
        grid = np.zeros(max(dim, 1) * (max(opt.nbins, 1) + 1))
        trace = np.zeros(2 * max(itmax, 1))
        rc = self.fn["integrate"](int(family), p.ctypes.data_as(_dp) if p is not None else None,
                                  int(dim), int(ncall), int(itmax), float(rel_tol), int(seed),
                                  ctypes.byref(opt), ctypes.byref(res), grid.ctypes.data_as(_dp),
                                  trace.ctypes.data_as(_dp))
        return rc, res, grid.reshape(max(dim, 1), -1), trace.reshape(-1, 2)[:max(res.iterations, 0)]

    def plan(self, family, params, dim, ncall, seed, opt):
        p = None if params is None else np.ascontiguousarray(params, dtype=np.float64)
        h = _vp()
        rc = self.fn["plan_create"](int(family), p.ctypes.data_as(_dp) if p is not None else None,
                                    int(dim), int(ncall), int(seed), ctypes.byref(opt),
                                    ctypes.byref(h))
        return rc, h

    def destroy(self, h):
        self.fn["plan_destroy"](h)

    def iterate(self, h, grid_in, iteration, dim, nb):
        g = np.ascontiguousarray(grid_in, dtype=np.float64).reshape(-1)
        I, v = ctypes.c_double(), ctypes.c_double()
        bins = np.zeros(dim * nb)
        out = np.zeros(dim * (nb + 1))
        rc = self.fn["iterate"](h, g.ctypes.data_as(_dp), int(iteration), ctypes.byref(I),
                                ctypes.byref(v), bins.ctypes.data_as(_dp),
                                out.ctypes.data_as(_dp))
        return rc, I.value, v.value, bins.reshape(dim, nb), out.reshape(dim, nb + 1)


def options(nbins=500, adapt_iters=-1, skip=0, alpha=1.5, stream_id=0):
    o = Options()
    o.nbins, o.adapt_iters, o.skip, o.alpha, o.stream_id = nbins, adapt_iters, skip, alpha, stream_id
    return o
