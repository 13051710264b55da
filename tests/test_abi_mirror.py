"""The boundary calls exported twice, by the HIP library (mcubes_*) and by
the CPU reference (mcubes_oracle_*), with the same argument lists and the
same record layouts, so tests drive both through one signature table
(tests/abi_mirror.py).  CPU only: no kernel is launched; the library side
is called only where it rejects its arguments before touching a device."""
import os
import subprocess

import numpy as np
import pytest

import abi_mirror as am
import oracle
import paper_2302_05730_amd as mc
import workloads
from parity_util import random_grid

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_PROBE = r"""
#include <stddef.h>
#include <stdio.h>
#include HEADER
#define F(T, m) printf(#m " %zu %zu\n", offsetof(T, m), sizeof(((T *)0)->m));
int main(void) {
    printf("options %zu\n", sizeof(OPT));
    F(OPT, nbins) F(OPT, adapt_iters) F(OPT, skip) F(OPT, block_size) F(OPT, blocks)
    F(OPT, stream_id) F(OPT, precision) F(OPT, alpha) F(OPT, stream)
    printf("result %zu\n", sizeof(RES));
    F(RES, estimate) F(RES, error) F(RES, chi2_dof) F(RES, iterations) F(RES, dof)
    F(RES, converged) F(RES, status) F(RES, cube_side) F(RES, ncubes)
    F(RES, samples_per_cube) F(RES, samples_per_iter) F(RES, kernel_ms)
    return 0;
}
"""


def _layout(tmp_path, header, opt, res, tag):
    src = tmp_path / f"probe_{tag}.c"
    src.write_text(_PROBE)
    exe = tmp_path / f"probe_{tag}"
    subprocess.run(["gcc", "-std=gnu11", f'-DHEADER="{header}"', f"-DOPT={opt}", f"-DRES={res}",
                    str(src), "-o", str(exe)], check=True)
    return subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout


def test_records_have_one_layout(tmp_path):
    a = _layout(tmp_path, os.path.join(ROOT, "include", "mcubes.h"), "mcubes_options",
                "mcubes_result", "lib")
    b = _layout(tmp_path, os.path.join(ROOT, "oracle", "mcubes_oracle.h"), "mco_options",
                "mco_result", "oracle")
    assert a == b
    rows = dict(line.split(" ", 1) for line in a.strip().split("\n"))
    import ctypes
    assert int(rows["options"]) == ctypes.sizeof(am.Options)
    assert int(rows["result"]) == ctypes.sizeof(am.Result)
    for name, _ in am.Options._fields_:
        assert int(rows[name].split()[0]) == getattr(am.Options, name).offset, name
    for name, _ in am.Result._fields_:
        assert int(rows[name].split()[0]) == getattr(am.Result, name).offset, name


def test_both_libraries_export_the_table():
    oracle.lib()
    gpu = am.Side(mc.LIB_PATH, am.PREFIX["gpu"])
    ora = am.Side(oracle.LIB_PATH, am.PREFIX["oracle"])
    assert set(gpu.fn) == set(ora.fn) == set(am.TABLE)


_BAD = [  # (family, params, dim, ncall, itmax, rel_tol, nbins) -> one error each
    (1, "ok", 3, 10**5, 0, 1e-3, 100),       # itmax < 1
    (1, "ok", 3, 10**5, 5, -1.0, 100),       # rel_tol < 0
    (1, "ok", 3, 10**5, 5, float("nan"), 100),
    (1, "ok", 0, 10**5, 5, 1e-3, 100),       # dim < 1
    (1, "ok", 11, 10**5, 5, 1e-3, 100),      # dim > 10
    (1, "ok", 3, 1, 5, 1e-3, 100),           # ncall < 2
    (1, "ok", 3, 10**5, 5, 1e-3, 1),         # nbins < 2
    (1, "ok", 3, 10**5, 5, 1e-3, 501),       # nbins > 500
    (99, "ok", 3, 10**5, 5, 1e-3, 100),      # unknown family
    (1, "zero_a", 3, 10**5, 5, 1e-3, 100),   # product peak with a_i = 0
    (3, "nan", 3, 10**5, 5, 1e-3, 100),      # non-finite parameter
]


@pytest.mark.parametrize("case", _BAD)
def test_both_sides_reject_the_same_arguments(case):
    family, pk, dim, ncall, itmax, rel_tol, nb = case
    d = max(dim, 1)
    params = np.concatenate([np.full(d, 5.0), np.full(d, 0.5)])
    if pk == "zero_a":
        params[0] = 0.0
    if pk == "nan":
        params[d] = float("nan")
    oracle.lib()
    sides = [am.Side(mc.LIB_PATH, am.PREFIX["gpu"]), am.Side(oracle.LIB_PATH, am.PREFIX["oracle"])]
    codes = []
    for side in sides:
        rc, res, _, _ = side.integrate(family, params, dim, ncall, itmax, rel_tol, 0,
                                       am.options(nbins=nb))
        codes.append(rc)
    assert codes[0] == codes[1] and codes[0] < 0, codes


def test_oracle_integrate_entry_point_is_the_oracle():
    """mcubes_oracle_integrate returns what the oracle's own loop computes
    (3-D product peak, 10 iterations): same estimate, error, chi2, trace and
    final grid."""
    pr = workloads.small_product_peak()
    ora = am.Side(oracle.LIB_PATH, am.PREFIX["oracle"])
    rc, res, grid, trace = ora.integrate(pr.family, pr.params, pr.dim, pr.ncall, pr.itmax, 0.0,
                                         pr.seed, am.options(nbins=pr.nbins))
    ref = oracle.integrate(pr.family, pr.params, pr.dim, pr.ncall, pr.itmax, 0.0, pr.seed,
                           nb=pr.nbins)
    assert rc == 1 and res.status == 1 and res.iterations == pr.itmax  # rel_tol 0: never met
    assert (res.estimate, res.error, res.chi2_dof) == (ref["estimate"], ref["error"],
                                                       ref["chi2_dof"])
    assert (res.cube_side, res.ncubes, res.samples_per_cube) == (ref["g"], ref["m"], ref["p"])
    assert np.array_equal(trace[:, 0], ref["trace_I"]) and np.array_equal(trace[:, 1],
                                                                          ref["trace_var"])
    assert np.array_equal(grid, ref["grid"])


def test_oracle_iterate_entry_point_is_one_iteration():
    pr = workloads.small_product_peak()
    ora = am.Side(oracle.LIB_PATH, am.PREFIX["oracle"])
    rc, h = ora.plan(pr.family, pr.params, pr.dim, pr.ncall, pr.seed, am.options(nbins=pr.nbins))
    assert rc == 0
    try:
        grid = random_grid(np.random.default_rng(4), pr.dim, pr.nbins)
        rc, I, v, bins, new = ora.iterate(h, grid, 3, pr.dim, pr.nbins)
        assert rc == 0
        I_ref, v_ref, bins_ref = oracle.iteration(pr.family, pr.params, pr.dim, pr.nbins,
                                                  pr.ncall, pr.seed, 3, grid)
        assert (I, v) == (I_ref, v_ref)
        assert np.array_equal(bins, bins_ref)
        assert np.array_equal(new, oracle.refine(grid, bins_ref))
        bad = grid.copy()
        bad[0, 5] = bad[0, 7]  # not monotone
        bad[0, 6] = bad[0, 4]
        assert ora.iterate(h, bad, 3, pr.dim, pr.nbins)[0] == -1
    finally:
        ora.destroy(h)
