"""The C interface: libmcubes.so loads, exports every function declared in
include/mcubes.h, the Python binding's structs match the C layout, and the
host-side logic (plan sizes, argument validation) behaves -- no GPU needed,
no kernel is launched."""
import ctypes
import os
import re
import subprocess

import pytest

import oracle
import paper_2302_05730_amd as mc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mcubes.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mcubes_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 14
    L = mc.lib()
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", mc.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (mcubes_\w+)", out))
    assert set(names) <= exported
    assert set(names) == set(mc._SIGNATURES)


_LAYOUT = r"""
#include <stddef.h>
#include <stdio.h>
#include "mcubes.h"
#define F(T, m) printf(#T " " #m " %zu\n", offsetof(T, m));
int main(void) {
    printf("mcubes_options size %zu\n", sizeof(mcubes_options));
    F(mcubes_options, nbins) F(mcubes_options, alpha) F(mcubes_options, stream)
    F(mcubes_options, stream_id) F(mcubes_options, precision)
    printf("mcubes_result size %zu\n", sizeof(mcubes_result));
    F(mcubes_result, chi2_dof) F(mcubes_result, status) F(mcubes_result, cube_side)
    F(mcubes_result, kernel_ms)
    printf("mcubes_plan_info size %zu\n", sizeof(mcubes_plan_info));
    F(mcubes_plan_info, lds_bytes) F(mcubes_plan_info, cube_side) F(mcubes_plan_info, state_len)
    F(mcubes_plan_info, precision)
    printf("mcubes_batch_item size %zu\n", sizeof(mcubes_batch_item));
    F(mcubes_batch_item, ncall) F(mcubes_batch_item, params)
    printf("mcubes_batch_info size %zu\n", sizeof(mcubes_batch_info));
    F(mcubes_batch_info, grids_len) F(mcubes_batch_info, last_iterations)
    F(mcubes_batch_info, streams) F(mcubes_batch_info, precision)
    F(mcubes_batch_info, last_samples) F(mcubes_batch_info, last_ms)
    printf("mcubes_batch_class size %zu\n", sizeof(mcubes_batch_class));
    F(mcubes_batch_class, shares) F(mcubes_batch_class, samples) F(mcubes_batch_class, tuned_ms)
    F(mcubes_batch_class, default_ms)
    printf("mcubes_flow_options size %zu\n", sizeof(mcubes_flow_options));
    F(mcubes_flow_options, train_items) F(mcubes_flow_options, tail_rounds) F(mcubes_flow_options, batch) F(mcubes_flow_options, round_lr) F(mcubes_flow_options, tail_lr) F(mcubes_flow_options, train_precision) F(mcubes_flow_options, anchor_rounds) F(mcubes_flow_options, min_iters)
    printf("mcubes_flow_report size %zu\n", sizeof(mcubes_flow_report));
    F(mcubes_flow_report, final_loss) F(mcubes_flow_report, used_flow)
    F(mcubes_flow_report, tail_shape)
    printf("MCUBES_STATE_LEN x %d\n", MCUBES_STATE_LEN);
    return 0;
}
"""


def test_struct_layouts_match_binding(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(_LAYOUT)
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", f"-I{os.path.join(ROOT, 'include')}", str(src), "-o",
                    str(exe)], check=True)
    lines = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    for line in filter(None, lines):
        tname, field, val = line.split()
        if tname == "MCUBES_STATE_LEN":
            assert int(val) == mc.MCUBES_STATE_LEN
            continue
        T = getattr(mc, tname)
        if field == "size":
            assert ctypes.sizeof(T) == int(val), tname
        else:
            assert getattr(T, field).offset == int(val), (tname, field)


@pytest.mark.parametrize("dim", [1, 2, 3, 5, 8, 10])
@pytest.mark.parametrize("ncall", [2, 7, 1000, 100_000, 2**26, 2**30, 5 * 10**9])
def test_plan_sizes_match_oracle(dim, ncall):
    assert mc.mcubes_plan_sizes(dim, ncall) == oracle.plan(dim, ncall)


def test_plan_caps_strata_per_axis():
    # 1-D plans stop at MCUBES_MAX_SIDE = 2^20 strata (so c + u stays exact in
    # FP64) and put the rest of the budget into samples per cube
    assert mc.mcubes_plan_sizes(1, 2**21 + 1) == (2**20, 2**20, 2, 2**21)
    assert mc.mcubes_plan_sizes(1, 2**22 + 3) == (2**20, 2**20, 4, 2**22)
    assert mc.mcubes_plan_sizes(1, 2 * 2**32 + 4) == (2**20, 2**20, 8192, 2**33)


def _create(family=3, params=None, dim=2, ncall=1000, **opt):
    if params is None:
        params = [1.0] * (2 * dim)
    return mc.mcubes_plan_create(family, params, dim, ncall, 0, mc.mcubes_default_options(**opt))


@pytest.mark.parametrize("kwargs,code", [
    (dict(dim=0), mc.MCUBES_E_ARG),
    (dict(dim=11), mc.MCUBES_E_ARG),
    (dict(ncall=1), mc.MCUBES_E_ARG),
    (dict(family=8), mc.MCUBES_E_INTEGRAND),
    (dict(family=7, params=[0.0, 0.5, 0.3, 0.6]), mc.MCUBES_E_INTEGRAND),
    (dict(family=7, params=[0.1, 1.0, 0.3, 0.6]), mc.MCUBES_E_INTEGRAND),
    (dict(family=7, params=[0.1, -0.2, 0.3, 0.6]), mc.MCUBES_E_INTEGRAND),
    (dict(family=7, dim=1, params=[0.1, 0.3]), mc.MCUBES_E_INTEGRAND),
    (dict(family=-1), mc.MCUBES_E_INTEGRAND),
    (dict(params=[float("nan"), 1.0, 1.0, 1.0]), mc.MCUBES_E_INTEGRAND),
    (dict(params=[1.0, float("inf"), 1.0, 1.0]), mc.MCUBES_E_INTEGRAND),
    (dict(family=1, params=[0.0, 1.0, 0.5, 0.5]), mc.MCUBES_E_INTEGRAND),
    (dict(nbins=1), mc.MCUBES_E_ARG),
    (dict(nbins=501), mc.MCUBES_E_ARG),
    (dict(alpha=float("nan")), mc.MCUBES_E_ARG),
    (dict(skip=-1), mc.MCUBES_E_ARG),
    (dict(block_size=100), mc.MCUBES_E_ARG),
    (dict(block_size=2048), mc.MCUBES_E_ARG),
    (dict(precision=2), mc.MCUBES_E_ARG),
    (dict(dim=2, ncall=2 * 2**32 + 4), mc.MCUBES_E_ARG),  # m = 2^32 cubes
])
def test_plan_create_rejects(kwargs, code):
    with pytest.raises(mc.MCubesError) as ei:
        _create(**kwargs)
    assert ei.value.code == code
    assert mc.mcubes_last_error()


@pytest.mark.parametrize("fn", ["mcubes_integrate", "mcubes_integrate_noalloc"])
def test_integrate_rejects_bad_arguments(fn):
    for itmax, tol in ((0, 0.1), (2000, 0.1), (3, float("nan")), (3, -1.0)):
        with pytest.raises(mc.MCubesError) as ei:
            getattr(mc, fn)(3, [1.0, 0.5], 1, 1000, itmax, tol, 0)
        assert ei.value.code == mc.MCUBES_E_ARG


def test_default_options():
    o = mc.mcubes_default_options()
    assert (o.nbins, o.adapt_iters, o.skip, o.block_size, o.blocks, o.alpha, o.precision) == \
        (500, -1, 0, 0, 0, 1.5, mc.MCUBES_FP64)
    assert not o.stream


_GOOD = (3, 2, 1000, [1.0, 1.0, 0.5, 0.5])


@pytest.mark.parametrize("items,opt,code", [
    ([], {}, mc.MCUBES_E_ARG),
    ([_GOOD, (9, 2, 1000, [1.0] * 4)], {}, mc.MCUBES_E_INTEGRAND),
    ([_GOOD, (3, 0, 1000, None)], {}, mc.MCUBES_E_ARG),
    ([_GOOD, (3, 11, 1000, None)], {}, mc.MCUBES_E_ARG),
    ([(3, 2, 1, [1.0] * 4)], {}, mc.MCUBES_E_ARG),
    ([_GOOD, _GOOD, (1, 2, 1000, [0.0, 1.0, 0.5, 0.5])], {}, mc.MCUBES_E_INTEGRAND),
    ([(0, 2, 1000, [float("nan"), 1.0, 0.5, 0.5])], {}, mc.MCUBES_E_INTEGRAND),
    ([(3, 2, 2 * 2**32 + 4, [1.0, 1.0, 0.5, 0.5])], {}, mc.MCUBES_E_ARG),
    ([_GOOD], dict(precision=mc.MCUBES_BF16), mc.MCUBES_E_ARG),
    ([_GOOD], dict(nbins=501), mc.MCUBES_E_ARG),
    ([_GOOD], dict(block_size=96), mc.MCUBES_E_ARG),
    ([_GOOD], dict(skip=-2), mc.MCUBES_E_ARG),
])
def test_batch_create_rejects(items, opt, code):
    """Every item is validated on the host before the device is touched; the
    message names the offending item."""
    with pytest.raises(mc.MCubesError) as ei:
        mc.Batch(items, 0, mc.mcubes_default_options(**opt))
    assert ei.value.code == code
    msg = mc.mcubes_last_error()
    if len(items) > 1:
        assert f"item {len(items) - 1}" in msg, msg


def test_flow_entry_points_reject_bad_arguments():
    """Checks that return before any device work: NULL objects and buffers,
    non-finite parameters, unknown precisions."""
    L = mc.lib()
    E = mc.MCUBES_E_ARG
    out = ctypes.c_void_p()
    assert L.mcubes_flow_create(None, ctypes.byref(out)) == E
    theta = (ctypes.c_double * mc.MCUBES_FLOW_PARAMS)()
    theta[5] = float("nan")
    assert L.mcubes_flow_create(theta, ctypes.byref(out)) == E
    assert L.mcubes_flow_train(None, mc.MCUBES_BF16, None, None, 10, 1, 16, 1e-3, None, None) == E
    assert L.mcubes_flow_loss_grad(None, mc.MCUBES_FP32, None, None, 10, None, None, None) == E
    assert L.mcubes_flow_draw(None, mc.MCUBES_BF16, None, 0, 10, None, None, None) == E
    assert L.mcubes_flow_vsample(None, mc.MCUBES_BF16, None, 0, None, None) == E
    assert L.mcubes_flow_density(None, mc.MCUBES_FP32, None, 1, None, None, None) == E
    assert L.mcubes_flow_sample(None, mc.MCUBES_FP32, None, 1, None, None, None) == E
    assert L.mcubes_flow_weight_tail(None, None, None) == E
    # (host buffers stand in for device ones: the checks fail before any use)
    est = (ctypes.c_double * 2)()
    state = (ctypes.c_double * mc.MCUBES_STATE_LEN)()
    assert L.mcubes_flow_combine(0, None, state, 0.0, 1, None) == E
    assert L.mcubes_flow_combine(0, est, None, 0.0, 1, None) == E
    assert L.mcubes_flow_combine(mc.MCUBES_MAX_ITERATIONS, est, state, 0.0, 1, None) == E
    assert L.mcubes_flow_combine(0, est, state, -1.0, 1, None) == E
    assert L.mcubes_flow_combine(0, est, state, float("nan"), 1, None) == E
    assert L.mcubes_flow_combine(0, est, state, 0.0, 0, None) == E
    xs = (ctypes.c_double * 24)()
    ws = (ctypes.c_double * 4)()
    xo = (ctypes.c_double * 24)()
    wo = (ctypes.c_double * 4)()
    assert L.mcubes_flow_shuffle(xs, ws, -1, xo, wo, None) == E
    assert L.mcubes_flow_shuffle(xs, ws, 1 << 32, xo, wo, None) == E
    assert L.mcubes_flow_shuffle(None, ws, 4, xo, wo, None) == E
    assert L.mcubes_flow_shuffle(xs, ws, 4, xs, wo, None) == E  # output on its input
    assert L.mcubes_flow_shuffle(xs, ws, 4, xo, xo, None) == E  # outputs overlap
    assert L.mcubes_flow_shuffle(xs, ws, 0, xo, wo, None) == mc.MCUBES_OK  # nothing to do
    assert L.mcubes_weight_tail_shape(None, None, None) == E
    res = mc.mcubes_result()
    assert L.mcubes_flow_integrate(None, mc.MCUBES_MIXTURE, None,
                                   1 << 20, 4, 0.0, 1, None, None, ctypes.byref(res),
                                   None) == E
    assert L.mcubes_last_error()


def test_default_flow_options():
    fo = mc.mcubes_flow_options()
    mc.lib().mcubes_default_flow_options(ctypes.byref(fo))
    assert (fo.warmup_iters, fo.train_items, fo.epochs, fo.rounds, fo.round_samples,
            fo.round_epochs, fo.tail_rounds, fo.batch) == (8, 1 << 20, 10, 4, 1 << 25, 2, 4,
                                                           65536)
    assert (fo.lr, fo.round_lr, fo.tail_power, fo.tail_lr) == (4e-3, 2e-3, 1.75, 8e-4)
    assert fo.precision == mc.MCUBES_BF16 and fo.train_precision == mc.MCUBES_BF16
    assert fo.anchor_rounds == 2 and fo.min_iters == 4
