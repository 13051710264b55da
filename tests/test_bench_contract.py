"""CPU checks of the benchmark's contract: it refuses more than one GPU
before touching any, reports the stored HBM traffic and VALU figures only
for the kernel sources they were measured on, and its per-sample work
models are the documented counts."""
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_is_refused(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_stored_profiles_follow_the_kernel_sources(monkeypatch):
    vals = bench._profile_values(bench.TRAFFIC_PROFILE)
    if vals is not None:
        # the committed profile was taken on these sources: it is reported
        assert bench.stored_traffic() > 0
    # on other sources neither figure is reported
    monkeypatch.setattr(bench, "source_digest", lambda: "0" * 64)
    assert bench.stored_traffic() is None
    assert bench.stored_valu_busy() is None


def test_fp64_work_per_sample():
    # 8-D Gaussian, p = 2: 10 per axis (80), 8 per sample, 6/p per cube (3),
    # integrand 4 per axis + negation + exp (34)
    assert bench.flops_per_sample(3, 8, 2) == 80 + 8 + 3 + 34
    # addition integrand in 1-D with p = 6: 10 + 8 + 1 + 1
    assert bench.flops_per_sample(6, 1, 6) == 20
    for fam in range(7):
        assert bench.flops_per_sample(fam, 9, 2) > bench.flops_per_sample(fam, 8, 2)


def test_flow_work_models():
    # one network: four layers of 96x64, 64x64 and 64x99 products, 2 flops each
    assert bench.FLOW_GEMM_FLOPS == 132608
    assert bench.FLOW_TRAIN_FLOPS == 3 * 132608
    # per layer: writes 878 B, reads back 168 B, weight-gradient reads 978 B
    assert bench.FLOW_TRAIN_BYTES == 4 * (878 + 168 + 978)
