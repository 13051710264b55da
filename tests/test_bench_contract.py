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


def test_digest_sees_code_not_comments():
    """The digest that ties a stored profile to the kernel sources ignores
    comments and blank lines, and nothing else."""
    code = "int f(int a) {\n    return a + 1;  // one more\n}\n"
    assert bench._code_only(code) == bench._code_only(
        "/* helper */\nint f(int a) {\n\n    return a + 1;\n}\n// end\n")
    assert bench._code_only(code) != bench._code_only(code.replace("a + 1", "a + 2"))
    assert bench._code_only("x = 1; /* a\n b */ y = 2;") == "x = 1;  y = 2;"


def test_fp64_work_per_sample():
    # 9 d + 7 + F_f: 8-D Gaussian 72 + 7 + (32 + exp) = 112, oscillatory
    # 72 + 7 + (16 + 2 + cos) = 98, corner peak 72 + 7 + (16 + 1 + 8 + 1) = 105
    assert bench.flops_per_sample(3, 8) == 112
    assert bench.flops_per_sample(0, 8) == 98
    assert bench.flops_per_sample(2, 8) == 105
    # addition integrand in 1-D: 9 + 7 + 1
    assert bench.flops_per_sample(6, 1) == 17
    for fam in range(8):
        assert bench.flops_per_sample(fam, 9) > bench.flops_per_sample(fam, 8)
        assert bench.flops_per_sample(fam, 8, 2) == bench.flops_per_sample(fam, 8, 7)
    # every FP64 operation the kernel issues: 10 per axis, 8 per sample, 6/p per
    # cube, and the integrand as evaluated (8-D Gaussian, p = 2: 80 + 8 + 3 + 34)
    assert bench.fp64_ops_per_sample(3, 8, 2) == 80 + 8 + 3 + 34
    assert bench.fp64_ops_per_sample(6, 1, 6) == 20


def test_closed_form_fixture_matches_the_workloads():
    # the stored exact integrals belong to the benchmark's parameters
    import workloads
    cf = bench.closed_forms()
    for pr in workloads.large_8d_set():
        assert cf[pr.name]["params"] == pr.params and cf[pr.name]["family"] == pr.family
    for k in range(1, 7):
        fam, params = workloads.paper_integrand(k, 8)
        assert cf[f"paper_f{k}_8d"]["params"] == params
    assert abs(cf["mixture_6d"]["integral"] - 1.0) < 1e-9
    assert cf["paper_sum_8d"]["integral"] == 4.0


def test_host_cpu_description():
    c = bench.host_cpu()
    assert c["logical_cpus"] >= 1 and 1 <= c["usable_cpus"] <= c["logical_cpus"]


def test_flow_work_models():
    # one network: four layers of 96x64, 64x64 and 64x99 products, 2 flops each
    assert bench.FLOW_GEMM_FLOPS == 132608
    assert bench.FLOW_TRAIN_FLOPS == 3 * 132608
    # per layer: writes 878 B, reads back 168 B, weight-gradient reads 978 B
    assert bench.FLOW_TRAIN_BYTES == 4 * (878 + 168 + 978)
