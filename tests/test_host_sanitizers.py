"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The batched form's bookkeeping (paper_2302_05730_amd/csrc/batch_plan.h: the
  split of classes into tiles, the per-integrand partial ranges, the share
  counts and the spread of classes over streams) is compiled, HIP-free, into
  tests/batch_plan_check.cpp and driven through the convergence schedule of
  a 20-integrand batch -- a new plan whenever 2% of the planned samples have
  finished, as the re-splitting runtime did -- and through random schedules;
  every plan is checked for exact coverage of the running integrands' work.
* The oracle's C sources are compiled with tests/oracle_sanitize_check.c,
  which calls every public function on small and degenerate inputs.
"""
import os
import shutil
import subprocess

import pytest

import oracle
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2302_05730_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")


def _compile(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]


def _run(exe, stdin):
    r = subprocess.run([exe], input=stdin, capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0 and r.stdout.startswith("ok"), (r.stdout[-2000:], r.stderr[-6000:])
    return r.stdout


@pytest.fixture(scope="module")
def plan_check(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("san") / "batch_plan_check")
    _compile(["g++", "-std=c++17", *SAN, f"-I{CSRC}",
              os.path.join(ROOT, "tests", "batch_plan_check.cpp"), "-o", exe])
    return exe


def test_batch_plan_convergence_schedule(plan_check):
    """The 20-integrand batch whose integrands stop at different iterations
    (rel_tol 2e-3, 100 bins; stopping iterations from the oracle), planned on
    the device's geometry (4 streams, 1024 resident workgroups of 256) and
    on a small one."""
    probs = workloads.batch_problems(n=20, seed=13, ncall_lo=5e3, ncall_hi=5e4,
                                     families=(workloads.PRODUCT_PEAK, workloads.GAUSSIAN,
                                               workloads.C0, workloads.CORNER_PEAK),
                                     dims=(2, 3, 4, 5))
    lines = []
    stops = []
    for i, pr in enumerate(probs):
        r = oracle.integrate(pr.family, pr.params, pr.dim, pr.ncall, 12, 2e-3, 9, nb=100,
                             stream=i)
        stops.append(r["iterations"])
        lines.append(f"{pr.family} {pr.dim} {r['m']} {r['p']} {r['iterations']}")
    assert len(set(stops)) >= 3, stops  # the schedule really re-plans
    for geometry in ("4 1024 256", "3 16 64", "1 1 1024"):
        out = _run(plan_check, f"schedule {geometry} {len(probs)}\n" + "\n".join(lines) + "\n")
        assert int(out.split()[1]) >= 3  # several plans were built and checked


def test_batch_plan_random_schedules(plan_check):
    """Random batches (1-40 integrands, one-cube and tiny integrands, p up to
    31, 1-4 streams, 1-300 resident workgroups, workgroups of 64-1024)."""
    for seed in (1, 2, 3):
        _run(plan_check, f"fuzz {seed} 40\n")


def test_oracle_under_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_check")
    srcs = [os.path.join(ROOT, "oracle", f) for f in
            ("mcubes_oracle.c", "mcubes_oracle_abi.c", "flow_oracle.c")]
    _compile(["gcc", "-std=gnu11", "-ffp-contract=off", *SAN, f"-I{os.path.join(ROOT, 'oracle')}",
              *srcs, os.path.join(ROOT, "tests", "oracle_sanitize_check.c"), "-o", exe, "-lm"])
    _run(exe, "")
