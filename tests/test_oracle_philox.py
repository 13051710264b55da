"""Pins of the oracle's counter-based generator (Philox4x32-10, SC'11).

The oracle's Philox is checked bit for bit against an independent
implementation, rocRAND's Philox4x32-10 engine, whose ten-round bijection is
compiled for the host from the installed ROCm header (no GPU needed).  The
uniform conversion is checked against its exact definition and the stream
against basic distribution properties.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import stats

import oracle

ROCRAND_HEADER = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"

_PROBE = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
struct Exposed : rocrand_device::philox4x32_10_engine {
    static uint4 run(uint4 c, uint2 k) { Exposed e; return e.ten_rounds(c, k); }
};
int main() {
    unsigned a, b, c, d, k0, k1;
    while (std::scanf("%u %u %u %u %u %u", &a, &b, &c, &d, &k0, &k1) == 6) {
        uint4 o = Exposed::run(make_uint4(a, b, c, d), make_uint2(k0, k1));
        std::printf("%u %u %u %u\n", o.x, o.y, o.z, o.w);
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def rocrand_probe(tmp_path_factory):
    if not os.path.exists(ROCRAND_HEADER) or shutil.which("g++") is None:
        pytest.skip("rocRAND header or g++ not available")
    d = tmp_path_factory.mktemp("rocrand")
    src = d / "probe.cpp"
    src.write_text(_PROBE)
    exe = d / "probe"
    subprocess.run(["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    str(src), "-o", str(exe)], check=True)
    return str(exe)


def test_philox_matches_rocrand(rocrand_probe):
    rng = np.random.default_rng(123)
    cases = rng.integers(0, 2**32, size=(2000, 6), dtype=np.uint64)
    # include structured counters like the ones the integrator uses
    cases[:16] = [[c, 0, k, t, 0, 0] for c in range(4) for k, t in ((0, 0), (1, 0), (0, 1), (3, 7))]
    cases[16:20] = [[2**32 - 1] * 6, [0] * 6, [0, 0, 0, 0, 2**32 - 1, 2**32 - 1], [1, 1, 1, 1, 1, 1]]
    inp = "\n".join(" ".join(str(int(v)) for v in row) for row in cases) + "\n"
    out = subprocess.run([rocrand_probe], input=inp, capture_output=True, text=True, check=True)
    ref = [list(map(int, line.split())) for line in out.stdout.strip().splitlines()]
    assert len(ref) == len(cases)
    for row, expect in zip(cases, ref):
        got = oracle.philox4x32_10(row[:4], row[4:])
        assert got == expect, (row, got, expect)


def test_uniform_is_cell_midpoint():
    assert oracle.uniform(0) == 2.0**-33
    assert oracle.uniform(2**32 - 1) == 1.0 - 2.0**-33
    rng = np.random.default_rng(5)
    for r in rng.integers(0, 2**32, size=200):
        assert oracle.uniform(int(r)) == (int(r) + 0.5) / 2.0**32  # exact in FP64


def test_philox_avalanche():
    """Flipping one input bit flips about half of the 128 output bits."""
    rng = np.random.default_rng(9)
    flips = []
    for _ in range(200):
        ctr = [int(v) for v in rng.integers(0, 2**32, size=4)]
        key = [int(v) for v in rng.integers(0, 2**32, size=2)]
        base = oracle.philox4x32_10(ctr, key)
        word, bit = int(rng.integers(0, 6)), int(rng.integers(0, 32))
        c2, k2 = list(ctr), list(key)
        if word < 4:
            c2[word] ^= 1 << bit
        else:
            k2[word - 4] ^= 1 << bit
        other = oracle.philox4x32_10(c2, k2)
        flips.append(sum(bin(a ^ b).count("1") for a, b in zip(base, other)))
    assert 60 < np.mean(flips) < 68


def test_uniform_stream_distribution():
    """The uniforms of consecutive counters: mean 1/2, variance 1/12, KS test."""
    u = []
    for c in range(5000):
        for w in oracle.philox4x32_10([c, 0, 0, 3], [17, 0]):
            u.append(oracle.uniform(w))
    u = np.array(u)
    assert abs(u.mean() - 0.5) < 4 * np.sqrt(1 / 12 / len(u))
    assert abs(u.var() - 1 / 12) < 0.004
    assert stats.kstest(u, "uniform").pvalue > 1e-3
