"""Microbenchmarks that attribute the V-Sample time (run on the GPU):

    python -m paper_2302_05730_amd.microbench

Prints one JSON line per measurement: the integrand-only throughput of the
paper's benchmark integrands f1-f6 and the addition integrand at 5-8-D (the
analogue of the integrand-invocation experiment of §5.1: every thread
evaluates the integrand serially on points prepared on the host), the Philox
throughput per sample, and FP64/FP32 exp, cos and pow.
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

BLOCKS, BLOCK = 2048, 256  # 8 blocks of 256 per CU


def timed(fn, reps=3):
    import torch
    s = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        fn()
        e1.record(s)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def main():
    import torch

    import paper_2302_05730_amd as mc
    import workloads

    torch.cuda.set_device(0)
    out = torch.empty(BLOCKS * BLOCK, dtype=torch.float64, device="cuda")
    threads = BLOCKS * BLOCK
    rng = np.random.default_rng(2023)
    names = {1: "f1", 2: "f2", 3: "f3", 4: "f4", 5: "f5", 6: "f6", 7: "addition"}
    for dim in (5, 6, 7, 8):
        npts = 256  # 16 KB at 8-D: L1-resident, so the kernel measures the integrand arithmetic
        pts = torch.from_numpy(rng.uniform(0, 1, (npts, dim))).cuda()
        for k in range(1, 8):
            fam, params = workloads.paper_integrand(k, dim)
            calls = 1024
            ms = timed(lambda: mc.mcubes_microbench(mc.MCUBES_MB_INTEGRAND, out, BLOCKS, BLOCK,
                                                    calls, fam, params, dim, pts, npts))
            print(json.dumps({"kind": "integrand", "integrand": names[k], "dim": dim,
                              "ms": round(ms, 4), "evals_per_s": threads * calls / (ms * 1e-3)}),
                  flush=True)
    for dim in (5, 8):
        calls = 1024
        ms = timed(lambda: mc.mcubes_microbench(mc.MCUBES_MB_PHILOX, out, BLOCKS, BLOCK, calls,
                                                dim=dim))
        print(json.dumps({"kind": "philox", "dim": dim, "ms": round(ms, 4),
                          "samples_per_s": threads * calls / (ms * 1e-3),
                          "philox_calls_per_sample": (dim + 3) // 4}), flush=True)
    for kind, name in ((mc.MCUBES_MB_EXP64, "exp_f64"), (mc.MCUBES_MB_COS64, "cos_f64"),
                       (mc.MCUBES_MB_POW64, "pow_f64"), (mc.MCUBES_MB_EXP32, "exp_f32"),
                       (mc.MCUBES_MB_COS32, "cos_f32"), (mc.MCUBES_MB_POW32, "pow_f32")):
        calls = 2048
        ms = timed(lambda: mc.mcubes_microbench(kind, out, BLOCKS, BLOCK, calls))
        print(json.dumps({"kind": "math", "function": name, "ms": round(ms, 4),
                          "calls_per_s": threads * calls / (ms * 1e-3)}), flush=True)


if __name__ == "__main__":
    main()
