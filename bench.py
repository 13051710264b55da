"""Benchmark of the MI355X m-Cubes path on the 8-D Genz workload.

Workload: the 8-D Gaussian, oscillatory and corner-peak integrands with
a_i ~ U(5, 15), u_i ~ U(0, 1) (parameter seeds 1, 2, 3), 500 bins per axis,
2^30 samples requested per iteration (12^8 cubes x 2 samples = 859,963,392
evaluations), FP64 throughout.  One step = one whole iteration (V-Sample,
reduction, combination, refinement) of each of the three integrands, so a step
evaluates 3 x 859,963,392 samples.  Inputs (grids, parameters) are resident on
the GPU before the timed region starts.

Prints one JSON line.  Besides throughput it reports, for the V-Sample kernel,
the achieved FP64 rate against the vector peak (HIP events around every
launch), a CPU baseline (the single-threaded oracle on a bounded sample) and
the wall time to a 1e-3 relative error.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402

FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X: 256 CUs x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz


def flops_per_sample(family, d, p=2):
    """Algorithmic FP64 flops of one sample, 9 d + 7 + F_f (FMA = 2; exp, cos
    and a division count 1 each): per axis the uniform from the random word
    (fma: 2), the stratified coordinate (add, mul: 2) and the map through the
    grid (bin fraction, width, fma, Jacobian factor: 5); per sample the
    Jacobian scale, the weight, the cube statistics and w^2 (7); F_f the
    integrand:
      oscillatory 2 d + 2 + cos, product peak 3 d + d divisions, corner peak
      2 d + 1 + d (power chain) + 1 division, Gaussian 4 d + exp, C0 3 d + exp,
      discontinuous 2 d + exp, addition d, mixture 8 d + 12 (two quadratic
      forms, two exp).
    The count does not depend on p."""
    f = {0: 2 * d + 3, 1: 4 * d, 2: 3 * d + 2, 3: 4 * d + 1, 4: 3 * d + 1, 5: 2 * d + 1,
         6: d, 7: 8 * d + 12}[family]
    return 9 * d + 7 + f


def fp64_ops_per_sample(family, d, p):
    """Every FP64 operation the kernel issues for one sample, in the same units:
    per axis the uniform (2), stratum offset (1), bin coordinate (1), in-bin
    fraction (1), width (1), mapped point (2), Jacobian factor (1) and the
    bin update (1) -> 10 d; per sample the Jacobian scale, weight, cube sum,
    shift, the two shifted sums and w^2 -> 8; per cube the variance and two
    running sums -> 6/p; plus the integrand as evaluated (the product peak's
    divisions are folded into its coefficients)."""
    f = {0: 2 * d + 1, 1: 4 * d + 1, 2: 3 * d + 1, 3: 4 * d + 2, 4: 3 * d + 2, 5: 2 * d + 1,
         6: d, 7: 8 * d + 12}[family]
    return 10 * d + 8 + 6.0 / p + f


CLOSED_FORMS = os.path.join(ROOT, "tests", "golden", "bench_closed_forms.json")


def closed_forms():
    """Exact integrals of the benchmark integrands (a stored fixture written from
    the closed forms; see tests/golden/make_bench_closed_forms.py)."""
    with open(CLOSED_FORMS) as fh:
        return json.load(fh)


def host_cpu():
    """Model name of the host CPU and the logical CPUs this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def _code_only(text):
    """C/C++ source without its comments and blank lines (the part that
    decides what the compiler builds)."""
    import re
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.split("\n") if line.strip())


def source_digest():
    """SHA-256 over the code (comments dropped) of the sources that define the
    single-integrand V-Sample kernel and its launch (identifies the kernel
    build that a stored counter profile belongs to): the kernel template, its
    per-family instantiations, the shared declarations and the host code that
    sizes the launch."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2302_05730_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(csrc)):
        if (name in ("vsample_impl.h", "mcubes_internal.h", "mcubes_api.hip")
                or (name.startswith("vsample_f") and name.endswith(".hip"))):
            with open(os.path.join(csrc, name), encoding="utf-8") as fh:
                h.update(name.encode() + b"\0" + _code_only(fh.read()).encode())
    return h.hexdigest()


TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "vsample_8d_hbm_traffic.txt")
COUNTER_PROFILE = os.path.join(ROOT, "profiles", "vsample_8d_counters.txt")


def _profile_values(path):
    """key: value lines of a committed profile summary, or None when it is
    missing or was taken on different kernel sources."""
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith(("#", " ", "[")):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != source_digest():
        return None
    return vals


def stored_traffic():
    """HBM bytes per V-Sample launch from the committed FETCH_SIZE/WRITE_SIZE
    profile (None if it belongs to other kernel sources)."""
    vals = _profile_values(TRAFFIC_PROFILE)
    try:
        return float(vals["mean_bytes_per_launch"]) if vals else None
    except (KeyError, ValueError):
        return None


def stored_valu_busy():
    """Fraction of VALU issue cycles used, per family, from the committed
    counter profile (None if it belongs to other kernel sources)."""
    vals = _profile_values(COUNTER_PROFILE)
    if not vals:
        return None
    return {k[len("valu_busy_"):]: float(v) for k, v in vals.items() if k.startswith("valu_busy_")}


def cpu_baseline(problems, ncall):
    """The oracle, single-threaded, one iteration of each integrand at `ncall`;
    then the same work split over contiguous cube ranges on every usable host
    CPU (one thread each; the C oracle runs without the interpreter lock) as a
    timing-only all-cores figure."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    total = 0
    t0 = time.perf_counter()
    for pr in problems:
        grid = oracle.uniform_grid(pr.dim, pr.nbins)
        oracle.iteration(pr.family, pr.params, pr.dim, pr.nbins, ncall, pr.seed, 0, grid)
        total += oracle.plan(pr.dim, ncall)[3]
    dt = time.perf_counter() - t0
    cpu = host_cpu()
    threads = max(1, cpu["usable_cpus"] or 1)
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        for pr in problems:
            grid = oracle.uniform_grid(pr.dim, pr.nbins)
            g, m, p, _ = oracle.plan(pr.dim, ncall)
            cut = [m * k // (4 * threads) for k in range(4 * threads + 1)]
            list(ex.map(lambda ab: oracle.sample_range(pr.family, pr.params, pr.dim, pr.nbins,
                                                       g, m, p, pr.seed, 0, grid, ab[0], ab[1]),
                        zip(cut[:-1], cut[1:])))
    dt_all = time.perf_counter() - t0
    return {"value": total / dt, "unit": "evals/s", "cores": 1, "kind": "oracle",
            "sample": (f"one iteration of each of the three 8-D integrands at {ncall} samples "
                       f"requested ({total} evaluated), 500 bins, uniform grid, "
                       f"{dt:.1f} s single-threaded"),
            "cpu_model": cpu["model"], "logical_cpus": cpu["logical_cpus"],
            "usable_cpus": cpu["usable_cpus"],
            "all_cores_timing_only": {"value": total / dt_all, "unit": "evals/s",
                                      "threads": threads, "seconds": round(dt_all, 3),
                                      "kind": "oracle over cube ranges, one thread per usable CPU"}}


def bench_batch(mc, n, iters, full=True):
    """The batched form on the n-integrand workload: throughput of `iters`
    fixed iterations (rel_tol 0) with the default split, graph replay against
    eager launches, and (full) after the autotuner and the time until every
    integrand reaches 1e-3 relative error (or 20 iterations)."""
    problems = workloads.batch_problems(n=n)
    items = [(p.family, p.dim, p.ncall, p.params) for p in problems]
    t_a = time.perf_counter()
    b = mc.Batch(items, seed=0)
    t_b = time.perf_counter()
    plans = [mc.mcubes_plan_sizes(p.dim, p.ncall) for p in problems]
    flops_iter = sum(flops_per_sample(p.family, p.dim) * pl[3]
                     for p, pl in zip(problems, plans))

    def run(use_graph, itmax=iters, rel_tol=0.0, batch=None):
        bb = batch if batch is not None else b
        rc, res = bb.integrate(itmax, rel_tol, use_graph=use_graph)
        info = bb.info()
        ms = info["last_ms"]
        return {"ms": round(ms, 3), "iterations": info["last_iterations"],
                "samples": info["last_samples"],
                "evals_per_s": info["last_samples"] / (ms * 1e-3),
                "ms_per_iteration": round(ms / info["last_iterations"], 3),
                "replans": info["last_replans"]}, res

    b.integrate(1, 0.0)  # warm-up: graph capture, first-touch of the buffers
    default_graph, _ = run(True)
    default_eager, _ = run(False)
    info = b.info()
    default_graph["tflops"] = flops_iter * default_graph["iterations"] / (
        default_graph["ms"] * 1e-3) / 1e12
    default_graph["frac_of_fp64_vector_peak"] = default_graph["tflops"] / FP64_VECTOR_PEAK_TFLOPS
    out = {"workload": (f"{n} Genz integrands (6 families, dims 2-10 uniform, budgets "
                        "log-uniform 1e6-1e8 samples/iter, seeded parameters), 500 bins"),
           "integrands": n, "samples_per_iter": sum(pl[3] for pl in plans),
           "classes": info["classes"], "default_tiles": info["tiles"],
           "default_streams": info["streams"], "launches_per_iteration": info["launches"],
           "device_mib": round(info["device_bytes"] / 2**20, 1), "create_s": round(t_b - t_a, 3),
           "fixed_iterations_default_graph": default_graph,
           "fixed_iterations_default_eager": default_eager}
    # the same workload with the FP32 map and integrand (default split, graph)
    b32 = mc.Batch(items, seed=0, options=mc.mcubes_default_options(precision=mc.MCUBES_FP32))
    b32.integrate(1, 0.0)
    out["fixed_iterations_fp32_default_graph"], _ = run(True, batch=b32)
    b32.destroy()
    if not full:
        return out
    t_c = time.perf_counter()
    b.autotune()
    t_d = time.perf_counter()
    b.integrate(1, 0.0)
    tuned, _ = run(True)
    info = b.info()
    tuned["tflops"] = flops_iter * tuned["iterations"] / (tuned["ms"] * 1e-3) / 1e12
    tuned["frac_of_fp64_vector_peak"] = tuned["tflops"] / FP64_VECTOR_PEAK_TFLOPS
    to_tol, res = run(True, itmax=20, rel_tol=1e-3)
    to_tol["converged"] = sum(1 for r in res if r["converged"])
    to_tol["nonfinite"] = sum(1 for r in res if r["status"] == mc.MCUBES_E_NONFINITE)
    out.update({"autotune_s": round(t_d - t_c, 3), "tuned_tiles": info["tiles"],
                "tuned_streams": info["streams"], "fixed_iterations_tuned_graph": tuned,
                "to_1e-3_tuned_graph": to_tol})
    return out


def bench_time_to_tol(mc, problems, reps=3, rel_tol=1e-3):
    """Wall time of mcubes_integrate (plan, iterations, stop test) until the
    error estimate reaches rel_tol of the estimate, FP64 and FP32 forms of each
    8-D integrand.  One untimed call per form first (first-call set-up); the
    forms are interleaved and every entry is the median of `reps` runs (the
    runs are bit-identical: same samples).  The true error comes from the
    stored closed forms, read outside the timed region."""
    cf = closed_forms()
    forms = (("fp64", mc.MCUBES_FP64), ("fp32", mc.MCUBES_FP32))
    pr0 = problems[0]
    for _, prec in forms:
        mc.mcubes_integrate(pr0.family, pr0.params, pr0.dim, pr0.ncall, 1, rel_tol, pr0.seed,
                            mc.mcubes_default_options(nbins=500, precision=prec))
    times, res = {}, {}
    for _ in range(reps):
        for pr in problems:
            for name, prec in forms:
                key = f"{workloads.FAMILY_NAMES[pr.family]}_{name}"
                opts = mc.mcubes_default_options(nbins=500, precision=prec)
                t_a = time.perf_counter()
                r = mc.mcubes_integrate(pr.family, pr.params, pr.dim, pr.ncall, 50, rel_tol,
                                        pr.seed, opts)
                times.setdefault(key, []).append(time.perf_counter() - t_a)
                res[key] = r
    out = {}
    for pr in problems:
        fam = workloads.FAMILY_NAMES[pr.family]
        exact = cf[pr.name]["integral"]
        for name, _ in forms:
            key = f"{fam}_{name}"
            r = res[key]
            t = sorted(times[key])
            dev = abs(r["estimate"] - exact)
            out[key] = {"seconds": round(t[len(t) // 2], 4), "runs": [round(v, 4) for v in t],
                        "iterations": r["iterations"], "converged": r["converged"],
                        "estimate": r["estimate"], "error": r["error"],
                        "rel_error": (r["error"] / abs(r["estimate"]) if r["estimate"] else None),
                        "closed_form": exact, "true_rel_error": dev / abs(exact),
                        "error_in_sigma": dev / r["error"] if r["error"] else None,
                        "within_3_sigma": bool(dev <= 3 * r["error"])}
        a, b = out[f"{fam}_fp32"], out[f"{fam}_fp64"]
        # same samples in both forms: the difference is the FP32 rounding of the
        # map and the integrand, stated relative to the FP64 estimate and its error
        a["diff_vs_fp64"] = a["estimate"] - b["estimate"]
        a["diff_vs_fp64_in_sigma"] = (abs(a["diff_vs_fp64"]) / b["error"] if b["error"] else None)
    return out


# The paper's mean V100 CUDA times of the m-Cubes kernel (ms): Table 2 (§5.2),
# f1-f6 at 8-D, and Table 4 (§5.3), the addition integrand at 5-8-D.  The
# paper does not say which of its launch sizes (1e8 to 3e9 samples) a mean
# belongs to: context only.
PAPER_V100_CUDA_MS = {1: 286.7, 2: 402.1, 3: 284.5, 4: 385.7, 5: 284.3, 6: 283.8}
PAPER_V100_CUDA_SUM_MS = {5: 206.1, 6: 214.1, 7: 234.1, 8: 284.7}


def bench_paper_standin(mc, reps=3, sizes=(10**8, 3 * 10**9)):
    """V-Sample (with bin sums, uniform grid, 500 bins) on the paper's own
    integrands with its printed constants, at the smallest and largest
    samples per iteration of its kernel timings: mean launch time (HIP events
    on the launch stream) over `reps` launches after one untimed launch."""
    import torch
    stream = torch.cuda.current_stream()
    out = {}
    cases = [(f"f{k}_8d", k, 8) for k in range(1, 7)] + [(f"sum_{d}d", 7, d) for d in range(5, 9)]
    for ncall in sizes:
        for name, k, d in cases:
            fam, params = workloads.paper_integrand(k, d)
            pl = mc.mcubes_plan_create(fam, params, d, ncall, 0,
                                       mc.mcubes_default_options(nbins=500))
            b = mc.Buffers(pl)
            mc.mcubes_init_grid(pl, b.grid[0])
            mc.mcubes_vsample(pl, 0, b.grid[0], b.bins, b.partials)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for t in range(reps):
                mc.mcubes_vsample(pl, t, b.grid[0], b.bins, b.partials)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            n = pl.info["samples_per_iter"]
            entry = {"samples_per_iter": n, "vsample_ms": round(ms, 4),
                     "evals_per_s": n / (ms * 1e-3),
                     "fp64_tflops": flops_per_sample(fam, d) * n / (ms * 1e-3) / 1e12}
            entry["v100_cuda_ms"] = (PAPER_V100_CUDA_MS[k] if k <= 6
                                     else PAPER_V100_CUDA_SUM_MS[d])
            out[f"{name}_{ncall:.0e}".replace("+", "")] = entry
    return {"workload": ("the paper's f1-f6 (eqs. 1-6, printed constants) at 8-D and sum x_i "
                         "at 5-8-D, uniform grid, 500 bins, one V-Sample launch with bin sums"),
            "note": ("V100 means from Tables 2 and 4 are context: the paper does not say "
                     "which launch size each belongs to"), "cases": out}


# network multiply-adds per flow sample: 4 coupling layers, each 96x64 + 64x64 + 64x99
FLOW_GEMM_FLOPS = 2 * 4 * (96 * 64 + 64 * 64 + 64 * 99)
BF16_MFMA_PEAK_TFLOPS = 2500.0
HBM_PEAK_GBPS = 8000.0
# per training sample: the forward products, the input-gradient products and
# the weight-gradient sums (three times the network); and the scratch bytes
# per layer of the BF16 training step: the pass writes u (6 FP32), h1, h2,
# d2, d1 (64 BF16 each), the spline deltas (99 BF16), the third product's
# BF16 operands (128 B) and the ReLU bit masks (16 B), and reads back u, the
# operands and the masks; the five weight-gradient tiles read their inputs
# (2 and 1 u rows, h1, h2 twice) and deltas (d1 twice, d2, spline deltas
# 0-63 and 64-98)
FLOW_TRAIN_FLOPS = 3 * FLOW_GEMM_FLOPS
FLOW_TRAIN_BYTES = 4 * ((24 + 4 * 128 + 198 + 128 + 16) + (24 + 128 + 16)
                        + (8 + 128) + (4 + 128) + (128 + 128) + (128 + 128) + (128 + 70))


def bench_flow(mc, ncall, plain_iters=50):
    """The learned-proposal form on the 6-D correlated mixture (integral 1):
    plain FP64 m-Cubes for plain_iters iterations against the whole flow
    pipeline (warm-up, training, BF16 proposal iterations) run to 1e-3, with
    wall times, estimates, claimed and true errors."""
    pr = workloads.mixture_6d(ncall=ncall)
    opts = mc.mcubes_default_options(nbins=500)
    t_a = time.perf_counter()
    r = mc.mcubes_integrate(pr.family, pr.params, 6, ncall, plain_iters, 1e-3, 11, opts)
    t_b = time.perf_counter()
    plain = {"seconds": round(t_b - t_a, 4), "iterations": r["iterations"],
             "converged": r["converged"], "estimate": r["estimate"], "error": r["error"],
             "chi2_dof": r["chi2_dof"], "true_rel_error": abs(r["estimate"] - 1.0),
             "error_in_sigma": abs(r["estimate"] - 1.0) / r["error"] if r["error"] else None}
    # the plain method's own error bar would need (error / 1e-3)^2 times the iterations
    plain["iterations_for_claimed_1e-3"] = (r["iterations"] * (r["error"] / 1e-3) ** 2
                                            if r["error"] else None)
    fl = mc.Flow(workloads.flow_init(7))
    t_a = time.perf_counter()
    res, rep = fl.integrate(pr.family, pr.params, ncall, 10, 1e-3, 11, opts)
    t_b = time.perf_counter()
    fo = mc.mcubes_flow_options()
    mc.lib().mcubes_default_flow_options(mc.ctypes.byref(fo))
    items = min(fo.train_items, mc.mcubes_plan_sizes(6, ncall)[1])
    p = mc.mcubes_plan_sizes(6, ncall)[2]
    rows = max(items // fo.warmup_iters, 1) * p * fo.warmup_iters  # warm-up samples
    trained = (rows * fo.epochs
               + (fo.rounds + fo.tail_rounds) * fo.round_samples * fo.round_epochs
               + min(fo.anchor_rounds, fo.rounds) * rows * fo.round_epochs)
    n_eval = mc.mcubes_plan_sizes(6, ncall)[3]
    flow_s = rep["flow_ms"] * 1e-3
    evals = n_eval * res["iterations"] / flow_s if flow_s > 0 else None
    flow = {"seconds": round(t_b - t_a, 4), "total_ms": round(rep["total_ms"], 2),
            "warmup_ms": round(rep["warmup_ms"], 2), "train_ms": round(rep["train_ms"], 2),
            "proposal_ms": round(rep["flow_ms"], 2), "iterations": res["iterations"],
            "converged": res["converged"], "estimate": res["estimate"], "error": res["error"],
            "chi2_dof": res["chi2_dof"], "true_rel_error": abs(res["estimate"] - 1.0),
            "error_in_sigma": (abs(res["estimate"] - 1.0) / res["error"]
                               if res["error"] else None),
            "used_flow": rep["used_flow"], "weight_tail_shape": rep["tail_shape"],
            "last_plain_var": rep["last_plain_var"],
            "first_flow_var": rep["first_flow_var"],
            "training_samples_per_s": trained / (rep["train_ms"] * 1e-3),
            "training_network_tflops": trained / (rep["train_ms"] * 1e-3) * FLOW_TRAIN_FLOPS / 1e12,
            "training_scratch_gbps": trained / (rep["train_ms"] * 1e-3) * FLOW_TRAIN_BYTES / 1e9,
            "proposal_evals_per_s": evals,
            "proposal_network_tflops": (evals * FLOW_GEMM_FLOPS / 1e12) if evals else None}
    if flow["proposal_network_tflops"]:
        flow["proposal_frac_of_bf16_mfma_peak"] = (flow["proposal_network_tflops"]
                                                   / BF16_MFMA_PEAK_TFLOPS)
    flow["training_frac_of_bf16_mfma_peak"] = (flow["training_network_tflops"]
                                               / BF16_MFMA_PEAK_TFLOPS)
    flow["training_frac_of_hbm_peak"] = flow["training_scratch_gbps"] / HBM_PEAK_GBPS
    return {"workload": ("6-D mixture of two correlated Gaussians (sigma 0.05, correlation "
                         f"0.9, centres 1/3 and 2/3 on the diagonal), {ncall} samples/iter, "
                         "500 bins; integral 1"),
            "plain_fp64": plain, "flow_pipeline_bf16": flow}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--ncall", type=int, default=1 << 30)
    ap.add_argument("--cpu-ncall", type=int, default=1 << 25)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ttt", action="store_true")
    ap.add_argument("--no-standin", action="store_true",
                    help="skip the V-Sample timings on the paper's own integrands")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--blocks", type=int, default=0)
    ap.add_argument("--batch-n", type=int, default=512,
                    help="integrands of the batched-form measurement (0 = skip it)")
    ap.add_argument("--batch-iters", type=int, default=5)
    ap.add_argument("--flow-ncall", type=int, default=1 << 26,
                    help="samples per iteration of the learned-proposal section (0: skip)")
    ap.add_argument("--only-flow", action="store_true",
                    help="run only the learned-proposal section and print it")
    ap.add_argument("--only-batch", action="store_true",
                    help="measure only the batched form at its default geometry (no autotuner)"
                         " and print its figures as one JSON line (for profiling)")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="before the steps, run one plain device copy of this many MiB "
                         "(reference point for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout "
              "(cube ranges per GPU, one all-reduce of sums and bins per iteration) is "
              "described in the design notes but not built", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2302_05730_amd as mc

    torch.cuda.set_device(0)
    if args.calibrate_copy_mib:
        n = args.calibrate_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.only_batch:
        print(json.dumps({"batched": bench_batch(mc, args.batch_n or 512, args.batch_iters,
                                                 full=False)}), flush=True)
        return
    if args.only_flow:
        print(json.dumps({"learned_proposal": bench_flow(mc, args.flow_ncall or (1 << 26))}),
              flush=True)
        return
    problems = workloads.large_8d_set(ncall=args.ncall)
    opts = mc.mcubes_default_options(nbins=500, block_size=args.block, blocks=args.blocks)
    plans = [mc.mcubes_plan_create(pr.family, pr.params, pr.dim, pr.ncall, pr.seed, opts)
             for pr in problems]
    bufs = [mc.Buffers(pl) for pl in plans]
    for pl, b in zip(plans, bufs):
        mc.mcubes_init_grid(pl, b.grid[0])
    n_eval = plans[0].info["samples_per_iter"]
    p = plans[0].info["samples_per_cube"]
    stream = torch.cuda.current_stream()
    it = [0] * len(plans)

    def step(events=None):
        for k, (pl, b) in enumerate(zip(plans, bufs)):
            t = it[k]
            g_in, g_out = b.grid[t & 1], b.grid[(t + 1) & 1]
            mc.mcubes_fill(b.bins, 0.0)
            if events is not None:
                events[k][0].record(stream)
            mc.mcubes_vsample(pl, t, g_in, b.bins, b.partials)
            if events is not None:
                events[k][1].record(stream)
            mc.mcubes_reduce(pl, b.partials, b.est)
            mc.mcubes_combine(pl, t, b.est, b.state, 0.0)
            mc.mcubes_refine(pl, g_in, b.bins, g_out)
            it[k] = t + 1

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in plans]
           for _ in range(args.steps)]
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(evs[s])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    vs_ms = [[evs[s][k][0].elapsed_time(evs[s][k][1]) for s in range(args.steps)]
             for k in range(len(plans))]
    for b in bufs:
        st = b.state[:8].cpu().tolist()
        if st[6] != 0.0:
            raise RuntimeError("non-finite iteration estimate in the benchmark run")
    value = len(plans) * n_eval * args.steps / elapsed

    # dominant kernel: V-Sample; algorithmic FP64 flops per launch / mean launch time
    per_family = {}
    tot_flops, tot_ops, tot_ms = 0.0, 0.0, 0.0
    for pr, ms in zip(problems, vs_ms):
        mean_ms = sum(ms) / len(ms)
        fl = flops_per_sample(pr.family, pr.dim, p) * n_eval
        per_family[workloads.FAMILY_NAMES[pr.family]] = {
            "vsample_ms": round(mean_ms, 4), "evals_per_s": n_eval / (mean_ms * 1e-3),
            "tflops": fl / (mean_ms * 1e-3) / 1e12}
        tot_flops += fl
        tot_ops += fp64_ops_per_sample(pr.family, pr.dim, p) * n_eval
        tot_ms += mean_ms
    achieved = tot_flops / (tot_ms * 1e-3) / 1e12
    achieved_ops = tot_ops / (tot_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / FP64_VECTOR_PEAK_TFLOPS, 4),
                "traffic": stored_traffic(), "kernel": "vsample_kernel<family, 8, p=2>",
                "work_model": "9d + 7 + F_f algorithmic FP64 flops per sample",
                "frac_counting_every_fp64_op": round(achieved_ops / FP64_VECTOR_PEAK_TFLOPS, 4),
                "valu_busy_profiled": stored_valu_busy(), "per_family": per_family}

    # iterations after the grid has stopped adapting need no bin sums
    frozen = {}
    for pr, pl, b in zip(problems, plans, bufs):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for t in range(args.steps):
            mc.mcubes_vsample(pl, it[0] + t, b.grid[0], None, b.partials)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        frozen[workloads.FAMILY_NAMES[pr.family]] = {"vsample_ms": round(ms, 4),
                                                     "evals_per_s": n_eval / (ms * 1e-3)}

    # FP32 map/integrand form: V-Sample throughput and its difference to FP64
    fp32 = {}
    opts32 = mc.mcubes_default_options(nbins=500, block_size=args.block, blocks=args.blocks,
                                       precision=mc.MCUBES_FP32)
    for pr, b in zip(problems, bufs):
        pl = mc.mcubes_plan_create(pr.family, pr.params, pr.dim, pr.ncall, pr.seed, opts32)
        b32 = mc.Buffers(pl)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        mc.mcubes_fill(b32.bins, 0.0)
        mc.mcubes_vsample(pl, it[0], b.grid[it[0] & 1], b32.bins, b32.partials)
        e0.record(stream)
        for t in range(args.steps):
            mc.mcubes_vsample(pl, it[0], b.grid[it[0] & 1], b32.bins, b32.partials)
        e1.record(stream)
        mc.mcubes_reduce(pl, b32.partials, b32.est)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        fp32[workloads.FAMILY_NAMES[pr.family]] = {"vsample_ms": round(ms, 4),
                                                   "evals_per_s": n_eval / (ms * 1e-3)}

    ttt = None if args.no_ttt else bench_time_to_tol(mc, problems)
    standin = None if args.no_standin else bench_paper_standin(mc)
    batched = bench_batch(mc, args.batch_n, args.batch_iters) if args.batch_n > 0 else None
    flow = bench_flow(mc, args.flow_ncall) if args.flow_ncall > 0 else None
    cpu = None if args.no_cpu else cpu_baseline(problems, args.cpu_ncall)
    out = {
        "metric": "integrand evals/s + time to 1e-3 rel err, plain FP64 vs FP32/flow form",
        "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": ("8-D Genz Gaussian + oscillatory + corner peak, a~U(5,15), "
                                "u~U(0,1), 500 bins/axis, 2^30 samples/iter, one iteration "
                                "of each per step"),
                   "samples_per_iter": n_eval, "cubes": plans[0].info["ncubes"],
                   "samples_per_cube": p, "block": plans[0].info["block_size"],
                   "blocks": plans[0].info["blocks"], "parallelism": "single GPU"},
        "roofline": roofline, "cpu_baseline": cpu, "time_to_1e-3": ttt,
        "paper_standin": standin,
        "frozen_grid_vsample": frozen, "fp32_vsample": fp32, "batched": batched,
        "learned_proposal": flow,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
