"""Write bench_closed_forms.json: the exact integrals over (0,1)^d of the
benchmark's integrands, against which the benchmark states the true error of
its time-to-1e-3 runs.

Entries: the three 8-D Genz integrands of the benchmark workload (parameters
from workloads.large_8d, seeds 1-3), the paper's f1-f6 at 8-D and the
addition integrand at 5-8-D (§5.2, §5.3; workloads.paper_integrand), and the
6-D correlated mixture of the learned-proposal workload.

Calls only oracle.closed_forms (mpmath at 50 digits, exact rationals for the
corner peak) on parameters from workloads; nothing else.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle import closed_forms as cf  # noqa: E402


def main():
    out = {}
    for pr in workloads.large_8d_set():
        out[pr.name] = {"family": pr.family, "dim": pr.dim, "params": pr.params,
                        "integral": float(cf.integral(pr.family, pr.params, pr.dim))}
    for k in range(1, 7):
        fam, params = workloads.paper_integrand(k, 8)
        out[f"paper_f{k}_8d"] = {"family": fam, "dim": 8, "params": params,
                                 "integral": float(cf.integral(fam, params, 8))}
    for d in range(5, 9):
        fam, params = workloads.paper_integrand(7, d)
        out[f"paper_sum_{d}d"] = {"family": fam, "dim": d, "params": params,
                                  "integral": float(cf.integral(fam, params, d))}
    pr = workloads.mixture_6d()
    out["mixture_6d"] = {"family": pr.family, "dim": pr.dim, "params": pr.params,
                         "integral": float(cf.integral(pr.family, pr.params, pr.dim))}
    with open(os.path.join(HERE, "bench_closed_forms.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
