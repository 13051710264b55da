"""Write paper_closed_forms.txt: the closed-form integrals over (0,1)^d of the
paper's benchmark integrands f1-f6 (eqs. 1-6, §5) for d = 2..8.

Calls only oracle.closed_forms (mpmath at 50 digits; exact rationals for f3).
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import closed_forms as cf  # noqa: E402


def main():
    out = os.path.join(HERE, "paper_closed_forms.txt")
    with open(out, "w") as fh:
        fh.write("# closed-form integral over (0,1)^d of the paper's f_k (eqs. 1-6)\n")
        fh.write("# written by make_paper_closed_forms.py from oracle/closed_forms.py\n")
        fh.write("# k d value\n")
        for k in range(1, 7):
            for d in range(2, 9):
                fam, params = cf.paper_params(k, d)
                fh.write(f"{k} {d} {float(cf.integral(fam, params, d))!r}\n")


if __name__ == "__main__":
    main()
