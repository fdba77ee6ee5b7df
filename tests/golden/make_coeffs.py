"""Writes kernel_coeffs.json: the reference's kernel coefficients.

Calls only ``oracle/``. Order 1 "paper" is Sec. 3.1's printed pair with the
labels read as swapped (intercept 0.773, root at the printed 4.386); the
"fit" entries are the L1-optimal ReLU polynomials of orders 1-3 on
[0, 2 ln 255] from ``oracle.coeffs.fit``; each entry carries the first
positive root found by bisection.

Run from the repository root:  python tests/golden/make_coeffs.py
"""
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
from oracle import coeffs, core  # noqa: E402


def main():
    out = {"source": "oracle.coeffs (L1 fit on [0, 2 ln 255]) and Sec. 3.1 printed f1", "sets": {}}
    c = list(coeffs.PAPER_F1)
    out["sets"]["paper1"] = {"order": 1, "c": c, "x0": core.first_root(c, 1, 0.0)}
    for n in (1, 2, 3):
        c = list(coeffs.fit(n))
        out["sets"][f"fit{n}"] = {"order": n, "c": c, "x0": core.first_root(c, n, 0.0),
                                  "l1": coeffs.l1_loss(c, n)}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "kernel_coeffs.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=2)
    print(path)


if __name__ == "__main__":
    main()
