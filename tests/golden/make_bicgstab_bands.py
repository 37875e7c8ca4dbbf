"""Writes bicgstab_bands.txt: the oracle's BiCGSTAB iteration counts on the
parity cases, for the right-hand side b and for K copies of b perturbed at
unit roundoff, b_k = b (1 + 1e-15 g_k) with g_k ~ N(0, 1) from
default_rng(99).

Why: the GPU sums its dot products in another (fixed) order, so its exit
iteration is only defined up to what rounding-level changes do to the
recurrence; on these nonsymmetric problems the oracle's own exit moves by
several iterations under such perturbations.  The parity test requires the
GPU's count in [min - 2, max + 2] of this band.  Stored here because the
64^3 case takes about 25 s per oracle solve.

Calls only the oracle and the input generators.  Run from the repository
root:  python tests/golden/make_bicgstab_bands.py
"""

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from problems import laplacian_scalar, lognormal_problem, random_blocks  # noqa: E402

K = 8
CASES = {
    "lap16_8cube": (lambda: laplacian_scalar(16, 16, 16, seed=1), (8, 8, 8)),
    "rand_ragged": (lambda: random_blocks(12, 10, 6, seed=5), (4, 5, 3)),
    "logn_24_32_40": (lambda: lognormal_problem(24, 32, 40, seed=7, sigma=2.0), (12, 16, 20)),
    # 64^3 3x3 random blocks with the automatic partition at 160 KB of LDS
    # and 256 compute units (8x8x16)
    "rand64_auto": (lambda: random_blocks(64, 64, 64, seed=2), (8, 8, 16)),
}


def main():
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bicgstab_bands.txt")
    lines = [
        "# Oracle BiCGSTAB iterations to rtol 1e-8 (right-preconditioned DD-ILU0,",
        "# Algorithm 1) for b and for 8 copies of b perturbed at 1e-15 relative",
        "# (default_rng(99)); written by make_bicgstab_bands.py from the oracle.",
        "# name sx sy sz iters_b min max all",
    ]
    for name, (make, sub) in CASES.items():
        p = make()
        st = O.setup(p, sub)
        its = [st.bicgstab(p.b, rtol=1e-8).iters]
        rng = np.random.default_rng(99)
        for _ in range(K):
            its.append(st.bicgstab(p.b * (1 + 1e-15 * rng.standard_normal(p.b.size)), rtol=1e-8).iters)
        print(name, its, flush=True)
        lines.append(f"{name} {sub[0]} {sub[1]} {sub[2]} {its[0]} {min(its)} {max(its)} "
                     + ",".join(str(i) for i in its))
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
