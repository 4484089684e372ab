"""Writes the stored expected values under tests/golden/ by calling only the
oracle (the 40-function box workload, sampled J/K entries by the definition,
Eq. J_and_K).  Run from the repository root: python tests/golden/make_golden.py"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402
import workloads as wl  # noqa: E402


def main():
    c = wl.config1()
    rng = np.random.default_rng(2024)
    cnt = 48
    i = rng.integers(0, c["D"].shape[0], cnt)
    p = rng.integers(0, 40, cnt)
    q = rng.integers(0, 40, cnt)
    J, K = oracle.jk_entries(c["centers"], c["alpha"], c["tau"], c["D"], i, p, q)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "box40_entries.txt")
    with open(out, "w") as f:
        f.write("# 40 s functions in a 10 bohr box (seed 1), m=4 densities N(0,1)/40 (seed 101),\n")
        f.write("# no screening. J_i[p][q], K_i[p][q] by the definition (Eq. J_and_K).\n")
        f.write("# i p q J K\n")
        for t in range(cnt):
            f.write(f"{i[t]} {p[t]} {q[t]} {J[t]:.17e} {K[t]:.17e}\n")


if __name__ == "__main__":
    main()
