"""Writes pcgs_headline_levels.json: the first two levels of the headline
march (alpha = 0.7, beta = 1.8, n = 2^20, M = 512) solved by the oracle's
FFT route (circulant-embedding products, Strang preconditioner, preconditioned
CGS to the recursive residual 1e-12 |g|), on 2048 seeded rows plus the ends,
with |u|_2, |g|_2 and the computed true residual |g - A u|_2 of each level.

Calls only oracle/ and workloads/.  Run from the repository root:
    python tests/golden/make_pcgs_headline_levels.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402


def main():
    prob = W.config_large()
    n = prob.n
    rng = np.random.default_rng(20160301)
    rows = np.unique(np.concatenate([[0, 1, 1023, 1024, n // 2, n - 2, n - 1], rng.integers(0, n, size=2048)]))
    U = [O.initial_level(prob)]
    levels = []
    for j in range(2):
        f = O.source_level(prob, j)
        u, its = O.level_solve_pcgs(prob, np.array(U), j, f, rtol=1e-12)
        g = O.rhs_fft(prob, np.array(U), j, f)
        r = g - O.embedding_product(prob, j, u, "A")
        U.append(u)
        levels.append({"j": j + 1, "iterations": its, "values": u[rows].tolist(), "max_abs": float(np.max(np.abs(u))),
                       "u_norm": float(np.linalg.norm(u)), "g_norm": float(np.linalg.norm(g)),
                       "residual_norm": float(np.linalg.norm(r))})
        print(f"level {j + 1}: {its} iterations", flush=True)
    out = {"what": "u^1, u^2 of the headline march by the oracle's FFT-PCGS route (rtol 1e-12)",
           "n": n, "M": prob.M, "alpha": prob.alpha, "beta": prob.beta, "rows": rows.tolist(), "levels": levels}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "pcgs_headline_levels.json"), "w") as fh:
        json.dump(out, fh)


if __name__ == "__main__":
    main()
