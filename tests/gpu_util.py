"""Helpers shared by the GPU tests (not collected: no test_ prefix)."""
import sys

import numpy as np
import pytest
import torch

import oracle as O


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev():
    return torch.device("cuda", 0)


def t64(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev())


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def relerr(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def sample_rows(n, seed, k=48, width=1024):
    """Both ends, the tile and row boundaries of a `width`-wide transform,
    the middle, and k random rows."""
    fixed = [0, 1, 2, width // 2 - 1, width // 2, width - 1, width, width + 1, 2 * width - 1,
             n // 2 - 1, n // 2, n // 2 + 1, n - width - 1, n - 2, n - 1]
    rnd = np.random.default_rng(seed).integers(0, n, size=k)
    return np.unique(np.concatenate([fixed, rnd]))


def row_scale(prob, j, x):
    """S = (eta + sigma (|gamma|/h + (d+ + d-) h^-beta sum|omega|)) max|x|,
    an upper bound of sum_k |A_ik x_k| for every row i."""
    e, gam, dp, dm = O.level_scalars(prob, j)
    wsum = float(np.sum(np.abs(O.wsgd_weights(prob.beta, prob.n + 1))))
    h, sg = O.mesh_h(prob), O.sigma_of(prob.alpha)
    return (abs(e) + sg * (abs(gam) / h + (dp + dm) * h ** (-prob.beta) * wsum)) * float(np.max(np.abs(x)))


def sources(s, prob, levels=None):
    """f of every level (rows) at the plan's own nodes and sampling instants
    t_{j+sigma} (tsfcde_nodes, tsfcde_level_time), on the device; the oracle
    samples its own.  Manufactured sources go through their separable form."""
    import workloads as W
    ts = s.level_times()[: (levels if levels is not None else s.M)]
    x = s.nodes()
    if prob.solution is not None and prob.f_fn is None:
        return W.device_sources(prob, x, ts, dev())
    return t64(np.stack([prob.f(x, t) for t in ts]))


def batch_sources(bs, probs):
    """sources() for every member of a BatchSolver (each at its own nodes and
    instants)."""
    import workloads as W
    out = []
    for i, prob in enumerate(probs):
        x, ts = bs.nodes(i), bs.level_times(i)
        if prob.solution is not None and prob.f_fn is None:
            out.append(W.device_sources(prob, x, ts, dev()))
        else:
            out.append(t64(np.stack([prob.f(x, t) for t in ts])))
    return out
