"""Helpers shared by the GPU tests (not collected: no test_ prefix)."""
import sys

import numpy as np
import pytest
import torch


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
