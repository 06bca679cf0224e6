"""Helpers shared by the GPU tests (no solver arithmetic here)."""
import os
import sys

import numpy as np
import pytest

D_, N_ = 0, 1

BC_SETS = {
    "DDNNNN": (D_, D_, N_, N_, N_, N_),
    "NDNNDN": (N_, D_, N_, N_, D_, N_),
    "NNNDNN": (N_, N_, N_, D_, N_, N_),
    "DDDDDD": (D_,) * 6,
    "NNNNND": (N_, N_, N_, N_, N_, D_),
}


def gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def require_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.linalg.norm(a - b)
    nb = np.linalg.norm(b)
    return d / nb if nb > 0 else d


def to_dev(x, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype).contiguous()


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()
