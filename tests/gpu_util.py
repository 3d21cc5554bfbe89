"""Helpers shared by the GPU parity tests (layout conversion and metrics)."""
import sys

import numpy as np
import torch


def announce(msg):
    """Name the case before a GPU step so a crash log says what was running."""
    print("[case] " + msg, flush=True)
    sys.stdout.flush()


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64) if not t.is_complex() else t.detach().cpu().numpy().astype(np.complex128)


def soa(a_n3):
    """(N, 3) oracle layout -> (3, N) library layout."""
    return np.ascontiguousarray(np.asarray(a_n3).T)


def aos(a_3n):
    return np.ascontiguousarray(np.asarray(a_3n).reshape(3, -1).T)


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))
