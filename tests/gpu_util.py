"""Helpers shared by the GPU tests: layout conversion between the oracle and the C ABI."""
import numpy as np


def to_abi(a):
    """(V, 3, 3) or (V, 12) oracle arrays -> component-major (ncomp, V) contiguous."""
    V = a.shape[0]
    return np.ascontiguousarray(a.reshape(V, -1).T)


def from_abi(a, tensor=True):
    """(ncomp, V) -> (V, 3, 3) (tensor) or (V, ncomp)."""
    out = np.ascontiguousarray(a.T)
    return out.reshape(-1, 3, 3) if tensor else out


def cuda(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def rel_norm(a, b):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
