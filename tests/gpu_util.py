"""Helpers shared by the GPU parity tests (host side only)."""
import numpy as np
import pytest
import torch


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1501_01855_amd as ovl
    ovl.lib()
    return ovl


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).cuda()


def to_host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b):
    a = np.asarray(a).reshape(-1)
    b = np.asarray(b).reshape(-1)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def max_rel_elem(a, b):
    """max_i |a_i - b_i| / max_i |b_i|  (element-wise, scaled by the field's size)."""
    a = np.asarray(a).reshape(-1)
    b = np.asarray(b).reshape(-1)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
