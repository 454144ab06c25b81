"""Helpers shared by the GPU tests (tensor plumbing only)."""
import numpy as np
import pytest
import torch


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2602_05081_amd as gf  # noqa: F401
    return gf


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def bits_to_numpy(t):
    return host(t).view(np.uint32)


def tau_tolerance(abs_sum):
    """optical-depth parity bar: |tau_gpu - tau_ref| <= 1e-5 * sum_i |tau_i| per ray"""
    return 1e-5 * abs_sum
