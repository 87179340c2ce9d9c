"""Shared helpers of the GPU parity tests."""
import numpy as np
import pytest
import torch

import oracle

# cm, cm, cm, 1/GeV (1/50 GeV: the smallest |kappa| the workloads generate), rad, rad
FLOORS = np.array([1.0, 1.0, 1.0, 0.02, 1.0, 1.0])


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def to_dev(a, dtype=None):
    a = np.ascontiguousarray(a)
    t = torch.from_numpy(a)
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def mask_dev(mask):
    return to_dev(np.asarray(mask, np.uint32).view(np.int32))


def rel_state_err(gpu_state, ref_state):
    """Per-parameter relative error: |d| / max(|ref|, floor), phi wrapped."""
    d = np.asarray(gpu_state, np.float64) - ref_state
    d[4] = (d[4] + np.pi) % (2 * np.pi) - np.pi
    return np.abs(d) / np.maximum(np.abs(ref_state), FLOORS[:, None])


def cov_err(gpu_cov, ref_cov):
    """max_ij |dC_ij| / sqrt(C_ii C_jj) per track."""
    g = oracle.unpack_cov(np.asarray(gpu_cov, np.float64))
    r = oracle.unpack_cov(ref_cov)
    d = np.sqrt(np.einsum('iin->in', r))
    return np.max(np.abs(g - r) / (d[:, None, :] * d[None, :, :]), axis=(0, 1))
