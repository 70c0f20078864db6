"""Shared plumbing of the GPU parity tests: device check, seeded inputs,
oracle-side references (CPU) and comparisons."""
import numpy as np
import pytest

from paper_2312_10615_amd.workloads import random_state, sinusoid_forcing


def cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    return torch


def forcing_rhs(active, dims, h, seed):
    """b = (f, 0): seeded sinusoid forcing on the unknown faces, zero continuity."""
    f = sinusoid_forcing(*dims, h, seed=seed)
    return tuple(np.where(active[a], f[a], 0.0) for a in range(3)) + (np.zeros(dims),)


def random_fields(active, dims, seed):
    x = random_state(*dims, seed=seed)
    return tuple(np.where(m, v, 0.0) for m, v in zip(active, x))


def rel_err(got, want):
    num = np.sqrt(sum(float(np.sum((g - w) ** 2)) for g, w in zip(got, want)))
    den = np.sqrt(sum(float(np.sum(w ** 2)) for w in want))
    return num / den


def max_rel(got, want):
    num = max(float(np.abs(g - w).max()) for g, w in zip(got, want))
    den = max(float(np.abs(w).max()) for w in want)
    return num / den


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
