"""Shared helpers of the GPU parity tests (no method arithmetic here)."""
from __future__ import annotations

import copy

import numpy as np
import pytest
import torch


def gpu_available() -> bool:
    return torch.cuda.is_available()


requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="no GPU visible")


def r32(x):
    """Round to float32 and back to float64 (the values the GPU actually sees)."""
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def f32_problem(pb):
    """Copy of a synth.Problem whose float inputs are exactly float32 values,
    so the FP64 oracle and the FP32 GPU path consume identical inputs."""
    q = copy.deepcopy(pb)
    for name in ("gravity", "damping", "lo", "hi", "theta_true", "s0", "noise", "particles", "w_x", "u", "rho",
                 "lr_theta", "lr_S"):
        setattr(q, name, r32(getattr(q, name)))
    for name in ("dt", "sigma_obs", "sigma_def", "c", "eps_lam"):
        setattr(q, name, float(np.float32(getattr(q, name))))
    if q.arm is not None:
        q.arm = {k: (r32(v) if isinstance(v, np.ndarray) else float(np.float32(v))) for k, v in q.arm.items()}
    return q


def print_case(*parts):
    print("CASE", *parts, flush=True)
