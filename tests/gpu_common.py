"""Shared helpers of the GPU parity tests (HIP path vs FP64 oracle)."""
import numpy as np
import pytest
import torch

from paper_2607_20766_amd.engine import LAMBDA_P27


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def rel_err(got, ref, floor=0.0):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    return np.abs(got - ref) / np.maximum(np.abs(ref), floor)


def oracle_mol(O, ms):
    return (ms.xyz, O.alpha_from_radius(ms.radius, LAMBDA_P27))
