"""Shared helpers of the GPU parity tests (imported by tests/test_gpu_*.py)."""
import numpy as np

import oracle
import workloads

# Flags may differ only where the exact signed distance is inside this band
# (metres); signed distances must agree to the same amount.
BAND = 1e-5
SD_TOL = 1e-5
CENTRE_TOL = 1e-5


def load(name):
    data = workloads.load(name)
    return data, workloads.robot(data)


def f32_up(x):
    """FP32 values as FP64 (what the oracle reads when it mirrors GPU inputs)."""
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def print_case(*parts):
    print("[case]", *parts, flush=True)


def oracle_robot(desc):
    return oracle.Robot(desc)
