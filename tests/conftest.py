import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def orc():
    import oracle
    if not os.path.exists(os.path.join(ROOT, "oracle", "libmpm_oracle.so")):
        oracle.build(force=True)
    return oracle


def observations(orc, case, use_b1=True):
    """x = s(truth) + sigma * eps as float32 values widened to float64, i.e. the
    exact numbers the GPU library is given."""
    s = orc.simulate(case["proto"], case["truth"], case["b1"] if use_b1 else None)
    x = (s + case["sigma"] * case["eps"].astype(np.float64)).astype(np.float32)
    return x


def sigmoid(v):
    return 1.0 / (1.0 + np.exp(-v))


def map_errors(gpu, orc, mask=None):
    """Per-map parity metrics: max |gpu - orc| / max |orc| (relative on log
    maps), max absolute difference and RMS difference, over `mask` voxels."""
    gpu = np.asarray(gpu, dtype=np.float64).reshape(4, -1)
    orc = np.asarray(orc, dtype=np.float64).reshape(4, -1)
    if mask is not None:
        gpu, orc = gpu[:, mask], orc[:, mask]
    d = np.abs(gpu - orc)
    scale = np.maximum(np.abs(orc).max(axis=1), 1e-30)
    return d.max(axis=1) / scale, d.max(axis=1), np.sqrt((d ** 2).mean(axis=1))


def well_posed(orc_maps, truth, tol=1.0):
    """Voxels whose oracle solution stayed near the truth (not drifted towards
    the border of the physical domain, where the ML optimum of a noisy voxel
    can sit and FP32 / FP64 runs separate)."""
    return np.all(np.abs(np.asarray(orc_maps) - np.asarray(truth)) < tol, axis=0)


def f32(a):
    return None if a is None else np.asarray(a, dtype=np.float32).astype(np.float64)


def cuda(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()
