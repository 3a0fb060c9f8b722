"""Helpers shared by the GPU tests (inputs to device, error norms)."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def require_gpu():
    import torch
    from paper_2201_06914_amd import _lib
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    assert os.path.exists(_lib.LIB_PATH), "librtm.so must be built before the GPU tests"
    _lib.load()


def dev(a, dtype):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    return t.detach().cpu().double().numpy()


def rel(a, b) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()
