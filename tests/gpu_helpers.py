"""Helpers of the GPU parity tests: numpy <-> device tensors and the
relative-L2 comparison used throughout (||gpu - oracle|| / ||oracle||)."""
import numpy as np
import pytest


def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def dev(a):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def f32(a):
    """The FP32 rounding of an array, back in float64 (what both sides see)."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    nb = np.linalg.norm(b)
    d = np.linalg.norm(a - b)
    return d / nb if nb > 0 else d


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
