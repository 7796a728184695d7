"""Helpers shared by the GPU tests (not a test module)."""
import numpy as np
import torch


def dev():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch.device("cuda:0")


def upload(sec, d=None):
    """Section -> device tensors (data rounded to complex64)."""
    d = d or dev()
    return {
        "data": torch.from_numpy(np.ascontiguousarray(sec.data.astype(np.complex64))).to(d),
        "vel": torch.from_numpy(np.ascontiguousarray(sec.vel)).to(d),
        "omega": torch.from_numpy(np.ascontiguousarray(sec.omega)).to(d),
    }


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def data64(sec):
    """The complex64-rounded data promoted exactly, so input rounding is shared."""
    return sec.data.astype(np.complex64).astype(np.complex128)
