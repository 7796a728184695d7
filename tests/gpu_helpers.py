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


def assert_rows_close(got, ref, tol=1e-4, label="", axis=0, energy_floor=1e-3):
    """Element-wise parity of an image (or plane), row by row.

    * every element: |got - ref| <= tol * max|ref| (one scale for the whole
      array, so a wrong element in a quiet row cannot hide);
    * every row (index along ``axis``) whose L2 norm is at least
      ``energy_floor`` of the largest row's: relative L2 <= tol.
    Prints the worst figures so that the margins are on record."""
    got = np.moveaxis(np.asarray(got), axis, 0)
    ref = np.moveaxis(np.asarray(ref), axis, 0)
    assert got.shape == ref.shape
    scale = float(np.abs(ref).max())
    diff = np.abs(got - ref).reshape(ref.shape[0], -1)
    elem = diff.max(axis=1) / scale
    norms = np.linalg.norm(ref.reshape(ref.shape[0], -1), axis=1)
    live = norms >= energy_floor * norms.max()
    rows = np.linalg.norm(diff, axis=1)[live] / norms[live]
    worst_e = int(np.argmax(elem))
    print("%s: worst element error %.3e of max|ref| (row %d), worst row rel L2 %.3e over %d "
          "rows with energy" % (label, elem[worst_e], worst_e, rows.max() if rows.size else 0.0,
                                int(live.sum())), flush=True)
    assert np.isfinite(got).all(), label
    assert elem.max() <= tol, (label, worst_e, float(elem.max()))
    assert rows.size == 0 or rows.max() <= tol, (label, float(rows.max()))
