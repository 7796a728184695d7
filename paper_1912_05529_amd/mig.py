"""Python binding of libmig.so (C ABI in include/mig.h) over torch tensors.

Argument marshalling only: shapes and dtypes are checked, device pointers and
the current HIP stream are passed through, and every step of the method runs
in the library's kernels.  The library must be built (``__graft_entry__.build``
or ``python paper_1912_05529_amd/build.py``); if it is missing, every call
raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmig.so")

MIG_OK, MIG_E_ARG, MIG_E_UNSTABLE, MIG_E_DEVICE, MIG_E_WORKSPACE = 0, -1, -2, -3, -4

_lib = None


class MigError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__("%s failed: %s (%d)" % (what, strerror(code), code))


class CDesc(C.Structure):
    """ctypes mirror of ``mig_table_desc``."""

    _fields_ = [
        ("ntaps", C.c_int32), ("nk", C.c_int32),
        ("kmin", C.c_double), ("kmax", C.c_double),
        ("dx", C.c_double), ("dz", C.c_double),
        ("theta_max_deg", C.c_double),
        ("w_pass", C.c_double), ("w_trans", C.c_double), ("w_evan", C.c_double),
        ("ngrid", C.c_int32), ("ncheck", C.c_int32), ("nreweight", C.c_int32),
        ("reserved", C.c_int32),
        ("lambda_", C.c_double), ("beta", C.c_double), ("tau", C.c_double),
        ("margin", C.c_double),
    ]


class CSection(C.Structure):
    """ctypes mirror of ``mig_section``."""

    _fields_ = [
        ("data", C.c_void_p), ("vel", C.c_void_p), ("omega", C.c_void_p),
        ("image", C.c_void_p),
        ("nx", C.c_int32), ("nz", C.c_int32), ("nw", C.c_int32), ("reserved", C.c_int32),
    ]


class CTuning(C.Structure):
    """ctypes mirror of ``mig_tuning``."""

    _fields_ = [("omegas_per_group", C.c_int32), ("reducers", C.c_int32),
                ("stall_limit_us", C.c_int32), ("flags", C.c_int32),
                ("outputs_mid", C.c_int32)]


MIG_TUNE_FORCE_STALL = 1


def cdesc(d) -> CDesc:
    """Builds the C descriptor from any object with the TableDesc fields."""
    lam = d.lam if getattr(d, "lam", None) is not None else 1e-9 * d.ngrid
    return CDesc(int(d.ntaps), int(d.nk), float(d.kmin), float(d.kmax), float(d.dx),
                 float(d.dz), float(d.theta_max_deg), float(d.w_pass), float(d.w_trans),
                 float(d.w_evan), int(d.ngrid), int(d.ncheck), int(d.nreweight), 0,
                 float(lam), float(d.beta), float(d.tau), float(d.margin))


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libmig.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    L = C.CDLL(LIB_PATH)
    P, i32, sz = C.c_void_p, C.c_int32, C.c_size_t
    D = C.POINTER(CDesc)
    sig = {
        "mig_strerror": ([C.c_int], C.c_char_p),
        "mig_version": ([], C.c_char_p),
        "mig_design_workspace_size": ([D], sz),
        "mig_design_table": ([D, P, P, P, P, P, sz, P], C.c_int),
        "mig_table_index": ([P, P, D, i32, i32, i32, P, P], C.c_int),
        "mig_workspace_size": ([i32, i32, i32, D], sz),
        "mig_workspace_min_size": ([i32, i32, D], sz),
        "mig_workspace_status": ([P, P], C.c_int),
        "mig_extrapolate": ([P, P, P, P, P, D, i32, i32, i32, P, P, sz, P], C.c_int),
        "mig_image": ([P, P, i32, i32, P], C.c_int),
        "mig_migrate": ([P, P, P, P, D, i32, i32, i32, P, P, sz, P], C.c_int),
        "mig_migrate_noalloc": ([P, P, P, P, D, i32, i32, i32, P, P], C.c_int),
        "mig_kernel_kind": ([i32, i32], C.c_int),
        "mig_transform_workspace_size": ([i32, i32], sz),
        "mig_transform_t": ([P, i32, i32, C.c_double, P, i32, P, P, sz, P], C.c_int),
        "mig_demigrate_workspace_size": ([i32, i32, i32, D], sz),
        "mig_demigrate": ([P, P, P, P, D, i32, i32, i32, P, P, sz, P], C.c_int),
        "mig_batch_workspace_size": ([C.POINTER(CSection), i32, D, C.POINTER(CTuning)], sz),
        "mig_migrate_batched": ([C.POINTER(CSection), i32, P, D, C.POINTER(CTuning), P, sz, P],
                                C.c_int),
        "mig_design2d_workspace_size": ([D], sz),
        "mig_design_table_2d": ([D, P, P, P, P, P, sz, P], C.c_int),
        "mig_omegas_per_group_3d": ([i32, i32, i32, i32], C.c_int),
        "mig_migrate3d_workspace_size": ([i32, i32, i32, i32, i32], sz),
        "mig_migrate3d": ([P, P, P, P, D, i32, i32, i32, i32, i32, P, P, P, sz, P], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)   # AttributeError: the built library is older than this binding
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def strerror(code: int) -> str:
    return lib().mig_strerror(int(code)).decode()


def version() -> str:
    return lib().mig_version().decode()


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _need(t, dtype, shape, name):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("%s must be a CUDA tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))


def _check(rc, what):
    if rc != MIG_OK:
        raise MigError(rc, what)


def design_workspace_size(desc) -> int:
    cd = cdesc(desc)
    return int(lib().mig_design_workspace_size(C.byref(cd)))


def design_table(desc, device="cuda", ws=None):
    """A0: returns dict(tab64 [nk][M+1] complex128, tab32 complex64, maxgain, passerr)."""
    cd = cdesc(desc)
    K = (desc.ntaps - 1) // 2 + 1
    dev = torch.device(device)
    tab64 = torch.empty((desc.nk, K), dtype=torch.complex128, device=dev)
    tab32 = torch.empty((desc.nk, K), dtype=torch.complex64, device=dev)
    mg = torch.empty(desc.nk, dtype=torch.float64, device=dev)
    pe = torch.empty(desc.nk, dtype=torch.float64, device=dev)
    need = design_workspace_size(desc)
    if ws is None:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
    rc = lib().mig_design_table(C.byref(cd), _p(tab64), _p(tab32), _p(mg), _p(pe), _p(ws),
                                ws.numel(), _stream())
    _check(rc, "mig_design_table")
    return {"tab64": tab64, "tab32": tab32, "maxgain": mg, "passerr": pe}


def table_index(vel, omega, desc):
    """A1: vel [nrows][nx] float32, omega [nw] float64 -> int32 [nrows][nx][nw]."""
    if vel.dim() == 1:
        vel = vel[None]
    nrows, nx = vel.shape
    nw = omega.numel()
    _need(vel, torch.float32, (nrows, nx), "vel")
    _need(omega, torch.float64, (nw,), "omega")
    idx = torch.empty((nrows, nx, nw), dtype=torch.int32, device=vel.device)
    cd = cdesc(desc)
    _check(lib().mig_table_index(_p(vel), _p(omega), C.byref(cd), nx, nw, nrows, _p(idx),
                                 _stream()), "mig_table_index")
    return idx


def workspace_size(nx, nsteps, nw, desc) -> int:
    cd = cdesc(desc)
    return int(lib().mig_workspace_size(nx, nsteps, nw, C.byref(cd)))


def workspace_min_size(nx, nw, desc) -> int:
    cd = cdesc(desc)
    return int(lib().mig_workspace_min_size(nx, nw, C.byref(cd)))


def workspace_status(ws) -> int:
    """Status of the last depth-stepping call on workspace ``ws`` (synchronizes
    the current stream): MIG_OK, or MIG_E_DEVICE if a reduction was abandoned."""
    return int(lib().mig_workspace_status(_p(ws), _stream()))


def check_workspace(ws, what="depth stepping"):
    """Raises MigError unless the last call on ``ws`` formed every image row."""
    _check(workspace_status(ws), what)


def kernel_kind(nx, ntaps) -> int:
    return int(lib().mig_kernel_kind(nx, ntaps))


def extrapolate(wf, vel, omega, tab32, desc, nsteps=None, rows=True, out=None, ws=None,
                want_plane=True, rows_out=None):
    """A2-A4: advance wf [nx][nw] complex64 by nsteps (default vel.shape[0]).

    Returns (plane or None, rows [nsteps][nx] float64 or None)."""
    nx, nw = wf.shape
    if nsteps is None:
        nsteps = vel.shape[0]
    _need(wf, torch.complex64, (nx, nw), "wf")
    if vel.shape[0] < nsteps or vel.shape[1] != nx:
        raise ValueError("vel must have at least nsteps rows of nx")
    _need(vel, torch.float32, None, "vel")
    _need(omega, torch.float64, (nw,), "omega")
    _need(tab32, torch.complex64, (desc.nk, (desc.ntaps - 1) // 2 + 1), "tab32")
    if want_plane and out is None:
        out = torch.empty_like(wf)
    if out is not None:
        _need(out, torch.complex64, (nx, nw), "out")
    if rows_out is not None:
        _need(rows_out, torch.float64, (nsteps, nx), "rows_out")
        rws = rows_out
    else:
        rws = torch.empty((nsteps, nx), dtype=torch.float64, device=wf.device) if rows else None
    if ws is None and nsteps > 0:
        ws = torch.empty(max(workspace_size(nx, nsteps, nw, desc), 1), dtype=torch.uint8,
                         device=wf.device)
    cd = cdesc(desc)
    rc = lib().mig_extrapolate(_p(wf), _p(out), _p(vel), _p(omega), _p(tab32), C.byref(cd),
                               nx, nw, nsteps, _p(rws), _p(ws), 0 if ws is None else ws.numel(),
                               _stream())
    _check(rc, "mig_extrapolate")
    return out, rws


def image(wf):
    """A3: row[x] = sum_r Re wf[x][r] (float64)."""
    nx, nw = wf.shape
    row = torch.empty(nx, dtype=torch.float64, device=wf.device)
    return image_into(wf, row)


def image_into(wf, row):
    """A3 into a caller-provided contiguous float64 row of length nx."""
    nx, nw = wf.shape
    _need(wf, torch.complex64, (nx, nw), "wf")
    _need(row, torch.float64, (nx,), "row")
    _check(lib().mig_image(_p(wf), _p(row), nx, nw, _stream()), "mig_image")
    return row


def migrate(data, vel, omega, tab32, desc, ws=None, out=None):
    """Algorithm 1 end to end: data [nx][nw] complex64, vel [nz][nx] -> image [nz][nx]."""
    nx, nw = data.shape
    nz = vel.shape[0]
    _need(data, torch.complex64, (nx, nw), "data")
    _need(vel, torch.float32, (nz, nx), "vel")
    _need(omega, torch.float64, (nw,), "omega")
    _need(tab32, torch.complex64, (desc.nk, (desc.ntaps - 1) // 2 + 1), "tab32")
    if ws is None:
        ws = torch.empty(max(workspace_size(nx, max(nz - 1, 1), nw, desc), 1),
                         dtype=torch.uint8, device=data.device)
    img = out if out is not None else torch.empty((nz, nx), dtype=torch.float64,
                                                  device=data.device)
    _need(img, torch.float64, (nz, nx), "image")
    cd = cdesc(desc)
    rc = lib().mig_migrate(_p(data), _p(vel), _p(omega), _p(tab32), C.byref(cd), nx, nz, nw,
                           _p(img), _p(ws), ws.numel(), _stream())
    _check(rc, "mig_migrate")
    return img


def migrate_noalloc(data, vel, omega, tab32, desc, out=None):
    """Algorithm 1 end to end through the allocation-free entry point: the
    library's static per-GPU workspace instead of a caller workspace."""
    nx, nw = data.shape
    nz = vel.shape[0]
    _need(data, torch.complex64, (nx, nw), "data")
    _need(vel, torch.float32, (nz, nx), "vel")
    _need(omega, torch.float64, (nw,), "omega")
    _need(tab32, torch.complex64, (desc.nk, (desc.ntaps - 1) // 2 + 1), "tab32")
    img = out if out is not None else torch.empty((nz, nx), dtype=torch.float64,
                                                  device=data.device)
    _need(img, torch.float64, (nz, nx), "image")
    cd = cdesc(desc)
    rc = lib().mig_migrate_noalloc(_p(data), _p(vel), _p(omega), _p(tab32), C.byref(cd), nx, nz,
                                   nw, _p(img), _stream())
    _check(rc, "mig_migrate_noalloc")
    return img


def _sections(batch):
    """batch: list of dicts with tensors data [nx][nw] c64, vel [nz][nx] f32,
    omega [nw] f64 and image [nz][nx] f64 (allocated if missing)."""
    arr = (CSection * len(batch))()
    for i, b in enumerate(batch):
        data, vel, omega = b["data"], b["vel"], b["omega"]
        nx, nw = data.shape
        nz = vel.shape[0]
        _need(data, torch.complex64, (nx, nw), "data")
        _need(vel, torch.float32, (nz, nx), "vel")
        _need(omega, torch.float64, (nw,), "omega")
        if b.get("image") is None:
            b["image"] = torch.empty((nz, nx), dtype=torch.float64, device=data.device)
        _need(b["image"], torch.float64, (nz, nx), "image")
        arr[i] = CSection(data.data_ptr(), vel.data_ptr(), omega.data_ptr(),
                          b["image"].data_ptr(), nx, nz, nw, 0)
    return arr


def _tuning(tune):
    if tune is None:
        return None
    t = CTuning()
    t.omegas_per_group = int(tune.get("omegas_per_group", 0))
    t.reducers = int(tune.get("reducers", 0))
    t.stall_limit_us = int(tune.get("stall_limit_us", 0))
    t.flags = int(tune.get("flags", 0))
    t.outputs_mid = int(tune.get("outputs_mid", 0))
    return C.byref(t)


def batch_workspace_size(batch, desc, tune=None) -> int:
    arr = _sections(batch)
    cd = cdesc(desc)
    return int(lib().mig_batch_workspace_size(arr, len(batch), C.byref(cd), _tuning(tune)))


def migrate_batched(batch, tab32, desc, tune=None, ws=None):
    """Batched Algorithm 1: every section's image (dict key "image") is filled.

    tune: {"omegas_per_group": G, "reducers": R} or None (library defaults)."""
    arr = _sections(batch)
    _need(tab32, torch.complex64, (desc.nk, (desc.ntaps - 1) // 2 + 1), "tab32")
    cd = cdesc(desc)
    tn = _tuning(tune)
    if ws is None:
        n = int(lib().mig_batch_workspace_size(arr, len(batch), C.byref(cd), tn))
        ws = torch.empty(max(n, 1), dtype=torch.uint8, device=tab32.device)
    rc = lib().mig_migrate_batched(arr, len(batch), _p(tab32), C.byref(cd), tn, _p(ws),
                                   ws.numel(), _stream())
    _check(rc, "mig_migrate_batched")
    return [b["image"] for b in batch]


def demigrate_workspace_size(nx, nz, nw, desc) -> int:
    cd = cdesc(desc)
    return int(lib().mig_demigrate_workspace_size(nx, nz, nw, C.byref(cd)))


def demigrate(image, vel, omega, tab32, desc, nw=None, out=None, ws=None):
    """Adjoint of migrate: image [nz][nx] float64 -> surface plane [nx][nw] complex64."""
    nz, nx = image.shape
    nw = omega.numel() if nw is None else nw
    _need(image, torch.float64, (nz, nx), "image")
    _need(vel, torch.float32, (nz, nx), "vel")
    _need(omega, torch.float64, (nw,), "omega")
    _need(tab32, torch.complex64, (desc.nk, (desc.ntaps - 1) // 2 + 1), "tab32")
    if out is None:
        out = torch.empty((nx, nw), dtype=torch.complex64, device=image.device)
    _need(out, torch.complex64, (nx, nw), "data")
    if ws is None:
        ws = torch.empty(max(demigrate_workspace_size(nx, nz, nw, desc), 1), dtype=torch.uint8,
                         device=image.device)
    cd = cdesc(desc)
    rc = lib().mig_demigrate(_p(image), _p(vel), _p(omega), _p(tab32), C.byref(cd), nx, nz, nw,
                             _p(out), _p(ws), ws.numel(), _stream())
    _check(rc, "mig_demigrate")
    return out


def transform_workspace_size(nt, nw) -> int:
    """Bytes of workspace mig_transform_t needs (the FP32 DFT matrix)."""
    return int(lib().mig_transform_workspace_size(int(nt), int(nw)))


def transform_t(section, dt, omega, out=None, ws=None):
    """Transform along t: section [nx][nt] float32 -> plane [nx][nw] complex64."""
    nx, nt = section.shape
    nw = omega.numel()
    _need(section, torch.float32, (nx, nt), "section")
    _need(omega, torch.float64, (nw,), "omega")
    if out is None:
        out = torch.empty((nx, nw), dtype=torch.complex64, device=section.device)
    _need(out, torch.complex64, (nx, nw), "out")
    if ws is None:
        n = int(lib().mig_transform_workspace_size(nt, nw))
        ws = torch.empty(max(n, 1), dtype=torch.uint8, device=section.device)
    rc = lib().mig_transform_t(_p(section), nx, nt, float(dt), _p(omega), nw, _p(out), _p(ws),
                               ws.numel(), _stream())
    _check(rc, "mig_transform_t")
    return out


def migrate_tx(section, dt, vel, omega, tab32, desc, ws=None):
    """Algorithm 1 from a t-x section: transform along t, then migrate."""
    return migrate(transform_t(section, dt, omega), vel, omega, tab32, desc, ws=ws)


# --------------------------------------------------------------------------- #
# 3-D extension: circularly symmetric 2-D extrapolators.
# --------------------------------------------------------------------------- #
def design_table_2d(desc, device="cuda", ws=None):
    """2-D table: dict(tab64 [nk][NU] complex128, tab32 complex64, maxgain, passerr),
    NU = (M+1)(M+2)/2 unique coefficients c(a, b), a >= b, at a(a+1)/2 + b."""
    cd = cdesc(desc)
    M = (desc.ntaps - 1) // 2
    NU = (M + 1) * (M + 2) // 2
    dev = torch.device(device)
    tab64 = torch.empty((desc.nk, NU), dtype=torch.complex128, device=dev)
    tab32 = torch.empty((desc.nk, NU), dtype=torch.complex64, device=dev)
    mg = torch.empty(desc.nk, dtype=torch.float64, device=dev)
    pe = torch.empty(desc.nk, dtype=torch.float64, device=dev)
    need = int(lib().mig_design2d_workspace_size(C.byref(cd)))
    if need == 0:
        raise MigError(-1, "mig_design2d_workspace_size: descriptor out of range")
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    rc = lib().mig_design_table_2d(C.byref(cd), _p(tab64), _p(tab32), _p(mg), _p(pe), _p(ws),
                                   ws.numel(), _stream())
    _check(rc, "mig_design_table_2d")
    return {"tab64": tab64, "tab32": tab32, "maxgain": mg, "passerr": pe}


def omegas_per_group_3d(nx, ny, nw, want=0) -> int:
    return int(lib().mig_omegas_per_group_3d(nx, ny, nw, want))


def migrate3d_workspace_size(nx, ny, nw, nz, omegas_per_group=0) -> int:
    return int(lib().mig_migrate3d_workspace_size(nx, ny, nw, nz, omegas_per_group))


def migrate3d(data, vel, omega, tab32, desc, omegas_per_group=0, ws=None, out=None,
              plane_out=None):
    """3-D migration.  data [nw][nx][ny] complex64, vel [nz][nx][ny] float32,
    omega [nw] float64 -> image [nz][nx][ny] float64 (and the last plane into
    plane_out [nw][nx][ny] complex64 when given)."""
    nw, nx, ny = data.shape
    nz = vel.shape[0]
    _need(data, torch.complex64, (nw, nx, ny), "data")
    _need(vel, torch.float32, (nz, nx, ny), "vel")
    _need(omega, torch.float64, (nw,), "omega")
    M = (desc.ntaps - 1) // 2
    _need(tab32, torch.complex64, (desc.nk, (M + 1) * (M + 2) // 2), "tab32")
    if out is None:
        out = torch.empty((nz, nx, ny), dtype=torch.float64, device=data.device)
    _need(out, torch.float64, (nz, nx, ny), "out")
    if plane_out is not None:
        _need(plane_out, torch.complex64, (nw, nx, ny), "plane_out")
    if ws is None:
        n = migrate3d_workspace_size(nx, ny, nw, nz, omegas_per_group)
        ws = torch.empty(max(n, 1), dtype=torch.uint8, device=data.device)
    cd = cdesc(desc)
    rc = lib().mig_migrate3d(_p(data), _p(vel), _p(omega), _p(tab32), C.byref(cd), nx, ny, nw,
                             nz, omegas_per_group, _p(out), _p(plane_out), _p(ws), ws.numel(),
                             _stream())
    _check(rc, "mig_migrate3d")
    return out
