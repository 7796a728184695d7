"""ctypes marshalling for the C oracle (test infrastructure; no arithmetic here)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (IEEE double, no contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = [
            "gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp",
            "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
            "-Wno-unused-parameter", _SRC, "-o", tmp, "-lm",
        ]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _CDesc(C.Structure):
    _fields_ = [
        ("ntaps", C.c_int32), ("nk", C.c_int32),
        ("kmin", C.c_double), ("kmax", C.c_double),
        ("dx", C.c_double), ("dz", C.c_double),
        ("theta_max_deg", C.c_double),
        ("w_pass", C.c_double), ("w_trans", C.c_double), ("w_evan", C.c_double),
        ("ngrid", C.c_int32), ("ncheck", C.c_int32), ("nreweight", C.c_int32),
        ("pad_", C.c_int32),
        ("lambda_", C.c_double), ("beta", C.c_double), ("tau", C.c_double),
        ("margin", C.c_double),
    ]


@dataclass(frozen=True)
class OrcDesc:
    """Design descriptor, field for field the C struct ``orc_desc``."""

    ntaps: int
    nk: int
    kmin: float
    kmax: float
    dx: float
    dz: float
    theta_max_deg: float = 60.0
    w_pass: float = 1.0
    w_trans: float = 0.01
    w_evan: float = 0.01
    ngrid: int = 1024
    ncheck: int = 8192
    nreweight: int = 30
    lam: float | None = None  # None -> 1e-9 * ngrid
    beta: float = 1.0
    tau: float = 5e-4
    margin: float = 1e-5

    @classmethod
    def from_obj(cls, o) -> "OrcDesc":
        names = [f for f in cls.__dataclass_fields__]
        return cls(**{n: getattr(o, n) for n in names})

    def c(self) -> _CDesc:
        lam = self.lam if self.lam is not None else 1e-9 * self.ngrid
        return _CDesc(
            int(self.ntaps), int(self.nk), float(self.kmin), float(self.kmax),
            float(self.dx), float(self.dz), float(self.theta_max_deg),
            float(self.w_pass), float(self.w_trans), float(self.w_evan),
            int(self.ngrid), int(self.ncheck), int(self.nreweight), 0,
            float(lam), float(self.beta), float(self.tau), float(self.margin),
        )


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=False)
    lib = C.CDLL(_LIB)
    P = C.c_void_p
    i32 = C.c_int32
    D = C.POINTER(_CDesc)
    lib.orc_design_table.argtypes = [D, C.c_int, P, P, P, P]
    lib.orc_table_index.argtypes = [D, P, i32, P, i32, i32, P]
    lib.orc_extrapolate.argtypes = [D, P, P, i32, P, i32, i32, P, P, P]
    lib.orc_image.argtypes = [P, i32, i32, P]
    lib.orc_migrate.argtypes = [D, P, P, i32, P, i32, i32, P, P]
    lib.orc_demigrate.argtypes = [D, P, P, i32, P, i32, i32, P, P]
    lib.orc_num_threads.argtypes = []
    lib.orc_transform_t.argtypes = [P, i32, i32, C.c_double, P, i32, P]
    lib.orc_design_table_2d.argtypes = [D, C.c_int, P, P, P, P]
    lib.orc_migrate3d.argtypes = [D, P, P, i32, P, i32, i32, i32, P, P, P]
    for f in ("orc_design_table", "orc_table_index", "orc_extrapolate",
              "orc_image", "orc_migrate", "orc_demigrate", "orc_num_threads",
              "orc_transform_t", "orc_design_table_2d", "orc_migrate3d"):
        getattr(lib, f).restype = C.c_int
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError("oracle %s failed with code %d" % (what, rc))


def num_threads() -> int:
    return int(load().orc_num_threads())


def design_table(desc, apply_scale: bool = True):
    """Returns (tab complex128 [nk][M+1], maxgain [nk], passerr [nk], scale [nk])."""
    d = OrcDesc.from_obj(desc) if not isinstance(desc, OrcDesc) else desc
    K = (d.ntaps - 1) // 2 + 1
    tab = np.zeros((d.nk, K), np.complex128)
    mg = np.zeros(d.nk)
    pe = np.zeros(d.nk)
    sc = np.zeros(d.nk)
    cd = d.c()
    _check(load().orc_design_table(C.byref(cd), int(bool(apply_scale)), _ptr(tab),
                                   _ptr(mg), _ptr(pe), _ptr(sc)), "design_table")
    return tab, mg, pe, sc


def table_index(desc, omega, vel):
    """vel [nrows][nx] float32 -> int32 [nrows][nx][nw]."""
    d = OrcDesc.from_obj(desc) if not isinstance(desc, OrcDesc) else desc
    omega = _f64(omega)
    vel = _f32(np.atleast_2d(vel))
    nrows, nx = vel.shape
    idx = np.zeros((nrows, nx, omega.size), np.int32)
    cd = d.c()
    _check(load().orc_table_index(C.byref(cd), _ptr(omega), omega.size, _ptr(vel),
                                  nx, nrows, _ptr(idx)), "table_index")
    return idx


def extrapolate(desc, tab, omega, vel, plane, nsteps=None, rows=True):
    """Advance plane [nx][nw] by nsteps (default: vel rows).  Returns (plane, rows|None)."""
    d = OrcDesc.from_obj(desc) if not isinstance(desc, OrcDesc) else desc
    tab = _c128(tab)
    omega = _f64(omega)
    vel = _f32(np.atleast_2d(vel))
    plane = _c128(plane)
    nx, nw = plane.shape
    if nsteps is None:
        nsteps = vel.shape[0]
    assert vel.shape[0] >= nsteps and vel.shape[1] == nx and omega.size == nw
    out = np.zeros_like(plane)
    rws = np.zeros((nsteps, nx)) if rows else None
    cd = d.c()
    _check(load().orc_extrapolate(C.byref(cd), _ptr(tab), _ptr(omega), nw, _ptr(vel),
                                  nx, nsteps, _ptr(plane), _ptr(out), _ptr(rws)),
           "extrapolate")
    return out, rws


def image(plane):
    plane = _c128(plane)
    nx, nw = plane.shape
    row = np.zeros(nx)
    _check(load().orc_image(_ptr(plane), nx, nw, _ptr(row)), "image")
    return row


def migrate(desc, tab, omega, vel, data):
    """data [nx][nw] complex, vel [nz][nx] -> image [nz][nx] float64."""
    d = OrcDesc.from_obj(desc) if not isinstance(desc, OrcDesc) else desc
    tab = _c128(tab)
    omega = _f64(omega)
    vel = _f32(vel)
    data = _c128(data)
    nx, nw = data.shape
    nz = vel.shape[0]
    assert vel.shape[1] == nx and omega.size == nw
    img = np.zeros((nz, nx))
    cd = d.c()
    _check(load().orc_migrate(C.byref(cd), _ptr(tab), _ptr(omega), nw, _ptr(vel), nx, nz,
                              _ptr(data), _ptr(img)), "migrate")
    return img


def demigrate(desc, tab, omega, vel, img):
    """Adjoint of migrate: image [nz][nx] -> data [nx][nw] complex128."""
    d = OrcDesc.from_obj(desc) if not isinstance(desc, OrcDesc) else desc
    tab = _c128(tab)
    omega = _f64(omega)
    vel = _f32(vel)
    img = _f64(img)
    nz, nx = img.shape
    nw = omega.size
    assert vel.shape == (nz, nx)
    data = np.zeros((nx, nw), np.complex128)
    cd = d.c()
    _check(load().orc_demigrate(C.byref(cd), _ptr(tab), _ptr(omega), nw, _ptr(vel), nx, nz,
                                _ptr(img), _ptr(data)), "demigrate")
    return data


def transform_t(section, dt, omega):
    """section [nx][nt] float32 -> [nx][nw] complex128 (direct DFT at omega)."""
    section = _f32(section)
    omega = _f64(omega)
    nx, nt = section.shape
    out = np.zeros((nx, omega.size), np.complex128)
    _check(load().orc_transform_t(_ptr(section), nx, nt, float(dt), _ptr(omega), omega.size,
                                  _ptr(out)), "transform_t")
    return out


def design_table_2d(desc, apply_scale: bool = True):
    """2-D circularly symmetric table: (tab [nk][NU] complex128, maxgain, passerr, scale)."""
    d = OrcDesc.from_obj(desc) if not isinstance(desc, OrcDesc) else desc
    M = (d.ntaps - 1) // 2
    NU = (M + 1) * (M + 2) // 2
    tab = np.zeros((d.nk, NU), np.complex128)
    mg = np.zeros(d.nk)
    pe = np.zeros(d.nk)
    sc = np.zeros(d.nk)
    cd = d.c()
    _check(load().orc_design_table_2d(C.byref(cd), int(bool(apply_scale)), _ptr(tab), _ptr(mg),
                                      _ptr(pe), _ptr(sc)), "design_table_2d")
    return tab, mg, pe, sc


def migrate3d(desc, tab, omega, vel, data, want_plane=False):
    """data [nx][ny][nw] complex, vel [nz][nx][ny] -> image [nz][nx][ny]
    (and the last plane [nx][ny][nw] when want_plane)."""
    d = OrcDesc.from_obj(desc) if not isinstance(desc, OrcDesc) else desc
    tab = _c128(tab)
    omega = _f64(omega)
    vel = _f32(vel)
    data = _c128(data)
    nx, ny, nw = data.shape
    nz = vel.shape[0]
    assert vel.shape == (nz, nx, ny) and omega.size == nw
    img = np.zeros((nz, nx, ny))
    last = np.zeros_like(data) if want_plane else None
    cd = d.c()
    _check(load().orc_migrate3d(C.byref(cd), _ptr(tab), _ptr(omega), nw, _ptr(vel), nx, ny, nz,
                                _ptr(data), _ptr(img), _ptr(last)), "migrate3d")
    return (img, last) if want_plane else img
