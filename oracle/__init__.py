"""ctypes loader for the plain FP64 CPU oracle (oracle/vsw_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it to check and time the GPU library.  The GPU library
never imports, links or calls it, and it shares no code with the library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vsw_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# -ffp-contract=off: no fused multiply-add, one rounding per operation in
# the order the source writes it.  -fopenmp: the cell and face loops may run
# on several threads, with bitwise the same results for any thread count.
# No -march=native: the library is compiled on one host and may be loaded on
# another (the GPU host), whose CPU may lack the build host's extensions.
CFLAGS = ["-O3", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-Wall", "-Wextra"]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C, FP64)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_lp = ctypes.POINTER(ctypes.c_int64)


class OrcParams(ctypes.Structure):
    _fields_ = [("g", ctypes.c_double), ("cfl", ctypes.c_double),
                ("h_threshold", ctypes.c_double), ("dt_fixed", ctypes.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        L.orc_mesh_build.restype = ctypes.c_void_p
        L.orc_mesh_build.argtypes = [ctypes.c_int64, _dp, _dp, ctypes.c_int64, _ip, _dp,
                                     ctypes.c_char_p, ctypes.c_int]
        L.orc_mesh_free.argtypes = [ctypes.c_void_p]
        for f in ("orc_mesh_ncells", "orc_mesh_nedges", "orc_mesh_nwalls"):
            getattr(L, f).restype = ctypes.c_int64
            getattr(L, f).argtypes = [ctypes.c_void_p]
        L.orc_mesh_geometry.argtypes = [ctypes.c_void_p] + [_dp] * 11 + [_ip] * 3
        L.orc_reconstruct.argtypes = [ctypes.c_void_p, ctypes.POINTER(OrcParams), _dp, _dp, _dp,
                                      _dp, _dp, _ip, _dp]
        L.orc_residual.argtypes = [ctypes.c_void_p, ctypes.POINTER(OrcParams), _dp, _dp, _dp,
                                   _dp, _dp, _dp]
        L.orc_face_flux.argtypes = [ctypes.POINTER(OrcParams), _dp, _dp, ctypes.c_double,
                                    ctypes.c_double, _dp, _dp]
        L.orc_hll.argtypes = [ctypes.c_double, _dp, _dp, ctypes.c_double, ctypes.c_double,
                              _dp, _dp]
        L.orc_dt.restype = ctypes.c_double
        L.orc_dt.argtypes = [ctypes.c_void_p, ctypes.POINTER(OrcParams), _dp, _dp, _dp]
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_run.restype = ctypes.c_int
        L.orc_run.argtypes = [ctypes.c_void_p, ctypes.POINTER(OrcParams), _dp, _dp, _dp, _dp,
                              ctypes.c_int64, ctypes.c_double, _lp, _dp, _lp]
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's loops (results do not depend on it)."""
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def _d(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _i(a):
    return a.ctypes.data_as(_ip) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    pass


def params(g=9.81, cfl=0.45, h_threshold=1e-3, dt_fixed=0.0) -> OrcParams:
    return OrcParams(g, cfl, h_threshold, dt_fixed)


class Mesh:
    """Connectivity and geometry built by the oracle from raw input."""

    def __init__(self, vx, vy, tri, h):
        L = lib()
        self.vx, self.vy = _f64(vx), _f64(vy)
        self.tri = np.ascontiguousarray(tri, dtype=np.int32).reshape(-1, 3)
        self.h = _f64(h)
        err = ctypes.create_string_buffer(256)
        ptr = L.orc_mesh_build(len(self.vx), _d(self.vx), _d(self.vy), len(self.tri),
                               _i(self.tri), _d(self.h), err, 256)
        if not ptr:
            raise OracleError(err.value.decode())
        self._p = ctypes.c_void_p(ptr)
        self.nc = int(L.orc_mesh_ncells(self._p))
        self.ne = int(L.orc_mesh_nedges(self._p))
        self.nw = int(L.orc_mesh_nwalls(self._p))

    @classmethod
    def from_case(cls, case):
        return cls(case.vx, case.vy, case.tri, case.h)

    def __del__(self):
        p = getattr(self, "_p", None)
        if p is not None and _lib is not None:
            _lib.orc_mesh_free(p)
            self._p = None

    def geometry(self) -> dict:
        nc = self.nc
        out = {k: np.empty(nc) for k in ("cx", "cy", "area", "perim")}
        for k in ("len", "nx", "ny", "dx", "dy", "wx", "wy"):
            out[k] = np.empty((nc, 3))
        for k in ("nbr", "is_left", "tri"):
            out[k] = np.empty((nc, 3), dtype=np.int32)
        lib().orc_mesh_geometry(self._p, *[_d(out[k]) for k in (
            "cx", "cy", "area", "perim", "len", "nx", "ny", "dx", "dy", "wx", "wy")],
            _i(out["nbr"]), _i(out["is_left"]), _i(out["tri"]))
        return out

    def reconstruct(self, p: OrcParams, H, HU, HV) -> dict:
        nc = self.nc
        H, HU, HV = _f64(H), _f64(HU), _f64(HV)
        grad = np.empty((nc, 4, 2))
        alpha = np.empty((nc, 3))
        order = np.empty(nc, dtype=np.int32)
        face = np.empty((nc, 3, 5))
        lib().orc_reconstruct(self._p, ctypes.byref(p), _d(H), _d(HU), _d(HV), _d(grad),
                              _d(alpha), _i(order), _d(face))
        return {"grad": grad, "alpha": alpha, "order": order, "face": face}

    def residual(self, p: OrcParams, H, HU, HV):
        H, HU, HV = _f64(H), _f64(HU), _f64(HV)
        R = [np.empty(self.nc) for _ in range(3)]
        lib().orc_residual(self._p, ctypes.byref(p), _d(H), _d(HU), _d(HV), *[_d(r) for r in R])
        return R

    def dt(self, p: OrcParams, H, HU, HV) -> float:
        H, HU, HV = _f64(H), _f64(HU), _f64(HV)
        return float(lib().orc_dt(self._p, ctypes.byref(p), _d(H), _d(HU), _d(HV)))

    def run(self, p: OrcParams, H, HU, HV, t=0.0, nsteps=1, t_stop=np.inf,
            check=True):
        """Advance a copy of (H, HU, HV); returns dict with the new state."""
        H, HU, HV = _f64(H).copy(), _f64(HU).copy(), _f64(HV).copy()
        tt = ctypes.c_double(t)
        done = ctypes.c_int64(0)
        clamps = ctypes.c_int64(0)
        dts = np.zeros(max(int(nsteps), 1))
        rc = lib().orc_run(self._p, ctypes.byref(p), _d(H), _d(HU), _d(HV), ctypes.byref(tt),
                           int(nsteps), float(t_stop), ctypes.byref(done), _d(dts),
                           ctypes.byref(clamps))
        if rc != 0 and check:
            raise OracleError(f"oracle run failed after {done.value} steps")
        return {"H": H, "HU": HU, "HV": HV, "t": tt.value, "steps": done.value,
                "dts": dts[:done.value], "clamps": clamps.value, "rc": rc}


def face_flux(p: OrcParams, left, right, nx, ny):
    """One face: left/right = (eta, h, H, u, v); right=None for a wall."""
    left = _f64(left)
    phi = np.empty(3)
    pc = np.empty(2)
    r = _f64(right) if right is not None else None
    lib().orc_face_flux(ctypes.byref(p), _d(left), _d(r), float(nx), float(ny), _d(phi), _d(pc))
    return phi, pc


def hll(g, wl, wr, nx, ny):
    """HLL flux of primitive states (H, u, v); returns (phi, (sL, sR, u*, c*))."""
    wl, wr = _f64(wl), _f64(wr)
    phi = np.empty(3)
    sp = np.empty(4)
    lib().orc_hll(float(g), _d(wl), _d(wr), float(nx), float(ny), _d(phi), _d(sp))
    return phi, sp
