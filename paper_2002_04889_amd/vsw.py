"""Thin ctypes binding of the gfx950 library libvsw.so (include/vsw.h).

Argument marshalling only: every step of the solver runs in the library's
HIP kernels.  The functions carry the C names; ``Solver`` wraps a handle for
convenience.  Importing this module fails loudly when libvsw.so has not been
built (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import math
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# VSW_LIB names another build of the library (to compare builds)
LIB_PATH = os.environ.get("VSW_LIB") or os.path.join(_HERE, "libvsw.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "vsw.h")

VSW_OK, VSW_EINVAL, VSW_EMESH, VSW_ESTATE, VSW_ENOMEM, VSW_EDEVICE, VSW_EUNSTABLE = \
    0, -1, -2, -3, -4, -5, -6
VSW_FP64, VSW_FP32 = 0, 1
VSW_ORDER_HILBERT, VSW_ORDER_NONE, VSW_ORDER_RANDOM, VSW_ORDER_BISECTION = 0, 1, 2, 3
VSW_KERNEL_FUSED, VSW_KERNEL_TWO_PASS, VSW_KERNEL_FACES = 0, 1, 2
ERROR_NAMES = {0: "OK", -1: "EINVAL", -2: "EMESH", -3: "ESTATE", -4: "ENOMEM",
               -5: "EDEVICE", -6: "EUNSTABLE"}


class VswParams(ctypes.Structure):
    _fields_ = [("g", ctypes.c_double), ("cfl", ctypes.c_double),
                ("h_threshold", ctypes.c_double), ("dt_fixed", ctypes.c_double),
                ("precision", ctypes.c_int32), ("ordering", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


class VswError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"vsw error {ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_lp = ctypes.POINTER(ctypes.c_int64)
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_d = ctypes.c_double

_SIGS = {
    "vsw_create": (ctypes.c_int, [ctypes.POINTER(VswParams), ctypes.c_int, ctypes.POINTER(_vp)]),
    "vsw_destroy": (None, [_vp]),
    "vsw_upload_mesh": (ctypes.c_int, [_vp, _i64, _dp, _dp, _i64, _ip, _dp]),
    "vsw_upload_ensemble": (ctypes.c_int, [_vp, ctypes.c_int32, _lp, _dp, _dp, _lp, _ip, _dp]),
    "vsw_scenario_count": (ctypes.c_int, [_vp, _ip]),
    "vsw_scenario_status": (ctypes.c_int, [_vp, ctypes.c_int32, _dp, _dp, _lp]),
    "vsw_scenario_dt_history": (ctypes.c_int, [_vp, ctypes.c_int32, _i64, _dp, _lp]),
    "vsw_set_state": (ctypes.c_int, [_vp, _dp, _dp, _dp, _d]),
    "vsw_set_state_device": (ctypes.c_int, [_vp, _vp, _vp, _vp, _d]),
    "vsw_step": (ctypes.c_int, [_vp, _i64, _d, _lp, _dp]),
    "vsw_step_noalloc": (ctypes.c_int, [_vp, _i64, _d, _lp, _dp]),
    "vsw_get_state": (ctypes.c_int, [_vp, _dp, _dp, _dp, _dp]),
    "vsw_get_state_device": (ctypes.c_int, [_vp, _vp, _vp, _vp, _dp]),
    "vsw_last_dt": (ctypes.c_int, [_vp, _dp]),
    "vsw_dt_history": (ctypes.c_int, [_vp, _i64, _dp, _lp]),
    "vsw_clamp_count": (ctypes.c_int, [_vp, _lp]),
    "vsw_set_gauges": (ctypes.c_int, [_vp, ctypes.c_int32, _ip]),
    "vsw_get_gauges": (ctypes.c_int, [_vp, _i64, _dp, _dp, _lp]),
    "vsw_set_stream": (ctypes.c_int, [_vp, _vp]),
    "vsw_set_profiling": (ctypes.c_int, [_vp, ctypes.c_int]),
    "vsw_adjoint_gauge_loss": (ctypes.c_int, [_vp, _i64, _i64, ctypes.c_int32, _ip, _dp, _dp,
                                              _dp, _dp, _dp, _dp]),
    "vsw_set_graph": (ctypes.c_int, [_vp, ctypes.c_int]),
    "vsw_set_tile_order": (ctypes.c_int, [_vp, ctypes.c_int]),
    "vsw_set_occupancy": (ctypes.c_int, [_vp, ctypes.c_int]),
    "vsw_autotune": (ctypes.c_int, [_vp, _i64, _ip, _dp]),
    "vsw_set_kernel_variant": (ctypes.c_int, [_vp, ctypes.c_int]),
    "vsw_set_tile_size": (ctypes.c_int, [_vp, ctypes.c_int]),
    "vsw_tile_size": (ctypes.c_int, [_vp, _ip]),
    "vsw_kernel_times": (ctypes.c_int, [_vp, ctypes.c_int, _dp, _lp]),
    "vsw_kernel_name": (ctypes.c_char_p, [ctypes.c_int]),
    "vsw_prepare_mesh_host": (ctypes.c_int, [_i64, _dp, _dp, _i64, _ip, _dp, _dp, _dp, _dp,
                                             _ip, _ip, _lp, _lp]),
    "vsw_get_permutation": (ctypes.c_int, [_vp, _lp]),
    "vsw_mesh_info": (ctypes.c_int, [_vp, _lp, _lp, _lp]),
    "vsw_last_error": (ctypes.c_char_p, []),
    "vsw_version": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libvsw.so (raises if it is missing: build it first)."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime under the same soname
        # (libamdhip64.so.7).  Loading torch first makes libvsw.so bind to
        # that one runtime; two runtimes in one process do not share a device.
        import torch  # noqa: F401

        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not built; run __graft_entry__.build() "
                              "or python -m paper_2002_04889_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def header_symbols(path: str = HEADER):
    """Names of the functions include/vsw.h declares."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vsw_[a-z0-9_]+)\s*\(", text)))


def _check(rc):
    if rc != VSW_OK:
        raise VswError(rc, lib().vsw_last_error().decode())
    return rc


def _dptr(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- C names

def vsw_create(params: VswParams, device: int = 0):
    h = _vp()
    _check(lib().vsw_create(ctypes.byref(params), int(device), ctypes.byref(h)))
    return h


def vsw_destroy(h):
    lib().vsw_destroy(h)


def vsw_upload_mesh(h, vx, vy, tri, depth):
    vx, vy, depth = _f64(vx), _f64(vy), _f64(depth)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    return _check(lib().vsw_upload_mesh(h, len(vx), _dptr(vx), _dptr(vy), tri.size // 3,
                                        tri.ctypes.data_as(_ip), _dptr(depth)))


def vsw_upload_ensemble(h, meshes):
    """meshes: sequence of (vx, vy, tri, depth), one per scenario."""
    nv = np.array([len(m[0]) for m in meshes], dtype=np.int64)
    nc = np.array([np.asarray(m[2]).size // 3 for m in meshes], dtype=np.int64)
    vx = _f64(np.concatenate([np.asarray(m[0], dtype=np.float64) for m in meshes]))
    vy = _f64(np.concatenate([np.asarray(m[1], dtype=np.float64) for m in meshes]))
    tri = np.ascontiguousarray(np.concatenate([np.asarray(m[2], dtype=np.int32).reshape(-1)
                                               for m in meshes]))
    depth = _f64(np.concatenate([np.asarray(m[3], dtype=np.float64) for m in meshes]))
    return _check(lib().vsw_upload_ensemble(h, len(meshes), nv.ctypes.data_as(_lp), _dptr(vx),
                                            _dptr(vy), nc.ctypes.data_as(_lp),
                                            tri.ctypes.data_as(_ip), _dptr(depth)))


def vsw_scenario_count(h):
    n = ctypes.c_int32(0)
    _check(lib().vsw_scenario_count(h, ctypes.byref(n)))
    return n.value


def vsw_scenario_status(h):
    n = vsw_scenario_count(h)
    t, dt = np.empty(n), np.empty(n)
    steps = np.empty(n, dtype=np.int64)
    _check(lib().vsw_scenario_status(h, n, _dptr(t), _dptr(dt), steps.ctypes.data_as(_lp)))
    return t, dt, steps


def vsw_scenario_dt_history(h, scen):
    n = ctypes.c_int64(0)
    _check(lib().vsw_scenario_dt_history(h, int(scen), 0, None, ctypes.byref(n)))
    out = np.empty(n.value)
    _check(lib().vsw_scenario_dt_history(h, int(scen), n.value, _dptr(out), ctypes.byref(n)))
    return out


def vsw_set_state(h, H, HU, HV, t=0.0):
    H, HU, HV = _f64(H), _f64(HU), _f64(HV)
    return _check(lib().vsw_set_state(h, _dptr(H), _dptr(HU), _dptr(HV), float(t)))


def vsw_set_state_device(h, dH: int, dHU: int, dHV: int, t=0.0):
    return _check(lib().vsw_set_state_device(h, dH, dHU, dHV, float(t)))


def vsw_step(h, n, t_stop=math.inf, check=True):
    done = ctypes.c_int64(0)
    t = ctypes.c_double(0.0)
    rc = lib().vsw_step(h, int(n), float(t_stop), ctypes.byref(done), ctypes.byref(t))
    if check:
        _check(rc)
    return rc, done.value, t.value


VSW_NOALLOC_BYTES = 1 << 20


def vsw_step_noalloc(h, n, t_stop=math.inf, check=True):
    """vsw_step without allocation: logs in the library's fixed device array
    (n * (2 scenarios + gauges) doubles at most VSW_NOALLOC_BYTES / 8)."""
    done = ctypes.c_int64(0)
    t = ctypes.c_double(0.0)
    rc = lib().vsw_step_noalloc(h, int(n), float(t_stop), ctypes.byref(done), ctypes.byref(t))
    if check:
        _check(rc)
    return rc, done.value, t.value


def vsw_get_state(h, nc):
    H, HU, HV = np.empty(nc), np.empty(nc), np.empty(nc)
    t = ctypes.c_double(0.0)
    _check(lib().vsw_get_state(h, _dptr(H), _dptr(HU), _dptr(HV), ctypes.byref(t)))
    return H, HU, HV, t.value


def vsw_get_state_device(h, dH: int, dHU: int, dHV: int):
    t = ctypes.c_double(0.0)
    _check(lib().vsw_get_state_device(h, dH, dHU, dHV, ctypes.byref(t)))
    return t.value


def vsw_last_dt(h):
    d = ctypes.c_double(0.0)
    _check(lib().vsw_last_dt(h, ctypes.byref(d)))
    return d.value


def vsw_dt_history(h):
    n = ctypes.c_int64(0)
    _check(lib().vsw_dt_history(h, 0, None, ctypes.byref(n)))
    out = np.empty(n.value)
    _check(lib().vsw_dt_history(h, n.value, _dptr(out), ctypes.byref(n)))
    return out


def vsw_clamp_count(h):
    n = ctypes.c_int64(0)
    _check(lib().vsw_clamp_count(h, ctypes.byref(n)))
    return n.value


def vsw_set_gauges(h, cells):
    cells = np.ascontiguousarray(cells, dtype=np.int32)
    return _check(lib().vsw_set_gauges(h, len(cells), cells.ctypes.data_as(_ip)))


def vsw_get_gauges(h, ngauges):
    n = ctypes.c_int64(0)
    _check(lib().vsw_get_gauges(h, 0, None, None, ctypes.byref(n)))
    eta = np.empty((n.value, ngauges))
    t = np.empty(n.value)
    _check(lib().vsw_get_gauges(h, n.value, _dptr(eta), _dptr(t), ctypes.byref(n)))
    return t, eta


def vsw_set_stream(h, stream_handle: int | None):
    return _check(lib().vsw_set_stream(h, stream_handle))


def vsw_set_kernel_variant(h, variant: int):
    return _check(lib().vsw_set_kernel_variant(h, int(variant)))


def vsw_set_tile_size(h, cells: int):
    return _check(lib().vsw_set_tile_size(h, int(cells)))


def vsw_tile_size(h):
    n = ctypes.c_int32(0)
    _check(lib().vsw_tile_size(h, ctypes.byref(n)))
    return n.value


def vsw_adjoint_gauge_loss(h, nc, nsteps, checkpoint_every, gauges, eta_obs):
    """Returns (loss, dL/dH0, dL/dHU0, dL/dHV0, dL/dh) in the caller's order."""
    gauges = np.ascontiguousarray(gauges, dtype=np.int32)
    obs = _f64(np.asarray(eta_obs, dtype=np.float64).reshape(int(nsteps), len(gauges)))
    loss = ctypes.c_double(0.0)
    out = [np.empty(nc) for _ in range(4)]
    _check(lib().vsw_adjoint_gauge_loss(h, int(nsteps), int(checkpoint_every), len(gauges),
                                        gauges.ctypes.data_as(_ip), _dptr(obs),
                                        ctypes.byref(loss), *[_dptr(o) for o in out]))
    return (loss.value, *out)


VSW_TUNE_CONFIGS = 42
# kernel organisation of configuration c: TUNE_ORGS[c // 6] = (kernel, tile
# size, workgroups per CU cap (0 = as many as fit))
TUNE_ORGS = (("faces", 128, 0), ("faces", 256, 0), ("faces", 512, 0), ("fused", 256, 0),
             ("fused", 256, 3), ("fused", 256, 2), ("two-pass", 256, 0))
GRAPH_MODES = ("direct launches", "step-pair graph", "whole-call graph")


def vsw_set_tile_order(h, xcd_order: int):
    return _check(lib().vsw_set_tile_order(h, int(xcd_order)))


def vsw_set_occupancy(h, wg_per_cu: int):
    return _check(lib().vsw_set_occupancy(h, int(wg_per_cu)))


def vsw_autotune(h, steps: int):
    """Returns (chosen configuration, ms per step of every configuration)."""
    chosen = ctypes.c_int32(-1)
    ms = np.empty(VSW_TUNE_CONFIGS)
    _check(lib().vsw_autotune(h, int(steps), ctypes.byref(chosen), _dptr(ms)))
    return chosen.value, ms


def tune_config_name(c: int) -> str:
    kernel, tile, occ = TUNE_ORGS[c // 6]
    return (f"{kernel}, tiles of {tile}" + (", XCD tile order" if (c // 3) % 2 else
            ", index tile order") + ", " + GRAPH_MODES[c % 3]
            + (f", at most {occ} workgroups per CU" if occ else ""))


def vsw_set_graph(h, mode):
    """mode 0 direct launches, 1 (or True) step-pair graph, 2 whole-call graph."""
    return _check(lib().vsw_set_graph(h, int(mode)))


def vsw_set_profiling(h, on: bool):
    return _check(lib().vsw_set_profiling(h, 1 if on else 0))


def vsw_kernel_times(h, nkinds=8):
    ms = np.zeros(nkinds)
    n = np.zeros(nkinds, dtype=np.int64)
    _check(lib().vsw_kernel_times(h, nkinds, _dptr(ms), n.ctypes.data_as(_lp)))
    names = [lib().vsw_kernel_name(i).decode() for i in range(nkinds)]
    return {nm: (float(m), int(c)) for nm, m, c in zip(names, ms, n) if nm}


def vsw_prepare_mesh_host(vx, vy, tri, depth):
    vx, vy, depth = _f64(vx), _f64(vy), _f64(depth)
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    nc = tri.size // 3
    geom = np.empty((7, 3, nc))
    area, perim = np.empty(nc), np.empty(nc)
    nbr = np.empty((3, nc), dtype=np.int32)
    isl = np.empty((3, nc), dtype=np.int32)
    ne, nw = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().vsw_prepare_mesh_host(len(vx), _dptr(vx), _dptr(vy), nc, tri.ctypes.data_as(_ip),
                                       _dptr(depth), _dptr(geom), _dptr(area), _dptr(perim),
                                       nbr.ctypes.data_as(_ip), isl.ctypes.data_as(_ip),
                                       ctypes.byref(ne), ctypes.byref(nw)))
    names = ("nx", "ny", "len", "dx", "dy", "wx", "wy")
    out = {n: geom[i].T.copy() for i, n in enumerate(names)}
    out.update(area=area, perim=perim, nbr=nbr.T.copy(), is_left=isl.T.copy(),
               ne=ne.value, nw=nw.value)
    return out


def vsw_get_permutation(h, nc):
    p = np.empty(nc, dtype=np.int64)
    _check(lib().vsw_get_permutation(h, p.ctypes.data_as(_lp)))
    return p


def vsw_mesh_info(h):
    a, b, c = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib().vsw_mesh_info(h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def vsw_last_error():
    return lib().vsw_last_error().decode()


def vsw_version():
    return lib().vsw_version().decode()


# ---------------------------------------------------------------- wrapper

def make_params(g=9.81, cfl=0.45, h_threshold=1e-3, dt_fixed=0.0,
                ordering=VSW_ORDER_HILBERT, seed=0, precision=VSW_FP64) -> VswParams:
    return VswParams(g, cfl, h_threshold, dt_fixed, precision, ordering, seed)


class Solver:
    """Owns one vsw_solver handle."""

    def __init__(self, g=9.81, cfl=0.45, h_threshold=1e-3, dt_fixed=0.0,
                 ordering=VSW_ORDER_HILBERT, seed=0, device=0, precision=VSW_FP64):
        self.params = make_params(g, cfl, h_threshold, dt_fixed, ordering, seed, precision)
        self.h = vsw_create(self.params, device)
        self.nc = 0

    @classmethod
    def for_case(cls, case, **kw):
        d = dict(g=case.g, cfl=case.cfl, h_threshold=case.h_threshold)
        d.update(kw)
        s = cls(**d)
        s.upload_mesh(case.vx, case.vy, case.tri, case.h)
        s.set_state(case.H, case.HU, case.HV, case.t0)
        return s

    def close(self):
        if self.h is not None:
            vsw_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def upload_mesh(self, vx, vy, tri, depth):
        vsw_upload_mesh(self.h, vx, vy, tri, depth)
        self.nc = int(np.asarray(tri).size // 3)

    def upload_ensemble(self, meshes):
        vsw_upload_ensemble(self.h, meshes)
        self.nc = int(sum(np.asarray(m[2]).size // 3 for m in meshes))

    @classmethod
    def for_ensemble(cls, cases, **kw):
        """One solver over several cases (same g, CFL, H_thr), state set."""
        c0 = cases[0]
        d = dict(g=c0.g, cfl=c0.cfl, h_threshold=c0.h_threshold)
        d.update(kw)
        s = cls(**d)
        s.upload_ensemble([(c.vx, c.vy, c.tri, c.h) for c in cases])
        s.set_state(np.concatenate([c.H for c in cases]), np.concatenate([c.HU for c in cases]),
                    np.concatenate([c.HV for c in cases]), c0.t0)
        return s

    def set_state(self, H, HU, HV, t=0.0):
        vsw_set_state(self.h, H, HU, HV, t)

    def step(self, n, t_stop=math.inf, check=True):
        return vsw_step(self.h, n, t_stop, check)

    def state(self):
        return vsw_get_state(self.h, self.nc)
