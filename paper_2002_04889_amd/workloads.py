"""Seeded synthetic inputs: meshes, bathymetry and initial states.

This module holds input recipes only.  It generates triangle meshes, samples
a bathymetry at cell centroids and evaluates initial conditions.  It contains
none of the finite-volume scheme (no reconstruction, flux, source or time
stepping), so both the GPU library and the CPU oracle can consume its output.

Sign convention (Section 2.1): ``h`` is the still-water depth (positive below
the datum, negative on land), ``z = -h`` is the bed elevation, ``H = h + eta``
is the total depth and ``w = (H, Hu, Hv)`` is the conserved state.

Cases:

* ``thacker_case``   -- radially symmetric oscillating paraboloid (Section 3):
  [0,4]^2 m, bowl z = -h0 (1 - r^2/a^2), h0 = 0.1 m, a = 1 m, r0 = 0.8 m.
* ``basin_case``     -- 500 x 500 km synthetic ocean basin standing in for the
  real-case workload of Section 5 (the Rockall Bank bathymetry is not
  available): 4000 m abyss, linear shelf, dry land strip, Gaussian seamounts,
  2 m Gaussian hump, mesh graded 250 m (coast) to 2 km.
* ``coastal_case``   -- 1000 x 1000 km graded coastal mesh (12M triangles,
  50 m to 5 km, fractal coastline, 15% dry cells, elliptical uplift): the
  workload large enough that its state does not fit in the on-chip caches.
* ``ensemble_cases`` -- 64 basin-style scenarios of 50k to 500k triangles
  (log-uniform), each with its own mesh, seamounts and uplift.
* ``channel_case``   -- long flat channel with a dam over a dry bed, for the
  Ritter closed-form solution.

Every generator is deterministic in its seed: ``numpy.random.SeedSequence``
of ``200204889 + k`` spawned into mesh / bathymetry / initial-condition
streams.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 200204889
GRAVITY = 9.81

# Thacker paraboloid parameters (Section 3).
THACKER_H0 = 0.1
THACKER_ALPHA = 1.0
THACKER_R0 = 0.8
THACKER_L = 4.0


@dataclasses.dataclass
class Case:
    """A complete solver input: mesh, bathymetry, state and run parameters."""

    name: str
    vx: np.ndarray          # float64 [nv]
    vy: np.ndarray          # float64 [nv]
    tri: np.ndarray         # int32 [nc, 3]
    h: np.ndarray           # float64 [nc], still-water depth at centroids
    H: np.ndarray           # float64 [nc]
    HU: np.ndarray          # float64 [nc]
    HV: np.ndarray          # float64 [nc]
    g: float = GRAVITY
    cfl: float = 0.45
    h_threshold: float = 1e-3
    t0: float = 0.0
    t_end: float = math.inf
    info: dict = dataclasses.field(default_factory=dict)

    @property
    def nc(self) -> int:
        return int(self.tri.shape[0])

    @property
    def nv(self) -> int:
        return int(self.vx.shape[0])

    def centroids(self):
        t = self.tri
        cx = (self.vx[t[:, 0]] + self.vx[t[:, 1]] + self.vx[t[:, 2]]) / 3.0
        cy = (self.vy[t[:, 0]] + self.vy[t[:, 1]] + self.vy[t[:, 2]]) / 3.0
        return cx, cy

    def copy(self) -> "Case":
        return dataclasses.replace(
            self, vx=self.vx.copy(), vy=self.vy.copy(), tri=self.tri.copy(),
            h=self.h.copy(), H=self.H.copy(), HU=self.HU.copy(),
            HV=self.HV.copy(), info=dict(self.info))


def streams(k: int):
    """Independent (mesh, bathymetry, initial-condition) generators for case k."""
    ss = np.random.SeedSequence(SEED_BASE + k)
    return [np.random.default_rng(s) for s in ss.spawn(3)]


def _delaunay(px: np.ndarray, py: np.ndarray):
    from scipy.spatial import Delaunay

    pts = np.stack([px, py], axis=1)
    d = Delaunay(pts)
    tri = np.ascontiguousarray(d.simplices.astype(np.int32))
    # Drop vertices that the triangulation did not use (none expected).
    used = np.zeros(len(px), dtype=bool)
    used[tri.ravel()] = True
    if not used.all():
        remap = -np.ones(len(px), dtype=np.int64)
        remap[used] = np.arange(int(used.sum()))
        tri = remap[tri].astype(np.int32)
        px, py = px[used], py[used]
    return np.ascontiguousarray(px), np.ascontiguousarray(py), tri


def jittered_grid(nx: int, ny: int, lx: float, ly: float, rng, jitter=0.3):
    """nx x ny grid on [0,lx]x[0,ly]; interior points jittered in both
    directions, edge points only along their edge, corners fixed."""
    sx, sy = lx / (nx - 1), ly / (ny - 1)
    gx = np.linspace(0.0, lx, nx)
    gy = np.linspace(0.0, ly, ny)
    X, Y = np.meshgrid(gx, gy, indexing="ij")
    jx = rng.uniform(-jitter, jitter, X.shape) * sx
    jy = rng.uniform(-jitter, jitter, Y.shape) * sy
    on_x_edge = np.zeros(X.shape, dtype=bool)
    on_x_edge[0, :] = on_x_edge[-1, :] = True
    on_y_edge = np.zeros(X.shape, dtype=bool)
    on_y_edge[:, 0] = on_y_edge[:, -1] = True
    jx[on_x_edge] = 0.0
    jy[on_y_edge] = 0.0
    return (X + jx).ravel(), (Y + jy).ravel()


# ---------------------------------------------------------------- Thacker

def thacker_constants(g: float = GRAVITY):
    a, r0, h0 = THACKER_ALPHA, THACKER_R0, THACKER_H0
    A = (a * a - r0 * r0) / (a * a + r0 * r0)
    omega = math.sqrt(8.0 * g * h0) / a
    return {"A": A, "omega": omega, "T1": 2.0 * math.pi / omega,
            "h0": h0, "alpha": a, "r0": r0, "L": THACKER_L}


def thacker_exact(x, y, t, g: float = GRAVITY):
    """Closed-form Thacker solution (Section 3) at points (x, y) in [0,L]^2.

    Returns (eta, H, u, v).  The printed expression for "h(r,t)" subtracts
    the bed elevation, so it is the total depth; it is clipped at zero where
    the bowl is dry.  eta = H + z where wet and eta = z on dry ground."""
    c = thacker_constants(g)
    A, om, h0, a, L = c["A"], c["omega"], c["h0"], c["alpha"], c["L"]
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    xc, yc = x - L / 2.0, y - L / 2.0
    r2 = xc * xc + yc * yc
    den = 1.0 - A * math.cos(om * t)
    z = -h0 * (1.0 - r2 / (a * a))
    eta_w = h0 * (math.sqrt(1.0 - A * A) / den - 1.0
                  - r2 / (a * a) * ((1.0 - A * A) / (den * den) - 1.0))
    H = np.maximum(0.0, eta_w - z)
    wet = H > 0.0
    eta = np.where(wet, eta_w, z)
    fac = om * A * math.sin(om * t) / (2.0 * den)
    u = np.where(wet, fac * xc, 0.0)
    v = np.where(wet, fac * yc, 0.0)
    return eta, H, u, v


def thacker_case(n: int = 45, k: int = 0, t_end=None, still: bool = False,
                 cfl: float = 0.45, h_threshold: float = 1e-5) -> Case:
    """Thacker paraboloid on a seeded jittered n x n Delaunay mesh.

    ``still=True`` gives the lake-at-rest variant (eta = 0 in the bowl, dry
    rim) used for the well-balancing invariant."""
    rm, _, _ = streams(k)
    px, py = jittered_grid(n, n, THACKER_L, THACKER_L, rm)
    vx, vy, tri = _delaunay(px, py)
    cx = (vx[tri[:, 0]] + vx[tri[:, 1]] + vx[tri[:, 2]]) / 3.0
    cy = (vy[tri[:, 0]] + vy[tri[:, 1]] + vy[tri[:, 2]]) / 3.0
    r2 = (cx - 2.0) ** 2 + (cy - 2.0) ** 2
    h = THACKER_H0 * (1.0 - r2 / THACKER_ALPHA ** 2)
    c = thacker_constants()
    if still:
        H = np.maximum(0.0, h)
        HU = np.zeros_like(H)
        HV = np.zeros_like(H)
    else:
        _, H, u, v = thacker_exact(cx, cy, 0.0)
        HU, HV = H * u, H * v
    return Case(name=f"thacker{n}" + ("-still" if still else ""),
                vx=vx, vy=vy, tri=tri, h=h, H=H, HU=HU, HV=HV,
                cfl=cfl, h_threshold=h_threshold,
                t_end=c["T1"] if t_end is None else t_end,
                info={"n": n, "seed": SEED_BASE + k, **c})


# ---------------------------------------------------------------- basin

BASIN_L = 500e3
BASIN_SHORE_X = 480e3
BASIN_SHELF_X = 380e3


def _graded_columns(lx, ly, size_fn, rng, jitter=0.3):
    """Points in columns whose spacing follows size_fn(x) in both directions.

    Columns sit at x_0 = 0, x_{i+1} = x_i + size_fn(x_i), plus a last column
    at x = lx.  Each column holds evenly spaced points in y at the local size.
    Interior points are jittered in x and y; points on the boundary move only
    along it, corners not at all."""
    xs = [0.0]
    while xs[-1] + size_fn(xs[-1]) < lx - 0.5 * size_fn(lx):
        xs.append(xs[-1] + size_fn(xs[-1]))
    xs.append(lx)
    xs = np.array(xs)
    pxs, pys = [], []
    ncol = len(xs)
    for i, x in enumerate(xs):
        ny = max(2, int(round(ly / size_fn(x))) + 1)
        y = np.linspace(0.0, ly, ny)
        dy = ly / (ny - 1)
        jy = rng.uniform(-jitter, jitter, ny) * dy
        jy[0] = jy[-1] = 0.0
        if 0 < i < ncol - 1:
            sx = min(xs[i] - xs[i - 1], xs[i + 1] - xs[i])
            jx = rng.uniform(-jitter, jitter, ny) * sx
        else:
            jx = np.zeros(ny)
        pxs.append(x + jx)
        pys.append(y + jy)
    return np.concatenate(pxs), np.concatenate(pys)


def basin_size_field(k_grade: float, smin=250.0, smax=2000.0):
    def size(x):
        d = abs(x - BASIN_SHORE_X)
        return min(smax, smin + k_grade * d)
    return size


def basin_bed(x, y, mounts):
    """Bed elevation z (m) of the synthetic basin: abyss, shelf, land strip
    and Gaussian seamounts."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.where(x < BASIN_SHELF_X, -4000.0,
                 np.where(x < BASIN_SHORE_X,
                          -4000.0 * (BASIN_SHORE_X - x) / (BASIN_SHORE_X - BASIN_SHELF_X),
                          100.0 * (x - BASIN_SHORE_X) / (BASIN_L - BASIN_SHORE_X)))
    for (mx, my, amp, sig) in mounts:
        z = z + amp * np.exp(-((x - mx) ** 2 + (y - my) ** 2) / (2.0 * sig * sig))
    return z


# Grading slope tuned so the default basin lands within 5% of 1M triangles.
BASIN_K_1M = 0.0047


def basin_case(k_grade: float = BASIN_K_1M, k: int = 1, smin: float = 250.0,
               smax: float = 2000.0, scale: float = 1.0, eta_amp: float = 2.0,
               cfl: float = 0.45, h_threshold: float = 1e-3,
               n_mounts: int = 12, hump=None) -> Case:
    """Synthetic 500 x 500 km ocean basin (stand-in for the real case).

    ``scale`` multiplies both mesh sizes (not the grading slope), which gives
    small meshes of the same shape for tests (scale=8 gives about 61k
    triangles; scaling k_grade too scales the whole size field).  ``eta_amp=0`` is the
    lake-at-rest variant.  ``hump`` = (x0, y0, amplitude, sigma) replaces the
    default Gaussian initial hump (200 km, 250 km, eta_amp, 20 km)."""
    rm, rb, ri = streams(k)
    size = basin_size_field(k_grade, smin * scale, smax * scale)
    px, py = _graded_columns(BASIN_L, BASIN_L, size, rm)
    vx, vy, tri = _delaunay(px, py)
    mounts = []
    for _ in range(n_mounts):
        mx = rb.uniform(20e3, 360e3)
        my = rb.uniform(20e3, 480e3)
        amp = rb.uniform(1000.0, 3500.0)
        sig = rb.uniform(5e3, 25e3)
        mounts.append((mx, my, amp, sig))
    cx = (vx[tri[:, 0]] + vx[tri[:, 1]] + vx[tri[:, 2]]) / 3.0
    cy = (vy[tri[:, 0]] + vy[tri[:, 1]] + vy[tri[:, 2]]) / 3.0
    z = basin_bed(cx, cy, mounts)
    h = -z
    hx, hy, ha, sig0 = hump if hump is not None else (200e3, 250e3, eta_amp, 20e3)
    eta0 = ha * np.exp(-((cx - hx) ** 2 + (cy - hy) ** 2) / (2.0 * sig0 * sig0))
    H = np.maximum(0.0, eta0 + h)
    HU = np.zeros_like(H)
    HV = np.zeros_like(H)
    return Case(name=f"basin{len(tri)}", vx=vx, vy=vy, tri=tri, h=h, H=H,
                HU=HU, HV=HV, cfl=cfl, h_threshold=h_threshold,
                info={"k_grade": k_grade, "scale": scale, "seed": SEED_BASE + k,
                      "mounts": mounts, "eta_amp": eta_amp})


# ---------------------------------------------------------------- ensemble

def ensemble_cases(n_scen: int = 64, nmin: float = 5e4, nmax: float = 5e5, k: int = 3,
                   size_scale: float = 1.0, log=None):
    """Uneven-size scenario ensemble of basin-style meshes.

    Scenario i: target size N_i = round(exp U(ln nmin, ln nmax)) triangles
    (log-uniform), a basin whose whole size field is scaled by sqrt(1M / N_i)
    (times ``size_scale``), with its own mesh, seamount and point seeds
    (stream 1000 + i) and its own Gaussian uplift: centre U(50, 350) x
    U(50, 450) km, amplitude U(0.5, 5) m, width sigma U(10, 40) km.
    Returns the list of cases and the drawn parameters."""
    import os

    rng = np.random.default_rng(SEED_BASE + k)
    targets = np.round(np.exp(rng.uniform(math.log(nmin), math.log(nmax), n_scen))).astype(int)
    humps = [(rng.uniform(50e3, 350e3), rng.uniform(50e3, 450e3), rng.uniform(0.5, 5.0),
              rng.uniform(10e3, 40e3)) for _ in range(n_scen)]
    info = {"targets": targets.tolist(), "humps": humps}
    cache = os.environ.get("VSW_CASE_CACHE")
    path = (os.path.join(cache, f"ensemble_k{k}_{n_scen}_{nmin:g}_{nmax:g}_{size_scale:g}.npz")
            if cache else None)
    if path and os.path.exists(path):
        z = np.load(path)
        cases = []
        for i in range(n_scen):
            v0, v1, c0, c1 = z["voff"][i], z["voff"][i + 1], z["coff"][i], z["coff"][i + 1]
            c = Case(name=f"ens{i}-{c1 - c0}", vx=z["vx"][v0:v1], vy=z["vy"][v0:v1],
                     tri=z["tri"][c0:c1], h=z["h"][c0:c1], H=z["H"][c0:c1],
                     HU=np.zeros(c1 - c0), HV=np.zeros(c1 - c0))
            cases.append(c)
        return cases, info
    cases = []
    for i in range(n_scen):
        sc = math.sqrt(1.0e6 / targets[i]) * size_scale
        c = basin_case(k_grade=BASIN_K_1M * sc, k=1000 + i, scale=sc, hump=humps[i])
        c.name = f"ens{i}-{c.nc}"
        cases.append(c)
        if log:
            log(f"ensemble scenario {i}: {c.nc} cells (target {targets[i]})")
    if path:
        os.makedirs(cache, exist_ok=True)
        voff = np.cumsum([0] + [c.nv for c in cases])
        coff = np.cumsum([0] + [c.nc for c in cases])
        np.savez(path + ".tmp.npz", voff=voff, coff=coff,
                 vx=np.concatenate([c.vx for c in cases]), vy=np.concatenate([c.vy for c in cases]),
                 tri=np.concatenate([c.tri for c in cases]), h=np.concatenate([c.h for c in cases]),
                 H=np.concatenate([c.H for c in cases]))
        os.replace(path + ".tmp.npz", path)
    return cases, info


# ---------------------------------------------------------------- channel

def channel_case(length: float = 100.0, width: float = 2.0, n_len: int = 401,
                 n_wid: int = 9, x_dam: float = 50.0, H0: float = 1.0, k: int = 5,
                 cfl: float = 0.45, h_threshold: float = 1e-6) -> Case:
    """Flat-bed channel (h = 0) with water H0 for x < x_dam and a dry bed
    beyond: the dry dam break whose exact solution is Ritter's."""
    rm, _, _ = streams(k)
    px, py = jittered_grid(n_len, n_wid, length, width, rm, jitter=0.2)
    vx, vy, tri = _delaunay(px, py)
    cx = (vx[tri[:, 0]] + vx[tri[:, 1]] + vx[tri[:, 2]]) / 3.0
    h = np.zeros(len(tri))
    H = np.where(cx < x_dam, H0, 0.0)
    return Case(name=f"channel{len(tri)}", vx=vx, vy=vy, tri=tri, h=h, H=H,
                HU=np.zeros_like(H), HV=np.zeros_like(H), cfl=cfl,
                h_threshold=h_threshold,
                info={"x_dam": x_dam, "H0": H0, "length": length, "width": width})


# ---------------------------------------------------------------- wave

def standing_wave_case(n: int = 45, amp: float = 1e-6, depth: float = 1.0,
                       length: float = 4.0, k: int = 7, cfl: float = 0.45,
                       h_threshold: float = 1e-6) -> Case:
    """Flat basin of depth ``depth`` on [0,L]^2 with the lowest wall-bounded
    standing mode eta = amp cos(pi x / L) at rest: a smooth, everywhere wet
    state (no wet/dry front) for convergence checks."""
    rm, _, _ = streams(k)
    px, py = jittered_grid(n, n, length, length, rm)
    vx, vy, tri = _delaunay(px, py)
    cx = (vx[tri[:, 0]] + vx[tri[:, 1]] + vx[tri[:, 2]]) / 3.0
    h = np.full(len(tri), depth)
    H = depth + amp * np.cos(math.pi * cx / length)
    return Case(name=f"wave{n}", vx=vx, vy=vy, tri=tri, h=h, H=H,
                HU=np.zeros_like(H), HV=np.zeros_like(H), cfl=cfl,
                h_threshold=h_threshold,
                info={"amp": amp, "depth": depth, "length": length})


# ---------------------------------------------------------------- tiny meshes

def tiny_mesh(kind: str = "square2"):
    """Hand-made meshes: 'square2' (2 triangles), 'square8' (8 triangles
    around a centre vertex of a 2x2 patch)."""
    if kind == "square2":
        vx = np.array([0.0, 1.0, 1.0, 0.0])
        vy = np.array([0.0, 0.0, 1.0, 1.0])
        tri = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    elif kind == "square8":
        vx = np.array([0.0, 1.0, 2.0, 0.0, 1.0, 2.0, 0.0, 1.0, 2.0])
        vy = np.array([0.0, 0.0, 0.0, 1.0, 1.0, 1.0, 2.0, 2.0, 2.0])
        tri = np.array([[0, 1, 4], [0, 4, 3], [1, 2, 4], [2, 5, 4],
                        [3, 4, 6], [4, 7, 6], [4, 5, 8], [4, 8, 7]], dtype=np.int32)
    else:
        raise ValueError(kind)
    return vx, vy, tri


# ---------------------------------------------------------------- coastal

COAST_L = 1000e3
COAST_X0 = 800e3
COAST_AMP = 40e3
COAST_SHELF = 250e3


def fbm_1d(t, rng, hurst=0.6, octaves=10):
    """Seeded fractional-Brownian-like noise on t in [0, 1]: value noise with
    cosine interpolation, octave o on 2^o + 1 knots with amplitude 2^(-hurst o),
    scaled so that max |f| = 1 over the knots of the finest octave."""
    t = np.asarray(t, dtype=np.float64)
    f = np.zeros_like(t)
    for o in range(octaves):
        n = 2 ** o
        knots = rng.uniform(-1.0, 1.0, n + 1)
        u = t * n
        i = np.clip(np.floor(u).astype(np.int64), 0, n - 1)
        a = u - i
        w = 0.5 - 0.5 * np.cos(math.pi * a)
        f += 2.0 ** (-hurst * o) * ((1.0 - w) * knots[i] + w * knots[i + 1])
    return f


def value_noise_2d(x, y, rng, lx, octaves=8, base=8, hurst=0.6):
    """Seeded 2D value noise (bilinear, cosine-smoothed) summed over octaves,
    normalised by the sum of the octave amplitudes to lie in [-1, 1]."""
    x = np.asarray(x, dtype=np.float64) / lx
    y = np.asarray(y, dtype=np.float64) / lx
    f = np.zeros_like(x)
    tot = 0.0
    for o in range(octaves):
        n = base * 2 ** o
        g = rng.uniform(-1.0, 1.0, (n + 1, n + 1))
        u, v = np.clip(x * n, 0, n - 1e-9), np.clip(y * n, 0, n - 1e-9)
        i, j = u.astype(np.int64), v.astype(np.int64)
        a = 0.5 - 0.5 * np.cos(math.pi * (u - i))
        b = 0.5 - 0.5 * np.cos(math.pi * (v - j))
        amp = 2.0 ** (-hurst * o)
        f += amp * ((1 - a) * (1 - b) * g[i, j] + a * (1 - b) * g[i + 1, j]
                    + (1 - a) * b * g[i, j + 1] + a * b * g[i + 1, j + 1])
        tot += amp
    return f / tot


def _quadtree_points(L, size_fn, s0, max_level, rng, jitter=0.3):
    """Points graded by a size field on [0, L]^2 from a quadtree of square
    blocks: a block of side s is split while the target size at its centre is
    below s / sqrt(2) (down to max_level), and each leaf holds one point at its
    centre jittered by at most jitter * s.  Leaves on the domain boundary add
    their corners on that boundary, so the hull is the exact square."""
    n0 = int(round(L / s0))
    s = L / n0
    ix, iy = np.meshgrid(np.arange(n0), np.arange(n0), indexing="ij")
    bx = (ix.ravel() + 0.5) * s
    by = (iy.ravel() + 0.5) * s
    px, py, ex, ey = [], [], [], []
    for lev in range(max_level + 1):
        want = size_fn(bx, by)
        split = want < s / math.sqrt(2.0) if lev < max_level else np.zeros(len(bx), bool)
        lx, ly = bx[~split], by[~split]
        px.append(lx + rng.uniform(-jitter, jitter, len(lx)) * s)
        py.append(ly + rng.uniform(-jitter, jitter, len(ly)) * s)
        h = 0.5 * s
        for side in (0, 1):
            c = (lx, ly)[side]
            o = (ly, lx)[side]
            for edge in (0.0, L):
                on = np.abs(c - edge) < h * 1.0001
                for sgn in (-1.0, 1.0):
                    e_c = np.full(int(on.sum()), edge)
                    e_o = o[on] + sgn * h
                    if side == 0:
                        ex.append(e_c); ey.append(e_o)
                    else:
                        ex.append(e_o); ey.append(e_c)
        sx, sy = bx[split], by[split]
        q = 0.25 * s
        bx = np.concatenate([sx - q, sx + q, sx - q, sx + q])
        by = np.concatenate([sy - q, sy - q, sy + q, sy + q])
        s *= 0.5
        if len(bx) == 0:
            break
    bxy = np.unique(np.round(np.stack([np.concatenate(ex), np.concatenate(ey)], 1), 3), axis=0)
    return (np.concatenate(px + [bxy[:, 0]]), np.concatenate(py + [bxy[:, 1]]))


# Grading slopes (seaward, landward) tuned so the default coastal mesh has
# 12M triangles within 5% and 15% of them dry at t = 0.
COAST_K_SEA = 0.00455
COAST_K_LAND = 0.0261


def coastal_case(k_sea: float = COAST_K_SEA, k_land: float = COAST_K_LAND, k: int = 2,
                 smin: float = 50.0, smax: float = 5000.0, scale: float = 1.0,
                 uplift: float = 3.0, cfl: float = 0.45, h_threshold: float = 1e-3,
                 ordering_seed=None, log=None) -> Case:
    """Large graded coastal mesh on 1000 x 1000 km (see _coastal_base).

    ``ordering_seed`` shuffles the triangles with a seeded permutation (the
    random-ordering variant of the same mesh).  If the environment variable
    VSW_CASE_CACHE names a directory, the generated mesh and state are kept
    there as .npz and reused (generation of the 12M-cell mesh takes minutes).
    ``log`` (a print-like callable) receives progress lines."""
    import os

    key = f"coastal_k{k}_{k_sea:g}_{k_land:g}_{smin:g}_{smax:g}_{scale:g}_{uplift:g}"
    cache = os.environ.get("VSW_CASE_CACHE")
    path = os.path.join(cache, key + ".npz") if cache else None
    if path and os.path.exists(path):
        z = np.load(path)
        vx, vy, tri, h, H = z["vx"], z["vy"], z["tri"], z["h"], z["H"]
    else:
        vx, vy, tri, h, H = _coastal_base(k_sea, k_land, k, smin, smax, scale, uplift,
                                          log or (lambda *a: None))
        if path:
            os.makedirs(cache, exist_ok=True)
            np.savez(path + ".tmp.npz", vx=vx, vy=vy, tri=tri, h=h, H=H)
            os.replace(path + ".tmp.npz", path)
    if ordering_seed is not None:
        p = np.random.default_rng(ordering_seed).permutation(len(tri))
        tri, h, H = np.ascontiguousarray(tri[p]), h[p], H[p]
    return Case(name=f"coastal{len(tri)}", vx=vx, vy=vy, tri=tri, h=h, H=H,
                HU=np.zeros_like(H), HV=np.zeros_like(H), cfl=cfl, h_threshold=h_threshold,
                info={"k_sea": k_sea, "k_land": k_land, "scale": scale, "seed": SEED_BASE + k,
                      "dry_fraction": float(np.mean(H < h_threshold)),
                      "ordering_seed": ordering_seed})


def _coastal_base(k_sea, k_land, k, smin, smax, scale, uplift, log):
    """Large graded coastal mesh on 1000 x 1000 km (the HBM-roofline workload).

    Coastline x_c(y) = 800 km + 40 km f(y) with f seeded fractal noise (Hurst
    0.6, 10 octaves).  Bed: 4000 m abyss, linear shelf over the 250 km before
    the coast, land rising 2 m/km beyond it, plus +-20 m of 2D fractal bed
    noise within 15 km of the coast.  Mesh size min(5 km, 50 m + k d) with d
    the distance to the coastline (k_sea seaward, k_land landward; ``scale``
    multiplies both sizes).  Initial free surface: a cos^2-tapered elliptical
    uplift with semi-axes 30 km (x) and 75 km (y), 3 m peak, centre (650, 500)
    km; at rest.  Returns (vx, vy, tri, h, H)."""
    from scipy.spatial import cKDTree

    rm, rb, ri = streams(k)
    ycs = np.linspace(0.0, 1.0, 40001)
    xcs = COAST_X0 + COAST_AMP * fbm_1d(ycs, rm)
    ycs = ycs * COAST_L
    tree = cKDTree(np.stack([xcs, ycs], 1))
    coarse = cKDTree(np.stack([xcs[::40], ycs[::40]], 1))   # 1 km samples

    def coast_x(y):
        return np.interp(y, ycs, xcs)

    def coast_dist(x, y):
        """Distance to the coastline: 25 m samples within 25 km of it, 1 km
        samples (error below 1 km) farther out."""
        q = np.stack([x, y], 1)
        d, _ = coarse.query(q, workers=-1)
        near = d < 25e3
        dn, _ = tree.query(q[near], workers=-1, distance_upper_bound=26e3)
        d[near] = np.minimum(d[near], dn)
        return d

    def size(x, y):
        d = coast_dist(x, y)
        kk = np.where(x < coast_x(y), k_sea, k_land)
        return np.minimum(smax * scale, (smin + kk * d) * scale)

    px, py = _quadtree_points(COAST_L, size, smax * scale, 16, rm)
    log(f"coastal mesh: {len(px)} points, triangulating")
    vx, vy, tri = _delaunay(px, py)
    log(f"coastal mesh: {len(tri)} triangles, bathymetry")
    cx = (vx[tri[:, 0]] + vx[tri[:, 1]] + vx[tri[:, 2]]) / 3.0
    cy = (vy[tri[:, 0]] + vy[tri[:, 1]] + vy[tri[:, 2]]) / 3.0
    xi = coast_x(cy) - cx                       # > 0 at sea
    h = np.where(xi > 0, 4000.0 * np.minimum(1.0, xi / COAST_SHELF), 2e-3 * xi)
    d = coast_dist(cx, cy)
    band = np.clip(1.0 - d / 15e3, 0.0, 1.0)
    h = h - 20.0 * band * value_noise_2d(cx, cy, rb, COAST_L)
    rho = np.sqrt(((cx - 650e3) / 30e3) ** 2 + ((cy - 500e3) / 75e3) ** 2)
    eta0 = np.where(rho < 1.0, uplift * np.cos(0.5 * math.pi * np.minimum(rho, 1.0)) ** 2, 0.0)
    H = np.maximum(0.0, eta0 + h)
    return vx, vy, tri, h, H
