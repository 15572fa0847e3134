"""Pins of the differentiable (PyTorch CPU, FP64) statement of the scheme,
which supplies the tape gradient for the GPU adjoint: its forward equals the
C oracle (residual and whole steps), and its tape gradient agrees with
central finite differences of its own forward in smooth wet directions.
CPU only."""
import numpy as np
import pytest
import torch

from oracle import torch_scheme as TS
from paper_2002_04889_amd import workloads as W


def _setup(orc, case):
    m = orc.Mesh.from_case(case)
    G = TS.Geometry(m)
    t = lambda a: torch.tensor(np.asarray(a, dtype=np.float64))
    return m, G, t


@pytest.mark.parametrize("which", ["thacker", "basin"])
def test_residual_equals_c_oracle(orc, which):
    c = W.thacker_case(23) if which == "thacker" else W.basin_case(scale=32)
    m, G, t = _setup(orc, c)
    p = orc.params(g=c.g, cfl=c.cfl, h_threshold=c.h_threshold)
    # a state with motion: a few oracle steps first
    r = m.run(p, c.H, c.HU, c.HV, 0.0, 15)
    R_c = m.residual(p, r["H"], r["HU"], r["HV"])
    R_t = TS.residual(G, t(r["H"]), t(r["HU"]), t(r["HV"]), t(c.h), c.g, c.h_threshold)
    for a, b in zip(R_c, R_t):
        assert np.array_equal(a, b.numpy())


@pytest.mark.parametrize("which", ["thacker", "basin"])
def test_steps_equal_c_oracle(orc, which):
    c = W.thacker_case(23) if which == "thacker" else W.basin_case(scale=32)
    m, G, t = _setup(orc, c)
    p = orc.params(g=c.g, cfl=c.cfl, h_threshold=c.h_threshold)
    r = m.run(p, c.H, c.HU, c.HV, 0.0, 25)
    H, HU, HV, h = t(c.H), t(c.HU), t(c.HV), t(c.h)
    dts = []
    for _ in range(25):
        H, HU, HV, dt = TS.step(G, H, HU, HV, h, c.g, c.h_threshold, c.cfl)
        dts.append(float(dt))
    assert np.array_equal(np.array(dts), r["dts"])
    for k, v in (("H", H), ("HU", HU), ("HV", HV)):
        assert np.array_equal(v.numpy(), r[k]), k


def generic_basin(scale=32, seed=1, rough_bed=0.0):
    """The basin with random depth (0-1 m), bed (0-1 m) and momentum
    (+-1 m^2/s) noise on its wet cells: no two values tie in the CFL
    minimum, a limiter's max/min or the hydrostatic reconstruction's
    min(h_L, h_R), where the scheme is only one-sided differentiable (the
    plain basin's flat abyss at rest is full of such ties).  rough_bed > 0
    adds that much more bed noise (0 to rough_bed m) with the surface kept,
    so neighbouring depths stay apart by more than a bed perturbation moves
    them (fine meshes)."""
    c = W.basin_case(scale=scale)
    rng = np.random.default_rng(seed)
    wet = c.H > 10.0
    c.h = c.h + wet * rng.uniform(0.0, 1.0, c.nc)
    c.H = c.H + wet * rng.uniform(0.0, 1.0, c.nc)
    if rough_bed > 0.0:
        b = wet * rng.uniform(0.0, rough_bed, c.nc)
        c.h = c.h + b
        c.H = c.H + b
    c.HU = wet * rng.uniform(-1.0, 1.0, c.nc)
    c.HV = wet * rng.uniform(-1.0, 1.0, c.nc)
    return c


@pytest.mark.parametrize("dt_mode", ["cfl", "fixed"])
def test_tape_gradient_matches_finite_differences(orc, dt_mode):
    """Directional derivative of the gauge loss along smooth directions of
    the initial surface (wet cells) and of the bed, against central
    differences of the same forward, from a generic state."""
    c = generic_basin()
    m, G, t = _setup(orc, c)
    rng = np.random.default_rng(2)
    wet = np.flatnonzero(c.H > 10.0)
    gauges = rng.choice(wet, 5, replace=False)
    nsteps = 12
    obs = rng.normal(0.0, 0.5, (nsteps, 5))
    cx, cy = c.centroids()
    dt_fixed = 0.0 if dt_mode == "cfl" else 2.0

    def loss(H0, h):
        L, _ = TS.gauge_loss(G, H0, t(c.HU), t(c.HV), h, nsteps, gauges, obs, c.g,
                             c.h_threshold, c.cfl, dt_fixed)
        return L

    H0 = t(c.H).requires_grad_(True)
    h = t(c.h).requires_grad_(True)
    L = loss(H0, h)
    gH, gh = torch.autograd.grad(L, (H0, h))
    for k in range(3):
        # smooth bump in the wet interior
        x0, y0 = rng.uniform(100e3, 300e3), rng.uniform(100e3, 400e3)
        v = np.exp(-((cx - x0) ** 2 + (cy - y0) ** 2) / (2 * 40e3 ** 2)) * (c.H > 10.0)
        vt = t(v)
        for which, grad in (("eta0", gH), ("bed", gh)):
            # eta = H - h at 4000 m depth carries ~5e-13 m of round-off, which
            # swamps differences with small steps, while a large step meets
            # the limiter's and the upwind choice's kinks: take the best of
            # three steps (the differences approach the derivative as the
            # step shrinks until round-off takes over).  The bed direction
            # moves h and H together; its response is ~1e5 times weaker, so
            # it takes metre steps and a 1e-5 bar.
            if which == "bed":
                grad = gH + gh
                steps, tol = (3.0, 1.0, 0.3), 1e-5
            else:
                steps, tol = (1e-2, 1e-3, 1e-4), 1e-6
            ad = float((grad * vt).sum())
            scale = float((grad * vt).abs().sum())
            errs = []
            for eps in steps:
                if which == "eta0":
                    Lp = loss(t(c.H) + eps * vt, t(c.h))
                    Lm = loss(t(c.H) - eps * vt, t(c.h))
                else:
                    Lp = loss(t(c.H) + eps * vt, t(c.h) + eps * vt)
                    Lm = loss(t(c.H) - eps * vt, t(c.h) - eps * vt)
                errs.append(abs(float((Lp - Lm) / (2 * eps)) - ad))
            assert min(errs) <= tol * scale, (which, k, errs, ad, scale)
