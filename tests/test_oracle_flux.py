"""Pins of the oracle's per-face numerics against what the paper and the
mathematics fix, independent of the oracle's own formulas:

* consistency: identical states give the physical flux (Section 2.2 states
  this requirement of the numerical flux);
* conservation: the flux seen from the other side is the exact negative;
* Rankine-Hugoniot: the HLL star flux F* and the star state w* printed in
  Section 2.2 satisfy both jump conditions F* = F_L + s_L (w* - w_L) and
  F* = F_R + s_R (w* - w_R);
* Riemann invariants: the wave-speed estimates u*, c* of Section 2.2 are the
  two-rarefaction solution, u* + 2c* = u_nL + 2c_L and u* - 2c* = u_nR - 2c_R
  (textbook shallow-water invariants);
* upwinding: s_L >= 0 gives F_L, s_R < 0 gives F_R;
* rotation invariance of the flux;
* a wall face (Section 2.5) carries exactly zero mass flux;
* hydrostatic reconstruction keeps a lake at rest: equal surfaces and zero
  velocity give a face flux that balances the pressure of each side.
"""
import math

import numpy as np
import pytest

G = 9.81


def phys_flux(H, u, v, nx, ny):
    """Physical flux of the shallow water equations (Section 2.1) dotted
    with n: (H u.n, H u u.n + g/2 H^2 n_x, H v u.n + g/2 H^2 n_y)."""
    un = u * nx + v * ny
    return np.array([H * un, H * u * un + 0.5 * G * H * H * nx,
                     H * v * un + 0.5 * G * H * H * ny])


def rand_state(rng, dry_frac=0.0):
    H = rng.uniform(0.01, 5.0)
    if rng.random() < dry_frac:
        H = 0.0
    return np.array([H, rng.normal(0, 2.0), rng.normal(0, 2.0)])


def rand_normal(rng):
    a = rng.uniform(0, 2 * math.pi)
    return math.cos(a), math.sin(a)


def test_consistency(orc):
    rng = np.random.default_rng(11)
    for _ in range(2000):
        w = rand_state(rng)
        nx, ny = rand_normal(rng)
        phi, _ = orc.hll(G, w, w, nx, ny)
        ref = phys_flux(w[0], w[1], w[2], nx, ny)
        scale = np.abs(ref).max() + w[0] * math.sqrt(G * w[0])
        assert np.abs(phi - ref).max() <= 1e-14 * scale


def test_conservation_antisymmetry(orc):
    rng = np.random.default_rng(12)
    for _ in range(2000):
        wl, wr = rand_state(rng, 0.1), rand_state(rng, 0.1)
        nx, ny = rand_normal(rng)
        a, _ = orc.hll(G, wl, wr, nx, ny)
        b, _ = orc.hll(G, wr, wl, -nx, -ny)
        scale = 1.0 + np.abs(a).max()
        assert np.abs(a + b).max() <= 1e-14 * scale


def test_rankine_hugoniot_of_star_flux(orc):
    rng = np.random.default_rng(13)
    hits = 0
    for _ in range(3000):
        wl, wr = rand_state(rng), rand_state(rng)
        nx, ny = rand_normal(rng)
        phi, (sl, sr, _, _) = orc.hll(G, wl, wr, nx, ny)
        if not (sl < 0.0 <= sr):
            continue
        hits += 1
        cons = lambda w: np.array([w[0], w[0] * w[1], w[0] * w[2]])
        UL, UR = cons(wl), cons(wr)
        FL = phys_flux(*wl, nx, ny)
        FR = phys_flux(*wr, nx, ny)
        # star state as printed in Section 2.2
        wstar = (sr * UR - sl * UL - (FR - FL)) / (sr - sl)
        scale = 1.0 + np.abs(FL).max() + np.abs(FR).max() + abs(sl * sr) * np.abs(UR - UL).max()
        assert np.abs(phi - (FL + sl * (wstar - UL))).max() <= 1e-12 * scale
        assert np.abs(phi - (FR + sr * (wstar - UR))).max() <= 1e-12 * scale
    assert hits > 1000


def test_wave_speeds_are_two_rarefaction_solution(orc):
    rng = np.random.default_rng(14)
    for _ in range(2000):
        wl, wr = rand_state(rng), rand_state(rng)
        nx, ny = rand_normal(rng)
        _, (sl, sr, us, cs) = orc.hll(G, wl, wr, nx, ny)
        unl = wl[1] * nx + wl[2] * ny
        unr = wr[1] * nx + wr[2] * ny
        cl, cr = math.sqrt(G * wl[0]), math.sqrt(G * wr[0])
        sc = 1.0 + abs(unl) + abs(unr) + cl + cr
        # Riemann invariants across the left and right rarefactions
        assert abs((us + 2 * cs) - (unl + 2 * cl)) <= 1e-14 * sc
        assert abs((us - 2 * cs) - (unr - 2 * cr)) <= 1e-14 * sc
        # the speeds bound both the star and the side characteristics
        assert sl == min(unl - cl, us - cs)
        assert sr == max(us + cs, unr + cr)
        assert sl < sr


def test_dry_side_speeds(orc):
    """One dry side: the front moves at u + 2c (dry bed to the right) or
    u - 2c (dry bed to the left), the speed of Ritter's dam-break front."""
    rng = np.random.default_rng(15)
    for _ in range(500):
        w = rand_state(rng)
        dry = np.array([0.0, 0.0, 0.0])
        nx, ny = rand_normal(rng)
        un = w[1] * nx + w[2] * ny
        c = math.sqrt(G * w[0])
        _, (sl, sr, _, _) = orc.hll(G, w, dry, nx, ny)
        assert sl == un - c and sr == un + 2 * c
        _, (sl, sr, _, _) = orc.hll(G, dry, w, nx, ny)
        assert sl == un - 2 * c and sr == un + c
        phi, _ = orc.hll(G, dry, dry, nx, ny)
        assert (phi == 0).all()


def test_upwinding(orc):
    rng = np.random.default_rng(16)
    n_l = n_r = 0
    for _ in range(4000):
        wl, wr = rand_state(rng), rand_state(rng)
        wl[1] *= 6
        wr[1] *= 6
        phi, (sl, sr, _, _) = orc.hll(G, wl, wr, 1.0, 0.0)
        if sl >= 0:
            n_l += 1
            assert np.array_equal(phi, phys_flux(*wl, 1.0, 0.0)) or \
                np.abs(phi - phys_flux(*wl, 1.0, 0.0)).max() <= 1e-14 * (1 + np.abs(phi).max())
        if sr < 0:
            n_r += 1
            assert np.abs(phi - phys_flux(*wr, 1.0, 0.0)).max() <= 1e-14 * (1 + np.abs(phi).max())
    assert n_l > 20 and n_r > 20


def test_rotation_invariance(orc):
    rng = np.random.default_rng(17)
    for _ in range(1000):
        wl, wr = rand_state(rng, 0.1), rand_state(rng, 0.1)
        nx, ny = rand_normal(rng)
        phi, _ = orc.hll(G, wl, wr, nx, ny)
        # rotate everything by 90 degrees: (x, y) -> (-y, x)
        rl = np.array([wl[0], -wl[2], wl[1]])
        rr = np.array([wr[0], -wr[2], wr[1]])
        psi, _ = orc.hll(G, rl, rr, -ny, nx)
        rot = np.array([phi[0], -phi[2], phi[1]])
        assert np.abs(psi - rot).max() <= 1e-14 * (1 + np.abs(phi).max())


def test_wall_zero_mass_flux(orc):
    rng = np.random.default_rng(18)
    p = orc.params(g=G, h_threshold=1e-3)
    for _ in range(5000):
        H = rng.uniform(0.0, 5.0)
        h = rng.uniform(-2.0, 5.0)
        face = [H - h, h, H, rng.normal(0, 3), rng.normal(0, 3)]
        nx, ny = rand_normal(rng)
        phi, pc = orc.face_flux(p, face, None, nx, ny)
        assert phi[0] == 0.0
        # momentum flux is the pressure of the wall state along n (plus the
        # reflection term), so the tangential component vanishes for u = 0
    face = [1.0, 2.0, 3.0, 0.0, 0.0]
    phi, pc = orc.face_flux(p, face, None, 0.6, 0.8)
    assert abs(phi[1] * 0.8 - phi[2] * 0.6) <= 1e-15


def test_hydrostatic_face_balance(orc):
    """Lake at rest across a face with different bed depths on each side:
    phi + p_L n equals the pressure g/2 H_L^2 n of the left face depth, the
    same for the right; the mass flux vanishes (Audusse et al. reading)."""
    rng = np.random.default_rng(19)
    p = orc.params(g=G, h_threshold=1e-3)
    for _ in range(2000):
        hl, hr = rng.uniform(-1.0, 5.0, 2)
        eta = 0.0
        HL, HR = max(0.0, eta + hl), max(0.0, eta + hr)
        left = [eta if HL > 0 else -hl, hl, HL, 0.0, 0.0]
        right = [eta if HR > 0 else -hr, hr, HR, 0.0, 0.0]
        nx, ny = rand_normal(rng)
        phi, pc = orc.face_flux(p, left, right, nx, ny)
        assert abs(phi[0]) <= 1e-15
        for side, Hs in ((0, HL), (1, HR)):
            tot = np.array([phi[1] + pc[side] * nx, phi[2] + pc[side] * ny])
            ref = 0.5 * G * Hs * Hs * np.array([nx, ny])
            assert np.abs(tot - ref).max() <= 1e-13 * (1 + 0.5 * G * Hs * Hs)
