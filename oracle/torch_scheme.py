"""Differentiable FP64 statement of the scheme in plain PyTorch CPU ops.

TEST INFRASTRUCTURE ONLY: the tests use it for the tape-based gradient
(torch.autograd) that the GPU library's hand-written discrete adjoint is
checked against.  The GPU library never imports it.

It restates, cell by cell and vectorised over the mesh, the same method as
vsw_oracle.c (pinned against it in tests/test_oracle_adjoint.py), on the
connectivity and geometry that the C oracle builds:
  Section 2.1  w = (H, Hu, Hv), eta = H - h
  Section 2.2  HLL flux with the two-rarefaction speeds u*, c*; dry-bed speeds
  Section 2.3  SSP-RK(2,2) with the CFL time step (reading of the CFL rule)
  Section 2.4  least-squares gradients, Barth-Jespersen limiter, eq. (3),
               threshold depth H_thr
  Section 2.5  wall ghosts
with the hydrostatic reconstruction of the bed source.  Branches (wet/dry,
upwind choice, limiter, min/max) are `torch.where` selections made on the
values, so the tape differentiates the branch that the forward takes.  The
Barth-Jespersen factor is written as min(1, (q_max - q_0) / max_j d_j,
(q_min - q_0) / min_j d_j), which equals the per-face minimum of the
limiter's definition (the ratio is monotone in d_j).
"""
from __future__ import annotations

import numpy as np
import torch

F64 = torch.float64


class _Sqrt(torch.autograd.Function):
    """Correctly rounded square root (numpy's; torch's CPU float64 sqrt is
    off by one ulp for some inputs) with the derivative 1 / (2 sqrt x)."""

    @staticmethod
    def forward(ctx, x):
        r = torch.from_numpy(np.sqrt(x.detach().numpy()))
        ctx.save_for_backward(r)
        return r

    @staticmethod
    def backward(ctx, gr):
        (r,) = ctx.saved_tensors
        return gr / (2.0 * r)


def _sqrt(x):
    return _Sqrt.apply(x.contiguous())


def _where_div(mask, a, b):
    """a / b where mask, 0 elsewhere, without inf/nan on the untaken side."""
    return torch.where(mask, a / torch.where(mask, b, torch.ones_like(b)), torch.zeros_like(a))


def _ssqrt(x, mask):
    """sqrt(x) where mask (x > 0 there), 0 elsewhere, safe for the tape."""
    return torch.where(mask, _sqrt(torch.where(mask, x, torch.ones_like(x))),
                       torch.zeros_like(x))


def _vmax(a, b):  # (b > a) ? b : a
    return torch.where(b > a, b, a)


def _vmin(a, b):  # (b < a) ? b : a
    return torch.where(b < a, b, a)


class Geometry:
    """Connectivity and geometry of the C oracle, as torch tensors."""

    def __init__(self, orc_mesh):
        g = orc_mesh.geometry()
        self.nc = orc_mesh.nc
        t = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=F64)
        self.nx, self.ny, self.len = t(g["nx"]), t(g["ny"]), t(g["len"])
        self.dx, self.dy, self.wx, self.wy = t(g["dx"]), t(g["dy"]), t(g["wx"]), t(g["wy"])
        self.area, self.perim = t(g["area"]), t(g["perim"])
        nbr = np.asarray(g["nbr"], dtype=np.int64)
        self.wall = torch.tensor(nbr < 0)
        self.nb = torch.tensor(np.where(nbr < 0, np.arange(self.nc)[:, None], nbr))
        self.left = torch.tensor(np.asarray(g["is_left"]) != 0) | self.wall
        # face index of the shared face inside the neighbour
        jn = np.zeros_like(nbr)
        rows = np.arange(self.nc)
        for j in range(3):
            n = np.where(nbr[:, j] < 0, 0, nbr[:, j])
            for q in range(3):
                hit = (nbr[n, q] == rows) & (nbr[:, j] >= 0)
                jn[hit, j] = q
        self.jn = torch.tensor(jn)


def hll(g, HL, unL, utL, HR, unR, utR):
    """HLL flux in the face frame (Section 2.2), elementwise."""
    hg = 0.5 * g
    wetL, wetR = HL > 0.0, HR > 0.0
    cL, cR = _ssqrt(g * HL, wetL), _ssqrt(g * HR, wetR)
    us = 0.5 * (unL + unR) + (cL - cR)
    cs = 0.5 * (cL + cR) - 0.25 * (unR - unL)
    sL_w = _vmin(unL - cL, us - cs)
    sR_w = _vmax(us + cs, unR + cR)
    # left dry: s_L = u_R - 2 c_R, s_R = u_R + c_R; right dry: u_L - c_L, u_L + 2 c_L
    sL = torch.where(~wetL, unR - 2.0 * cR, torch.where(~wetR, unL - cL, sL_w))
    sR = torch.where(~wetL, unR + cR, torch.where(~wetR, unL + 2.0 * cL, sR_w))
    qL, qR = HL * unL, HR * unR
    fL = (qL, qL * unL + hg * (HL * HL), qL * utL)
    fR = (qR, qR * unR + hg * (HR * HR), qR * utR)
    dU = (HR - HL, qR - qL, HR * utR - HL * utL)
    both_dry = (~wetL) & (~wetR)
    upL = sL >= 0.0
    upR = (~upL) & (sR < 0.0)
    star = ~(upL | upR | both_dry)
    den = sR - sL
    sLR = sL * sR
    rd = _where_div(star, torch.ones_like(den), den)
    out = []
    for c in range(3):
        fs = ((sR * fL[c] - sL * fR[c]) + sLR * dU[c]) * rd
        f = torch.where(upL, fL[c], torch.where(upR, fR[c], fs))
        out.append(torch.where(both_dry, torch.zeros_like(f), f))
    return out


def reconstruct(G: Geometry, H, HU, HV, h, thr):
    """Face states (eta, h, H, u, v) [nc, 3] each, second-order flags, and
    the face values the bed source needs (Section 2.4, eq. (3))."""
    e = H - h
    wall, nb = G.wall, G.nb
    nx, ny = G.nx, G.ny
    mn = HU[:, None] * nx + HV[:, None] * ny
    qe = torch.where(wall, e[:, None].expand(-1, 3), H[nb] - h[nb])
    qu = torch.where(wall, HU[:, None] - (2.0 * mn) * nx, HU[nb])
    qv = torch.where(wall, HV[:, None] - (2.0 * mn) * ny, HV[nb])
    qh = torch.where(wall, h[:, None].expand(-1, 3), h[nb])
    Hs = torch.where(wall, H[:, None].expand(-1, 3), H[nb])
    cand = (H >= thr) & (Hs >= thr).all(dim=1)

    def project(qs, q0):
        d0, d1, d2 = qs[:, 0] - q0, qs[:, 1] - q0, qs[:, 2] - q0
        gx = (G.wx[:, 0] * d0 + G.wx[:, 1] * d1) + G.wx[:, 2] * d2
        gy = (G.wy[:, 0] * d0 + G.wy[:, 1] * d1) + G.wy[:, 2] * d2
        return gx[:, None] * G.dx + gy[:, None] * G.dy

    def limiter(q0, qs, pj):
        qmax, qmin = q0, q0
        for j in range(3):
            qmax = _vmax(qmax, qs[:, j])
            qmin = _vmin(qmin, qs[:, j])
        up, dn = qmax - q0, qmin - q0
        dpm = torch.zeros_like(q0)
        dnm = torch.zeros_like(q0)
        for j in range(3):
            dpm = _vmax(dpm, pj[:, j])
            dnm = _vmin(dnm, pj[:, j])
        one = torch.ones_like(q0)
        c1 = (dpm > 0.0) & (up < dpm)
        a = torch.where(c1, _where_div(c1, up, dpm), one)
        c2 = (dnm < 0.0) & (dn > dnm)
        r2 = _where_div(c2, dn, dnm)
        return torch.where(c2, _vmin(a, r2), a)

    pe, pu, pv, ph = project(qe, e), project(qu, HU), project(qv, HV), project(qh, h)
    ae, au, av = limiter(e, qe, pe), limiter(HU, qu, pu), limiter(HV, qv, pv)
    fe2 = e[:, None] + ae[:, None] * pe
    fu2 = HU[:, None] + au[:, None] * pu
    fv2 = HV[:, None] + av[:, None] * pv
    fh2 = h[:, None] + ph
    fH2 = fe2 + fh2
    second = cand & (fH2 >= thr).all(dim=1)
    s = second[:, None]
    fe = torch.where(s, fe2, e[:, None].expand(-1, 3))
    fu = torch.where(s, fu2, HU[:, None].expand(-1, 3))
    fv = torch.where(s, fv2, HV[:, None].expand(-1, 3))
    fh = torch.where(s, fh2, h[:, None].expand(-1, 3))
    fH = torch.where(s, fH2, H[:, None].expand(-1, 3))
    wet = fH >= thr
    rH = _where_div(wet, torch.ones_like(fH), fH)
    u = fu * rH
    v = fv * rH
    return (fe, fh, fH, u, v), second


def residual(G: Geometry, H, HU, HV, h, g, thr):
    """R(w) = (-sum_j +-l_j G_j + S_c) / |K| per cell (Sections 2.2, 2.4)."""
    hg = 0.5 * g
    (fe, fh, fH, u, v), second = reconstruct(G, H, HU, HV, h, thr)
    nb, jn, wall = G.nb, G.jn, G.wall
    own = (fe, fh, fH, u, v)
    oth = tuple(torch.where(wall, x, x[nb, jn]) for x in own)
    left = G.left
    pick = lambda a, b: (torch.where(left, a, b), torch.where(left, b, a))
    eL, eR = pick(fe, oth[0])
    hL, hR = pick(fh, oth[1])
    HL, HR = pick(fH, oth[2])
    uL, uR = pick(u, oth[3])
    vL, vR = pick(v, oth[4])
    nx = torch.where(left, G.nx, -G.nx)
    ny = torch.where(left, G.ny, -G.ny)
    unL, utL = uL * nx + vL * ny, vL * nx - uL * ny
    unR, utR = uR * nx + vR * ny, vR * nx - uR * ny
    hs = _vmin(hL, hR)
    zero = torch.zeros_like(hs)
    HsL = torch.where(eL + hs > 0.0, eL + hs, zero)
    HsR = torch.where(eR + hs > 0.0, eR + hs, zero)
    unR = torch.where(wall, -unL, unR)
    f0, f1, f2 = hll(g, HsL, unL, utL, HsR, unR, utR)
    pc = torch.where(left, hg * (HL * HL - HsL * HsL), hg * (HR * HR - HsR * HsR))
    phi1 = f1 * nx - f2 * ny
    phi2 = f1 * ny + f2 * nx
    t0 = G.len * f0
    t1 = G.len * (phi1 + pc * nx)
    t2 = G.len * (phi2 + pc * ny)
    sgn = lambda t: torch.where(left, -t, t)
    a0 = torch.zeros_like(H)
    a1 = torch.zeros_like(H)
    a2 = torch.zeros_like(H)
    for j in range(3):
        a0 = a0 + sgn(t0)[:, j]
        a1 = a1 + sgn(t1)[:, j]
        a2 = a2 + sgn(t2)[:, j]
    c = (G.len * (H[:, None] + fH)) * (fh - h[:, None])
    sx = (c[:, 0] * G.nx[:, 0] + c[:, 1] * G.nx[:, 1]) + c[:, 2] * G.nx[:, 2]
    sy = (c[:, 0] * G.ny[:, 0] + c[:, 1] * G.ny[:, 1]) + c[:, 2] * G.ny[:, 2]
    a1 = torch.where(second, a1 + hg * sx, a1)
    a2 = torch.where(second, a2 + hg * sy, a2)
    ra = 1.0 / G.area
    return a0 * ra, a1 * ra, a2 * ra


def cfl_dt(G: Geometry, H, HU, HV, g, thr, cfl):
    """dt = CFL min over wet cells of |K| / (P_K (|u| + sqrt(g H)))."""
    wet = H >= thr
    rH = _where_div(wet, torch.ones_like(H), H)
    u = HU * rH
    v = HV * rH
    # |u| is taken with a zero derivative at rest (u = v = 0)
    s = _ssqrt(u * u + v * v, (u * u + v * v) > 0.0) + _ssqrt(g * H, wet)
    r = torch.where(wet, G.area / (G.perim * torch.where(wet, s, torch.ones_like(s))),
                    torch.full_like(H, float("inf")))
    return cfl * torch.min(r)


def post_fix(H, HU, HV, thr):
    H = torch.where(H < 0.0, torch.zeros_like(H), H)
    dry = H < thr
    return H, torch.where(dry, torch.zeros_like(HU), HU), torch.where(dry, torch.zeros_like(HV), HV)


def step(G: Geometry, H, HU, HV, h, g, thr, cfl, dt_fixed=0.0):
    """One SSP-RK(2,2) step (Section 2.3); returns the new state and dt."""
    dt = cfl_dt(G, H, HU, HV, g, thr, cfl) if dt_fixed <= 0.0 else torch.tensor(dt_fixed, dtype=F64)
    R = residual(G, H, HU, HV, h, g, thr)
    H1, U1, V1 = post_fix(H + dt * R[0], HU + dt * R[1], HV + dt * R[2], thr)
    R1 = residual(G, H1, U1, V1, h, g, thr)
    H2 = 0.5 * H + 0.5 * (H1 + dt * R1[0])
    U2 = 0.5 * HU + 0.5 * (U1 + dt * R1[1])
    V2 = 0.5 * HV + 0.5 * (V1 + dt * R1[2])
    H2, U2, V2 = post_fix(H2, U2, V2, thr)
    return H2, U2, V2, dt


def gauge_loss(G: Geometry, H0, HU0, HV0, h, nsteps, gauges, eta_obs, g, thr, cfl,
               dt_fixed=0.0):
    """Sum over steps n = 1..nsteps and gauge cells of (eta - eta_obs)^2,
    eta = H - h after each step.  Returns (loss, per-step dts)."""
    H, HU, HV = H0, HU0, HV0
    loss = torch.zeros((), dtype=F64)
    dts = []
    gi = torch.as_tensor(gauges, dtype=torch.int64)
    obs = torch.as_tensor(eta_obs, dtype=F64)
    for n in range(nsteps):
        H, HU, HV, dt = step(G, H, HU, HV, h, g, thr, cfl, dt_fixed)
        dts.append(dt)
        r = (H[gi] - h[gi]) - obs[n]
        loss = loss + (r * r).sum()
    return loss, dts
