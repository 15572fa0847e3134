"""Differentiable FP64 statement of the scheme in plain PyTorch CPU ops.

TEST INFRASTRUCTURE ONLY: the tests use it for the tape-based gradient
(torch.autograd) that the GPU library's hand-written discrete adjoint is
checked against.  The GPU library never imports it.

It restates the method of vsw_oracle.c in the same order of work (pinned
bit for bit against it in tests/test_oracle_adjoint.py), vectorised over the
mesh, on the connectivity and geometry that the C oracle builds:
  Section 2.1  w = (H, Hu, Hv), eta = H - h
  Section 2.2  HLL flux with the two-rarefaction speeds u*, c*; dry-bed speeds
  Section 2.3  SSP-RK(2,2) with the CFL time step (reading of the CFL rule)
  Section 2.4  least-squares gradients, Barth-Jespersen limiter (one ratio
               per face, the minimum over the faces), eq. (3), threshold
               depth H_thr
  Section 2.5  wall ghosts
with the hydrostatic reconstruction of the bed source: a cell pass for the
reconstruction, one flux per face in canonical orientation whose two side
terms are handed to the face's cells, and a cell pass that sums each cell's
three faces in local order.  Branches (wet/dry, upwind choice, limiter,
min/max) are `torch.where` selections made on the values, so the tape
differentiates the branch that the forward takes.
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
        # faces in canonical orientation: the left side (a wall's only side)
        # and, for interior faces, the right side
        isl = np.asarray(g["is_left"]) != 0
        kl, jl = np.nonzero(isl)
        self.ekl, self.ejl = torch.tensor(kl), torch.tensor(jl)
        ew = nbr[kl, jl] < 0
        self.ewall = torch.tensor(ew)
        kr = np.where(ew, kl, nbr[kl, jl])
        jr = np.where(ew, jl, jn[kl, jl])
        self.ekr, self.ejr = torch.tensor(kr), torch.tensor(jr)
        # slot 3 k + j of every side term: left sides, then interior right
        # sides; inv puts them back in (cell, face) order
        slot = np.concatenate([3 * kl + jl, (3 * kr + jr)[~ew]])
        assert len(slot) == 3 * self.nc and len(np.unique(slot)) == 3 * self.nc
        inv = np.empty_like(slot)
        inv[slot] = np.arange(len(slot))
        self.side_inv = torch.tensor(inv)
        self.isl = torch.tensor(isl)


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
    out = []
    for c in range(3):
        fs = _where_div(star, (sR * fL[c] - sL * fR[c]) + sLR * dU[c], den)
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
        # Barth-Jespersen: per face j the largest phi_j in [0, 1] that keeps
        # the face value inside [q_min, q_max]; alpha = min_j phi_j
        qmax, qmin = q0, q0
        for j in range(3):
            qmax = _vmax(qmax, qs[:, j])
            qmin = _vmin(qmin, qs[:, j])
        up, dn = qmax - q0, qmin - q0
        one = torch.ones_like(q0)
        a = one
        for j in range(3):
            d = pj[:, j]
            dp, dm = d > 0.0, d < 0.0
            phi = torch.where(dp, _vmin(one, _where_div(dp, up, d)),
                              torch.where(dm, _vmin(one, _where_div(dm, dn, d)), one))
            a = _vmin(a, phi)
        return a

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
    u = _where_div(wet, fu, fH)
    v = _where_div(wet, fv, fH)
    return (fe, fh, fH, u, v), second


def residual(G: Geometry, H, HU, HV, h, g, thr):
    """R(w) = (-sum_j +-l_j G_j + S_c) / |K| per cell (Sections 2.2, 2.4)."""
    hg = 0.5 * g
    (fe, fh, fH, u, v), second = reconstruct(G, H, HU, HV, h, thr)
    # one flux per face, canonical orientation (n from left to right)
    kl, jl, kr, jr, wall = G.ekl, G.ejl, G.ekr, G.ejr, G.ewall
    nx, ny, ln = G.nx[kl, jl], G.ny[kl, jl], G.len[kl, jl]
    eL, hL, HL, uL, vL = fe[kl, jl], fh[kl, jl], fH[kl, jl], u[kl, jl], v[kl, jl]
    eR, hR, HR, uR, vR = fe[kr, jr], fh[kr, jr], fH[kr, jr], u[kr, jr], v[kr, jr]
    unL, utL = uL * nx + vL * ny, vL * nx - uL * ny
    unR, utR = uR * nx + vR * ny, vR * nx - uR * ny
    zero = torch.zeros_like(hL)
    # a wall's ghost mirrors the left state in the face frame (Section 2.5)
    hs = torch.where(wall, hL, _vmin(hL, hR))
    HsL = torch.where(eL + hs > 0.0, eL + hs, zero)
    HsR = torch.where(wall, HsL, torch.where(eR + hs > 0.0, eR + hs, zero))
    unR = torch.where(wall, -unL, unR)
    utR = torch.where(wall, utL, utR)
    f0, f1, f2 = hll(g, HsL, unL, utL, HsR, unR, utR)
    pcL = hg * (HL * HL - HsL * HsL)
    pcR = hg * (HR * HR - HsR * HsR)
    phi0 = f0
    phi1 = f1 * nx - f2 * ny
    phi2 = f1 * ny + f2 * nx
    tl = (ln * phi0, ln * (phi1 + pcL * nx), ln * (phi2 + pcL * ny))
    tr = (ln * phi0, ln * (phi1 + pcR * nx), ln * (phi2 + pcR * ny))
    inner = ~wall
    # side terms back in (cell, face) order: [nc, 3] per component
    term = [torch.cat([tl[c], tr[c][inner]])[G.side_inv].reshape(-1, 3) for c in range(3)]
    # each cell sums its faces in local order: minus on its left faces
    acc = [torch.zeros_like(H) for _ in range(3)]
    for j in range(3):
        lj = G.isl[:, j]
        for c in range(3):
            acc[c] = torch.where(lj, acc[c] - term[c][:, j], acc[c] + term[c][:, j])
    c = (G.len * (H[:, None] + fH)) * (fh - h[:, None])
    sx = (c[:, 0] * G.nx[:, 0] + c[:, 1] * G.nx[:, 1]) + c[:, 2] * G.nx[:, 2]
    sy = (c[:, 0] * G.ny[:, 0] + c[:, 1] * G.ny[:, 1]) + c[:, 2] * G.ny[:, 2]
    a1 = torch.where(second, acc[1] + hg * sx, acc[1])
    a2 = torch.where(second, acc[2] + hg * sy, acc[2])
    return acc[0] / G.area, a1 / G.area, a2 / G.area


def cfl_dt(G: Geometry, H, HU, HV, g, thr, cfl):
    """dt = CFL min over wet cells of |K| / (P_K (|u| + sqrt(g H)))."""
    wet = H >= thr
    u = _where_div(wet, HU, H)
    v = _where_div(wet, HV, H)
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
