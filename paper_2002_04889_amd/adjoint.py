"""Gauge-misfit loss of a forward run as a torch.autograd.Function whose
backward is the library's hand-written discrete adjoint (vsw_adjoint_gauge_loss).

    loss = GaugeLoss.apply(H0, HU0, HV0, h, mesh, params, nsteps, ckpt, gauges, obs)

H0, HU0, HV0 (initial state) and h (bed depth) are FP64 tensors in the
caller's cell order on any device; mesh = (vx, vy, tri) numpy arrays; params
= dict(g, cfl, h_threshold, dt_fixed).  The forward uploads the mesh with h,
runs the adjoint call once (forward run, loss and gradients) and keeps the
gradients for backward.  Gradients with respect to parameters that act
through h or the initial state (for instance bed-displacement amplitudes,
h = h0 - Phi a) follow by the chain rule in torch.
"""
from __future__ import annotations

import numpy as np
import torch

from . import vsw


class GaugeLoss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, H0, HU0, HV0, h, mesh, params, nsteps, ckpt, gauges, obs):
        vx, vy, tri = mesh
        npy = lambda t: t.detach().to("cpu", torch.float64).numpy()
        s = vsw.Solver(**params)
        try:
            s.upload_mesh(vx, vy, tri, npy(h))
            s.set_state(npy(H0), npy(HU0), npy(HV0), 0.0)
            loss, gH, gU, gV, gh = vsw.vsw_adjoint_gauge_loss(s.h, s.nc, nsteps, ckpt, gauges,
                                                              obs)
        finally:
            s.close()
        dev = H0.device
        ctx.save_for_backward(*[torch.from_numpy(a).to(dev) for a in (gH, gU, gV, gh)])
        return torch.tensor(loss, dtype=torch.float64, device=dev)

    @staticmethod
    def backward(ctx, go):
        gH, gU, gV, gh = ctx.saved_tensors
        return go * gH, go * gU, go * gV, go * gh, None, None, None, None, None, None


def displacement_basis(cx, cy, x0=100e3, y0=200e3, lx=200e3, ly=100e3, nx=20, ny=10,
                       sigma=10e3):
    """Gaussian bumps (sigma 10 km) on an nx x ny grid over the source box
    [x0, x0 + lx] x [y0, y0 + ly]: Phi [ncells, nx * ny]."""
    gx = x0 + (np.arange(nx) + 0.5) * lx / nx
    gy = y0 + (np.arange(ny) + 0.5) * ly / ny
    X, Y = np.meshgrid(gx, gy, indexing="ij")
    d2 = (cx[:, None] - X.ravel()[None, :]) ** 2 + (cy[:, None] - Y.ravel()[None, :]) ** 2
    return np.exp(-d2 / (2.0 * sigma * sigma))
