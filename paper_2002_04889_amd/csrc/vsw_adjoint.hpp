// Kernels of the discrete adjoint of one SSP-RK(2,2) step (FP64): the
// forward pieces the reverse sweep recomputes, the vector-Jacobian product
// of the residual R(w; h) and the reverse of the Runge-Kutta stages, the
// post-stage fix and the CFL time step.
#pragma once
#include "vsw_kernels.hpp"

namespace vsw {

// Adjoint of one cell's variables (H, HU, HV, h).
struct alignas(32) Adj4 {
    double H, HU, HV, h;
};

// Face states, centred source and order of every cell of W (no control).
__global__ void adj_faces_kernel(DevMesh m, TileMap tm, const Cell4* W, FaceBuf fb, double thr,
                                 double hg);
// R(W) from a face buffer, R[3 * k + c].
__global__ void adj_residual_kernel(DevMesh m, TileMap tm, FaceBuf fb, double g, double hg,
                                    double* R);
// Stage 1 forward on given dt: W1 = fix(W + dt R0); mask bit 0 = H kept,
// bit 1 = momentum kept (bits of the post-stage fix).
__global__ void adj_stage1_kernel(TileMap tm, const Cell4* W, const double* R0, double dt,
                                  double thr, Cell4* W1, uint8_t* mask1);
// Mask of stage 2 (the state itself is not needed by the reverse).
__global__ void adj_mask2_kernel(TileMap tm, const Cell4* W, const Cell4* W1, const double* R1,
                                 double dt, double thr, uint8_t* mask2);
// mu2 = dt/2 lt2, lamn = lt2 / 2, part[tile] = sum lt2/2 . R1 with
// lt2 = mask2 (.) lam (the adjoint of w^{n+1}).
__global__ void adj_rk2_pre_kernel(TileMap tm, const Adj4* lam, const uint8_t* mask2,
                                   const double* R1, double dt, double* mu, Adj4* lamn,
                                   double* part);
// Vector-Jacobian product of R at W with weights mu (3 per cell):
//  faces: face-state adjoints Fb[15 k + 5 j + c] (eta, h, H, u, v) of every
//         cell face, plus the direct (H, h) adjoints of the bed source in D;
//  recon: reverse of the reconstruction, per cell: own (H, HU, HV, h) in
//         C[16 k + 0..3], stencil member j in C[16 k + 4 + 4 j + 0..3];
//  gather: wb[k] = own + the stencil contributions of the face neighbours,
//         in fixed order (no atomics).
__global__ void adj_vjp_faces_kernel(DevMesh m, TileMap tm, FaceBuf fb, const Cell4* W,
                                     const double* mu, double g, double hg, double* Fb,
                                     double* D);
__global__ void adj_vjp_recon_kernel(DevMesh m, TileMap tm, const Cell4* W, const double* Fb,
                                     const double* D, double thr, double* C);
__global__ void adj_vjp_gather_kernel(DevMesh m, TileMap tm, const double* C, Adj4* wb);
// After the stage-2 product wb2: lam1 = lt2/2 + wb2, hbar += wb2.h,
// lt1 = mask1 (.) lam1, mu = dt lt1, lamn += lt1, part[tile] += lt1 . R0.
__global__ void adj_rk2_post_kernel(TileMap tm, const Adj4* lam, const uint8_t* mask2,
                                    const Adj4* wb2, const uint8_t* mask1, const double* R0,
                                    double dt, double* mu, Adj4* lamn, double* hbar, double* part);
// After the stage-1 product wb1: lamn += wb1, hbar += wb1.h.
__global__ void adj_rk1_post_kernel(TileMap tm, const Adj4* wb1, Adj4* lamn, double* hbar);
// CFL minimum of W (bits of the positive double) into *rmin (pre-set to +inf).
__global__ void adj_rmin_kernel(DevMesh m, TileMap tm, const Cell4* W, double g, double thr,
                                unsigned long long* rmin);
// Sum of part[0 .. n) in fixed order into *out (one block).
__global__ void adj_sum_kernel(const double* part, int n, double* out);
// dt = cfl * ratio of the minimising cell(s): lamn += lamdt * cfl * d ratio / d w there.
__global__ void adj_dt_kernel(DevMesh m, TileMap tm, const Cell4* W, double g, double thr,
                              double cfl, const unsigned long long* rmin, const double* lamdt,
                              Adj4* lamn);
// Gauge misfit of the state after a step: lam[cell].H += 2 r, hbar[cell] -= 2 r.
__global__ void adj_gauge_kernel(const int64_t* cells, int ng, const double* r, Adj4* lam,
                                 double* hbar);
// Caller-order gradient arrays from internal-order adjoints.
__global__ void adj_unpack_kernel(int64_t n, const int64_t* perm, const Adj4* lam,
                                  const double* hbar, double* gH, double* gHU, double* gHV,
                                  double* gh);

}  // namespace vsw
