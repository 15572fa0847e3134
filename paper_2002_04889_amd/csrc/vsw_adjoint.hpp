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

// Face states, centred source and order of every cell of W (no control);
// with rmin != nullptr also the CFL minimum of W (bits of the positive
// double, *rmin pre-set to +inf).
__global__ void adj_faces_kernel(DevMesh m, TileMap tm, const Cell4* W, FaceBuf fb, double g,
                                 double thr, double hg, unsigned long long* rmin);
// Stage 1 recomputed: R0 = R(W) from W's face buffer (kept), W1 =
// fix(W + dt R0) and its mask (bit 0: depth kept, bit 1: momentum kept).
__global__ void adj_stage1_kernel(DevMesh m, TileMap tm, FaceBuf fb, const Cell4* W, double g,
                                  double hg, double dt, double thr, double* R0, Cell4* W1,
                                  uint8_t* mask1);
// Stage 2 recomputed from W1's face buffer, R1 = R(W1), the mask of
// w^{n+1} = fix(W/2 + (W1 + dt R1)/2), and the start of its reverse with lam
// the adjoint of w^{n+1}: lt2 = mask2 (.) lam, mu = dt/2 lt2, lamn = lt2/2,
// part[tile] = sum lt2/2 . R1.
__global__ void adj_stage2_kernel(DevMesh m, TileMap tm, FaceBuf fb, const Cell4* W,
                                  const Cell4* W1, double g, double hg, double dt, double thr,
                                  const Adj4* lam, uint8_t* mask2, double* mu, Adj4* lamn,
                                  double* part);
// Vector-Jacobian product of R at W with weights mu (3 per cell):
//  faces: the adjoint of every face state from the terms of both cells that
//         share the face (each cell reverses its own term and its
//         neighbour's term of the face and keeps the part for its own face
//         state; measured faster than handing the neighbour's part over
//         through memory) and from the bed source: Fb[(5 j + c) nc + k]
//         (eta, h, H, u, v), the direct (H, h) adjoints of the source in D;
//  recon: per cell, the reverse of the reconstruction: own (H, HU, HV, h)
//         in C[16 k + 0..3], stencil member j in C[16 k + 4 + 4 j + 0..3];
//  gather: own + the stencil contributions of the face neighbours, in fixed
//         order (no atomics), then the Runge-Kutta reverse that follows:
//   after J_R(w1)^T: lam1 = lt2/2 + wb, hbar += wb.h, lt1 = mask1 (.) lam1,
//                    mu = dt lt1, lamn += lt1, part[tile] += lt1 . R0;
//   after J_R(w)^T:  lamn += wb, hbar += wb.h.
__global__ void adj_vjp_faces_kernel(DevMesh m, TileMap tm, FaceBuf fb, const Cell4* W,
                                     const double* mu, double g, double hg, double* Fb,
                                     double* D);
__global__ void adj_vjp_recon_kernel(DevMesh m, TileMap tm, const Cell4* W, const double* Fb,
                                     const double* D, double thr, double* C);
__global__ void adj_gather_rk2_kernel(DevMesh m, TileMap tm, const double* C, const Adj4* lam,
                                      const uint8_t* mask2, const uint8_t* mask1,
                                      const double* R0, double dt, double* mu, Adj4* lamn,
                                      double* hbar, double* part);
__global__ void adj_gather_rk1_kernel(DevMesh m, TileMap tm, const double* C, Adj4* lamn,
                                      double* hbar);
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
