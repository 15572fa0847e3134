// Kernels of the discrete adjoint of one SSP-RK(2,2) step (FP64): the
// vector-Jacobian product of the residual R(w; h) and the reverse of the
// Runge-Kutta stages, the post-stage fix and the CFL time step.  The
// stages' residuals, fix masks and states come from the tape the stage
// kernels record while replaying a checkpoint segment (see Tape).
#pragma once
#include "vsw_kernels.hpp"

namespace vsw {

// Adjoint of one cell's variables (H, HU, HV, h).  In the records of the
// state adjoints lam the h field carries the running adjoint of the bed
// depth (the bed is the same in every state).
struct alignas(32) Adj4 {
    double H, HU, HV, h;
};

// Where the vector-Jacobian product leaves its results for the gathers: the
// own adjoint of each cell (with the contributions of the stencil members in
// its tile), and the contributions to stencil members in other tiles, one
// per halo item of the contributing cell's tile (the tile map's halo list,
// in its order).  xin[j nc + k] is the index in x of the contribution cell k
// receives across its face j, or -1 when none comes through x (a wall or a
// neighbour in k's own tile).
struct AdjC {
    Adj4* __restrict__ own;          // [nc]
    Adj4* __restrict__ x;            // [halo items]
    const int32_t* __restrict__ xin; // [3][nc]
};

// xin of the tile map (preset to -1): for halo item b of tile t, the cell
// outside t and its face that item names receive x index bstart[t] + b.
__global__ void adj_xin_kernel(TileMap tm, int64_t nc, int32_t* xin);
// Bits of the CFL minimum of W into *rmin (pre-set to +inf).
__global__ void adj_rmin_kernel(DevMesh m, TileMap tm, const Cell4* W, double g, double thr,
                                unsigned long long* rmin);
// Start of the reverse of a step from its tape (R1 = R(w1), mask2 of
// w^{n+1} = fix(w/2 + (w1 + dt R1)/2)) with lam the adjoint of w^{n+1}:
// lt2 = mask2 (.) lam, mua = dt/2 lt2 / |K|, lamn = (lt2/2, lam.h),
// part[tile] = sum lt2/2 . R1.
__global__ void adj_start_kernel(DevMesh m, TileMap tm, const Adj4* lam, const uint8_t* mask2,
                                 const double* R1, double dt, double* mua, Adj4* lamn,
                                 double* part);
// Vector-Jacobian product of R at W with weights mua = mu / |K| (3 per
// cell), one workgroup per tile (dynamic LDS: stage_lds_bytes(bmax)).  Each
// cell reverses its own term and its neighbour's term of each face (the
// forward evaluates a face from both sides) and keeps the part for its own
// face state, then reverses its reconstruction into its own adjoint and one
// contribution per stencil member.  A contribution to a member in the same
// tile is handed over through LDS and added to that member's own adjoint in
// face order; c.own[k] receives the own adjoint with those, and c.x the
// contribution to each stencil member in another tile, at the index of the
// halo item of this tile that names the member (for the gathers).  With
// argmin_reset, also sets that word to all ones for adj_gather_rk2_kernel.
__global__ void adj_vjp_kernel(DevMesh m, TileMap tm, const Cell4* W, const double* mua,
                               double g, double hg, double thr, AdjC c,
                               unsigned long long* argmin_reset);
// Gather: own (with its tile's contributions) + the stencil contributions of
// the face neighbours in other tiles, in fixed order (no atomics), then the
// Runge-Kutta reverse that follows J_R(w1)^T:
//   lam1 = lt2/2 + wb, lamn.h += wb.h (bed), lt1 = mask1 (.) lam1,
//   mua = dt lt1 / |K|, lamn += lt1, part[tile] += lt1 . R0.
// With argmin (preset to all ones), also the cell that sets the step's dt:
// *argmin becomes the smallest internal index among the cells of W = w^k
// whose CFL ratio bits equal *rmin.  At a tie the dt depends on the minimum
// of equal ratios, whose derivative is taken as that one cell's.
__global__ void adj_gather_rk2_kernel(DevMesh m, TileMap tm, AdjC c, const Adj4* lam,
                                      const uint8_t* mask2, const uint8_t* mask1,
                                      const double* R0, double dt, double* mua, Adj4* lamn,
                                      double* part, const Cell4* W, double g, double thr,
                                      const unsigned long long* rmin,
                                      unsigned long long* argmin);
// End of the reverse of step k, in one pass per cell: after J_R(w)^T the
// gathered contributions (lamn += wb, the bed's wb.h into lamn.h); with
// argmin, the CFL term dt = CFL ratio(w^k) at cell *argmin (lamn += lamdt
// CFL d ratio/d w, lamdt = the sum of part[0 .. tiles) in fixed order,
// formed by that cell's workgroup); with r, the gauge misfit of w^k
// (lamn.H += 2 r, lamn.h -= 2 r per gauge on the cell).  lamn then holds the
// adjoint of w^k.  With mask2p, also the start of the reverse of step k-1
// from its tape (R1p, mask2p, dtp), as adj_start_kernel: mua, lamp and
// partp (a second array, as part is read during the pass).
__global__ void adj_turn_kernel(DevMesh m, TileMap tm, AdjC c, const Cell4* W, double g,
                                double thr, double cfl, const unsigned long long* argmin,
                                const double* part, const int64_t* cells, int ng,
                                const double* r, Adj4* lamn, const uint8_t* mask2p,
                                const double* R1p, double dtp, double* mua, Adj4* lamp,
                                double* partp);
// Gauge misfit of the state after a step: lam[cell].H += 2 r, lam[cell].h -= 2 r.
__global__ void adj_gauge_kernel(const int64_t* cells, int ng, const double* r, Adj4* lam);
// Caller-order gradient arrays from internal-order adjoints.
__global__ void adj_unpack_kernel(int64_t n, const int64_t* perm, const Adj4* lam, double* gH,
                                  double* gHU, double* gHV, double* gh);

}  // namespace vsw
