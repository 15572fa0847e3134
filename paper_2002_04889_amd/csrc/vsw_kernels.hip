// Stage kernels of the SSP-RK(2,2) shallow-water step (Section 2.3) on
// gfx950, and the small control kernels around them.
//
// Per step, two stages; per stage two kernels:
//   recon_kernel   one thread per cell: reconstruction (Section 2.4) of the
//                  cell's three faces, written to a face buffer (SoA)
//   update_kernel  one thread per cell: the three face fluxes, each in the
//                  face's canonical orientation so both cells of a face get
//                  the same number with opposite signs (no atomics, exact
//                  conservation), the bed source, the Runge-Kutta stage and
//                  the post-stage fix; stage 2 also reduces the CFL ratio of
//                  the new state for the next step's dt (wavefront min, LDS,
//                  one 64-bit atomic min per block on the bits of a positive
//                  double).
// The time step and the current time live in a small device control block,
// so the host never synchronises between steps.
#include "vsw_common.hpp"

namespace vsw {

// ---------------------------------------------------------------- control

__global__ void ctrl_init_kernel(Ctrl* c, Seg* sg, int nseg, const double* t0, int par,
                                 int keep) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        c->err = 0;
        c->err_step = 0x7FFFFFFF;
        c->clamps = 0;
        c->kbase = 0;
        c->par = par;
    }
    for (int s = int(blockIdx.x * blockDim.x + threadIdx.x); s < nseg;
         s += int(gridDim.x * blockDim.x)) {
        Seg q;
        q.rmin[0] = (keep >= 0) ? sg[s].rmin[keep] : 0x7FF0000000000000ull;
        q.rmin[1] = 0x7FF0000000000000ull;
        q.t[0] = q.t[1] = t0[s];
        q.dt_last = 0.0;
        q.steps_done = 0;
        q.pad[0] = q.pad[1] = 0;
        sg[s] = q;
    }
}

__global__ void step_bump_kernel(Ctrl* c, int by) {
    if (blockIdx.x == 0 && threadIdx.x == 0) c->kbase += by;
}

__global__ __launch_bounds__(kBlock) void dt_init_kernel(DevMesh m, TileMap tm,
                                                         const Cell4* __restrict__ W, double g,
                                                         double thr, Seg* sg) {
    const TileInfo ti = tile_info(tm.tinfo[blockIdx.x]);
    const int64_t k = int64_t(blockIdx.x) * kTile + threadIdx.x;
    double r = __longlong_as_double(0x7FF0000000000000ll);
    if (int(threadIdx.x) < ti.cnt) {
        const Cell4 q = W[k];
        r = cfl_ratio(q.H, q.HU, q.HV, m.area[k], m.perim[k], g, thr);
    }
    block_min_atomic(r, &sg[ti.seg].rmin[0]);
}

// ---------------------------------------------------------------- two-pass kernels

// The two-pass kernels run one block per tile (kBlock == kTile).
template <int STAGE>
__global__ __launch_bounds__(kBlock) void recon_kernel(DevMesh m, TileMap tm,
                                                       const Cell4* __restrict__ Wa,
                                                       const Cell4* __restrict__ Wb,
                                                       const Cell4* __restrict__ W1, FaceBuf fb,
                                                       StepParams p, const Ctrl* c, const Seg* sg,
                                                       int slot, int step_arg) {
    const TileInfo ti = tile_info(tm.tinfo[blockIdx.x]);
    double dt, tn;
    if (!step_dt(c, sg + ti.seg, slot, p, dt, tn)) return;
    const Cell4 *Win, *Wout;
    step_buffers(c, c->kbase + step_arg, Wa, Wb, Win, Wout);
    const Cell4* __restrict__ W = (STAGE == 1) ? Win : W1;
    const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (int(threadIdx.x) >= ti.cnt) return;
    const int64_t nc = m.nc;
    Face f[3];
    double sc[2];
    const bool second = recon_cell(m, W, k, p.thr, p.hg, f, sc);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        fb.f[(5 * j + 0) * nc + k] = f[j].eta;
        fb.f[(5 * j + 1) * nc + k] = f[j].h;
        fb.f[(5 * j + 2) * nc + k] = f[j].H;
        fb.f[(5 * j + 3) * nc + k] = f[j].u;
        fb.f[(5 * j + 4) * nc + k] = f[j].v;
    }
    fb.sc[k] = sc[0];
    fb.sc[nc + k] = sc[1];
    fb.order[k] = second ? 2 : 1;
}

template __global__ void recon_kernel<1>(DevMesh, TileMap, const Cell4*, const Cell4*,
                                         const Cell4*, FaceBuf, StepParams, const Ctrl*,
                                         const Seg*, int, int);
template __global__ void recon_kernel<2>(DevMesh, TileMap, const Cell4*, const Cell4*,
                                         const Cell4*, FaceBuf, StepParams, const Ctrl*,
                                         const Seg*, int, int);

__global__ __launch_bounds__(kBlock) void update1_kernel(DevMesh m, TileMap tm,
                                                         const Cell4* __restrict__ Wa,
                                                         const Cell4* __restrict__ Wb,
                                                         Cell4* __restrict__ W1, FaceBuf fb,
                                                         StepParams p, Ctrl* c, Seg* sg, int slot,
                                                         int step_arg) {
    const TileInfo ti = tile_info(tm.tinfo[blockIdx.x]);
    double dt, tn;
    if (!step_dt(c, sg + ti.seg, slot, p, dt, tn)) return;
    const Cell4 *W, *Wout;
    step_buffers(c, c->kbase + step_arg, Wa, Wb, W, Wout);
    if (ti.first && threadIdx.x == 0) sg[ti.seg].rmin[slot ^ 1] = 0x7FF0000000000000ull;
    const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    unsigned long long clamp = 0;
    if (int(threadIdx.x) < ti.cnt) {
        double R[3];
        residual_from_faces(m, fb, k, p.g, p.hg, R);
        uint8_t mk;
        W1[k] = stage1_update(W[k], R, dt, p.thr, clamp, mk);
    }
    block_count_atomic(clamp, &c->clamps);
}

__global__ __launch_bounds__(kBlock) void update2_kernel(DevMesh m, TileMap tm,
                                                         Cell4* __restrict__ Wa,
                                                         Cell4* __restrict__ Wb,
                                                         const Cell4* __restrict__ W1, FaceBuf fb,
                                                         StepParams p, Ctrl* c, Seg* sg, int slot,
                                                         int step_arg, double* log) {
    const TileInfo ti = tile_info(tm.tinfo[blockIdx.x]);
    Seg* sgs = sg + ti.seg;
    const int step = c->kbase + step_arg;
    Cell4 *W, *Wout;
    step_buffers(c, step, Wa, Wb, W, Wout);
    double dt, tn;
    const bool active = step_dt(c, sgs, slot, p, dt, tn);
    if (!active) {
        carry_state(c, sgs, slot, p, W, Wout, int64_t(blockIdx.x) * kBlock, ti.cnt);
        stage2_bookkeeping(c, sgs, ti, tm.nseg, slot, step, false, 0.0, 0.0, p.t_stop, log);
        return;
    }
    const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    unsigned long long clamp = 0;
    double r = __longlong_as_double(0x7FF0000000000000ll);
    bool bad = false;
    if (int(threadIdx.x) < ti.cnt) {
        double R[3];
        residual_from_faces(m, fb, k, p.g, p.hg, R);
        uint8_t mk;
        const Cell4 o = stage2_update(W[k], W1[k], R, dt, p.thr, clamp, mk);
        Wout[k] = o;
        bad = !isfinite(o.H) || !isfinite(o.HU) || !isfinite(o.HV);
        r = cfl_ratio(o.H, o.HU, o.HV, m.area[k], m.perim[k], p.g, p.thr);
    }
    if (bad) {
        atomicOr(&c->err, 1);
        atomicMin(&c->err_step, step);
    }
    block_count_atomic(clamp, &c->clamps);
    block_min_atomic(r, &sgs->rmin[slot ^ 1]);
    stage2_bookkeeping(c, sgs, ti, tm.nseg, slot, step, true, dt, tn, p.t_stop, log);
}

// ---------------------------------------------------------------- fused stage

// One workgroup per tile of kTile cells, one thread per cell:
//  1. reconstruct the tile's cells and its halo faces into LDS (tile_faces);
//  2. per cell, the three face fluxes in canonical orientation from LDS (one
//     branch-free evaluation per face), the centred bed source, the residual
//     and the Runge-Kutta stage.
// Each face inside a tile is evaluated by both of its cells; a face list
// evaluated once per face (edge-parallel, with two more barriers to hand the
// terms over) measured slower on the 1M-cell basin.  TAPE adds the outputs
// the adjoint records (see Tape) and leaves the arithmetic as it is.
template <int STAGE, bool TAPE>
__device__ __forceinline__ void stage_body(const DevMesh& m, const TileMap& tm,
                                           Cell4* __restrict__ Wa, Cell4* __restrict__ Wb,
                                           Cell4* __restrict__ W1, const StepParams& p, Ctrl* c,
                                           Seg* sg, int slot, int step_arg, double* log,
                                           const Tape& tp) {
    extern __shared__ double lds[];
    const int stride = 3 * kTile + tm.bmax;
    const int t = tm.xcd_order ? xcd_tile(int(blockIdx.x), tm.ntiles) : int(blockIdx.x);
    const TileInfo ti = tile_info(tm.tinfo[t]);
    Seg* sgs = sg + ti.seg;
    const int step = c->kbase + step_arg;
    Cell4 *W, *Wout;
    step_buffers(c, step, Wa, Wb, W, Wout);
    double dt, tn;
    const bool active = step_dt(c, sgs, slot, p, dt, tn);
    if (!active) {
        if (STAGE == 2) {
            carry_state(c, sgs, slot, p, W, Wout, int64_t(t) * kTile, ti.cnt);
            stage2_bookkeeping(c, sgs, ti, tm.nseg, slot, step, false, 0.0, 0.0, p.t_stop, log);
        }
        return;
    }
    if (STAGE == 1 && ti.first && threadIdx.x == 0) sgs->rmin[slot ^ 1] = 0x7FF0000000000000ull;
    // state the stage reconstructs: w^n in stage 1, w1 in stage 2
    const Cell4* __restrict__ Ws = (STAGE == 1) ? W : W1;
    const int64_t nc = m.nc;
    const int64_t c0 = int64_t(t) * kTile;
    const int cnt = ti.cnt;
    const int i = threadIdx.x;
    const int64_t k = c0 + i;

    double sc[2], ownH[3];
    bool second;
    tile_faces(m, tm, Ws, t, c0, cnt, p.thr, p.hg, lds, stride, ownH, sc, second);
    __syncthreads();

    unsigned long long clamp = 0;
    double rr = __longlong_as_double(0x7FF0000000000000ll);
    bool bad = false;
    if (i < cnt) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const uint16_t s = tm.nloc[j * nc + k];
            const bool wall = (s == kNlocWall16);
            const Face own = lds_load_face(lds, stride, j * kTile + i, ownH[j]);
            const Face other =
                lds_load_face(lds, stride, wall ? j * kTile + i : int(s & 0x7FFFu), 0.0);
            double tt[3];
            const bool left = face_term(p.g, p.hg, own, other, wall, (s & 0x8000u) != 0,
                                        gf(m, 0, j, k), gf(m, 1, j, k), gf(m, 2, j, k), tt);
            if (left) {
                a0 = a0 - tt[0]; a1 = a1 - tt[1]; a2 = a2 - tt[2];
            } else {
                a0 = a0 + tt[0]; a1 = a1 + tt[1]; a2 = a2 + tt[2];
            }
        }
        if (second) {
            a1 = a1 + sc[0];
            a2 = a2 + sc[1];
        }
        const double ar = m.area[k];
        double R[3];
        div_area(a0, a1, a2, ar, R);
        uint8_t mk;
        if (STAGE == 1) {
            W1[k] = stage1_update(W[k], R, dt, p.thr, clamp, mk);
        } else {
            const Cell4 o = stage2_update(W[k], W1[k], R, dt, p.thr, clamp, mk);
            Wout[k] = o;
            bad = !isfinite(o.H) || !isfinite(o.HU) || !isfinite(o.HV);
            rr = cfl_ratio(o.H, o.HU, o.HV, ar, m.perim[k], p.g, p.thr);
        }
        if (TAPE) {
            tp.R[3 * k] = R[0];
            tp.R[3 * k + 1] = R[1];
            tp.R[3 * k + 2] = R[2];
            tp.mask[k] = mk;
        }
    }
    if (STAGE == 2 && bad) {
        atomicOr(&c->err, 1);
        atomicMin(&c->err_step, step);
    }
    block_count_atomic(clamp, &c->clamps);
    if (STAGE == 2) {
        block_min_atomic(rr, TAPE ? tp.rmin : &sgs->rmin[slot ^ 1]);
        stage2_bookkeeping(c, sgs, ti, tm.nseg, slot, step, true, dt, tn, p.t_stop, log);
    }
}

template <int STAGE>
__global__ __launch_bounds__(kBlock) void stage_kernel(DevMesh m, TileMap tm,
                                                       Cell4* __restrict__ Wa,
                                                       Cell4* __restrict__ Wb,
                                                       Cell4* __restrict__ W1, StepParams p,
                                                       Ctrl* c, Seg* sg, int slot, int step_arg,
                                                       double* log) {
    stage_body<STAGE, false>(m, tm, Wa, Wb, W1, p, c, sg, slot, step_arg, log, Tape{});
}

template <int STAGE>
__global__ __launch_bounds__(kBlock) void stage_tape_kernel(DevMesh m, TileMap tm,
                                                            Cell4* __restrict__ W,
                                                            Cell4* __restrict__ Wout,
                                                            Cell4* __restrict__ W1, StepParams p,
                                                            Ctrl* c, Seg* sg, int slot,
                                                            int step_arg, double* log, Tape tp) {
    stage_body<STAGE, true>(m, tm, W, Wout, W1, p, c, sg, slot, step_arg, log, tp);
}

template __global__ void stage_kernel<1>(DevMesh, TileMap, Cell4*, Cell4*, Cell4*, StepParams,
                                         Ctrl*, Seg*, int, int, double*);
template __global__ void stage_kernel<2>(DevMesh, TileMap, Cell4*, Cell4*, Cell4*, StepParams,
                                         Ctrl*, Seg*, int, int, double*);
template __global__ void stage_tape_kernel<1>(DevMesh, TileMap, Cell4*, Cell4*, Cell4*,
                                              StepParams, Ctrl*, Seg*, int, int, double*, Tape);
template __global__ void stage_tape_kernel<2>(DevMesh, TileMap, Cell4*, Cell4*, Cell4*,
                                              StepParams, Ctrl*, Seg*, int, int, double*, Tape);

// ---------------------------------------------------------------- gauges

// Free surface eta = H - h at the gauge cells after step `step`, if the
// gauge's scenario took the step (steps_done counts the steps it took in
// this call; once a scenario stops, it takes no later step of the call).
__global__ void gauge_kernel(const Cell4* __restrict__ Wa, const Cell4* __restrict__ Wb,
                             const int64_t* __restrict__ cells, int ng,
                             const int32_t* __restrict__ gseg, const Seg* sg, const Ctrl* c,
                             int step_arg, double* __restrict__ log) {
    const int gi = int(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gi >= ng) return;
    const int step = c->kbase + step_arg;
    const Cell4 *Win, *W;
    step_buffers(c, step, Wa, Wb, Win, W);
    const int64_t k = cells[gi];
    if (sg[gseg[gi]].steps_done <= step) return;
    const Cell4 q = W[k];
    log[int64_t(step) * ng + gi] = q.H - q.h;
}

// ---------------------------------------------------------------- state transfer

// Caller-order arrays (H, HU, HV) into internal-order state records; the
// still-water depth comes from h (internal order), copied to both buffers.
__global__ void pack_state_kernel(int64_t n, const int64_t* __restrict__ perm,
                                  const double* __restrict__ H, const double* __restrict__ HU,
                                  const double* __restrict__ HV, const double* __restrict__ h,
                                  Cell4* __restrict__ W, Cell4* __restrict__ W1) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t k = perm[i];
    if (k < 0) return;
    Cell4 q;
    q.H = H[k];
    q.HU = HU[k];
    q.HV = HV[k];
    q.h = h[i];
    W[i] = q;
    W1[i] = q;
}

__global__ void check_state_kernel(int64_t nc, const double* __restrict__ H,
                                   const double* __restrict__ HU, const double* __restrict__ HV,
                                   int* flag) {
    const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    int f = 0;
    if (k < nc) {
        const double a = H[k], b = HU[k], d = HV[k];
        if (!isfinite(a) || !isfinite(b) || !isfinite(d)) f |= 1;
        if (a < 0.0) f |= 2;
    }
    if (f) atomicOr(flag, f);
}

// Internal-order state records into caller-order arrays.
__global__ void unpack_state_kernel(int64_t n, const int64_t* __restrict__ perm,
                                    const Cell4* __restrict__ W, double* __restrict__ H,
                                    double* __restrict__ HU, double* __restrict__ HV) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t k = perm[i];
    if (k < 0) return;
    const Cell4 q = W[i];
    if (H) H[k] = q.H;
    if (HU) HU[k] = q.HU;
    if (HV) HV[k] = q.HV;
}

}  // namespace vsw
