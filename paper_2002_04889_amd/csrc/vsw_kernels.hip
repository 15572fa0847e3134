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
#include "vsw_kernels.hpp"

namespace vsw {

namespace {

__device__ __forceinline__ unsigned long long dbits(double x) {
    return (unsigned long long)__double_as_longlong(x);
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        double w = __shfl_xor(v, o, 64);
        v = (w < v) ? w : v;
    }
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// dt of the step using control slot `slot`: CFL rule (or fixed dt), clipped
// so the time lands exactly on t_stop.  False if the step is not taken.
__device__ __forceinline__ bool step_dt(const Ctrl* c, int slot, const StepParams& p,
                                        double& dt, double& tn) {
    if (c->err) return false;
    const double t = c->t[slot];
    if (!(t < p.t_stop)) return false;
    double d = (p.dt_fixed > 0.0) ? p.dt_fixed
                                  : p.cfl * __longlong_as_double((long long)c->rmin[slot]);
    const double rem = p.t_stop - t;
    if (d >= rem) {
        d = rem;
        tn = p.t_stop;
    } else {
        tn = t + d;
    }
    if (!(d > 0.0) || !isfinite(d)) return false;
    dt = d;
    return true;
}

// CFL ratio |K| / (P_K (|u| + sqrt(g H))) of a wet cell, +inf otherwise.
__device__ __forceinline__ double cfl_ratio(double H, double HU, double HV, double area,
                                            double perim, double g, double thr) {
    if (!(H >= thr)) return __longlong_as_double(0x7FF0000000000000ll);
    const double u = HU / H, v = HV / H;
    const double s = sqrt(u * u + v * v) + sqrt(g * H);
    return area / (perim * s);
}

// Block-wide min of a positive double, then one atomic min on its bits.
__device__ __forceinline__ void block_min_atomic(double v, unsigned long long* target) {
    __shared__ double part[kBlock / 64];
    v = wave_min(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) part[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = part[0];
#pragma unroll
        for (int i = 1; i < kBlock / 64; ++i) m = (part[i] < m) ? part[i] : m;
        if (m < __longlong_as_double(0x7FF0000000000000ll)) atomicMin(target, dbits(m));
    }
}

__device__ __forceinline__ void block_count_atomic(unsigned long long v, unsigned long long* target) {
    __shared__ unsigned long long part[kBlock / 64];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) part[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
#pragma unroll
        for (int i = 0; i < kBlock / 64; ++i) s += part[i];
        if (s) atomicAdd(target, s);
    }
}

}  // namespace

// ---------------------------------------------------------------- control

__global__ void ctrl_init_kernel(Ctrl* c, double t0) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c->rmin[0] = 0x7FF0000000000000ull;
        c->rmin[1] = 0x7FF0000000000000ull;
        c->t[0] = t0;
        c->t[1] = t0;
        c->err = 0;
        c->err_step = 0x7FFFFFFF;
        c->steps_done = 0;
        c->clamps = 0;
        c->dt_last = 0.0;
    }
}

__global__ __launch_bounds__(kBlock) void dt_init_kernel(DevMesh m, const double* __restrict__ H,
                                                         const double* __restrict__ HU,
                                                         const double* __restrict__ HV,
                                                         double g, double thr, Ctrl* c) {
    const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    double r = __longlong_as_double(0x7FF0000000000000ll);
    if (k < m.nc) r = cfl_ratio(H[k], HU[k], HV[k], m.area[k], m.perim[k], g, thr);
    block_min_atomic(r, &c->rmin[0]);
}

// ---------------------------------------------------------------- stage kernels

__global__ __launch_bounds__(kBlock) void recon_kernel(DevMesh m, const double* __restrict__ H,
                                                       const double* __restrict__ HU,
                                                       const double* __restrict__ HV,
                                                       FaceBuf fb, StepParams p, const Ctrl* c,
                                                       int slot) {
    double dt, tn;
    if (!step_dt(c, slot, p, dt, tn)) return;
    const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    if (k >= m.nc) return;
    const int64_t nc = m.nc;
    Face f[3];
    double sc[2];
    const bool second = recon_cell(m, H, HU, HV, k, p.thr, p.hg, f, sc);
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

__device__ __forceinline__ Face load_face(const FaceBuf& fb, int64_t nc, int j, int64_t k) {
    Face f;
    f.eta = fb.f[(5 * j + 0) * nc + k];
    f.h = fb.f[(5 * j + 1) * nc + k];
    f.H = fb.f[(5 * j + 2) * nc + k];
    f.u = fb.f[(5 * j + 3) * nc + k];
    f.v = fb.f[(5 * j + 4) * nc + k];
    return f;
}

// Residual of cell k from the face buffer: R = (-sum_j +-l_j G_j + S_c)/|K|.
__device__ __forceinline__ void residual_from_faces(const DevMesh& m, const FaceBuf& fb, int64_t k,
                                                    double g, double hg, double R[3]) {
    const int64_t nc = m.nc;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const uint32_t s = m.nbr[j * nc + k];
        const Face own = load_face(fb, nc, j, k);
        const double l = gf(m, 2, j, k);
        double phi[3], p;
        double nx = gf(m, 0, j, k), ny = gf(m, 1, j, k);
        bool left = true;
        if (s == kWallSlot) {
            wall_flux(g, hg, own, nx, ny, phi, p);
        } else {
            const int64_t n = int64_t(s >> 3);
            const int jn = int(s & 3u);
            const Face other = load_face(fb, nc, jn, n);
            double pl, pr;
            if (s & 4u) {
                face_flux(g, hg, own, other, nx, ny, phi, pl, pr);
                p = pl;
            } else {
                left = false;
                nx = -nx;
                ny = -ny;
                face_flux(g, hg, other, own, nx, ny, phi, pl, pr);
                p = pr;
            }
        }
        const double t0 = l * phi[0];
        const double t1 = l * (phi[1] + p * nx);
        const double t2 = l * (phi[2] + p * ny);
        if (left) {
            a0 = a0 - t0; a1 = a1 - t1; a2 = a2 - t2;
        } else {
            a0 = a0 + t0; a1 = a1 + t1; a2 = a2 + t2;
        }
    }
    if (fb.order[k] == 2) {
        a1 = a1 + fb.sc[k];
        a2 = a2 + fb.sc[nc + k];
    }
    const double ar = m.area[k];
    R[0] = a0 / ar;
    R[1] = a1 / ar;
    R[2] = a2 / ar;
}

// Stage 1: w1 = w + dt R(w), then the post-stage fix.
__global__ __launch_bounds__(kBlock) void update1_kernel(DevMesh m, const double* __restrict__ H,
                                                         const double* __restrict__ HU,
                                                         const double* __restrict__ HV,
                                                         double* __restrict__ H1,
                                                         double* __restrict__ HU1,
                                                         double* __restrict__ HV1, FaceBuf fb,
                                                         StepParams p, Ctrl* c, int slot) {
    double dt, tn;
    if (!step_dt(c, slot, p, dt, tn)) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) c->rmin[slot ^ 1] = 0x7FF0000000000000ull;
    const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    unsigned long long clamp = 0;
    if (k < m.nc) {
        double R[3];
        residual_from_faces(m, fb, k, p.g, p.hg, R);
        double h1 = H[k] + dt * R[0];
        double u1 = HU[k] + dt * R[1];
        double v1 = HV[k] + dt * R[2];
        if (h1 < 0.0) { h1 = 0.0; clamp = 1; }
        if (h1 < p.thr) { u1 = 0.0; v1 = 0.0; }
        H1[k] = h1;
        HU1[k] = u1;
        HV1[k] = v1;
    }
    block_count_atomic(clamp, &c->clamps);
}

// Stage 2: w^{n+1} = w/2 + (w1 + dt R(w1))/2, post-stage fix, the CFL ratio
// of the new state, and the time bookkeeping (block 0).
__global__ __launch_bounds__(kBlock) void update2_kernel(DevMesh m, double* __restrict__ H,
                                                         double* __restrict__ HU,
                                                         double* __restrict__ HV,
                                                         const double* __restrict__ H1,
                                                         const double* __restrict__ HU1,
                                                         const double* __restrict__ HV1,
                                                         FaceBuf fb, StepParams p, Ctrl* c,
                                                         int slot, int step, double* tlog,
                                                         double* dtlog) {
    double dt, tn;
    const bool active = step_dt(c, slot, p, dt, tn);
    if (!active) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            const double t = c->t[slot];
            c->t[slot ^ 1] = t;
            if (!c->err && t < p.t_stop) {  // no valid time step
                c->err = 2;
                c->err_step = step;
            }
        }
        return;
    }
    const int64_t k = int64_t(blockIdx.x) * kBlock + threadIdx.x;
    unsigned long long clamp = 0;
    double r = __longlong_as_double(0x7FF0000000000000ll);
    bool bad = false;
    if (k < m.nc) {
        double R[3];
        residual_from_faces(m, fb, k, p.g, p.hg, R);
        double hn = 0.5 * H[k] + 0.5 * (H1[k] + dt * R[0]);
        double un = 0.5 * HU[k] + 0.5 * (HU1[k] + dt * R[1]);
        double vn = 0.5 * HV[k] + 0.5 * (HV1[k] + dt * R[2]);
        if (hn < 0.0) { hn = 0.0; clamp = 1; }
        if (hn < p.thr) { un = 0.0; vn = 0.0; }
        H[k] = hn;
        HU[k] = un;
        HV[k] = vn;
        bad = !isfinite(hn) || !isfinite(un) || !isfinite(vn);
        r = cfl_ratio(hn, un, vn, m.area[k], m.perim[k], p.g, p.thr);
    }
    if (bad) {
        atomicOr(&c->err, 1);
        atomicMin(&c->err_step, step);
    }
    block_count_atomic(clamp, &c->clamps);
    block_min_atomic(r, &c->rmin[slot ^ 1]);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        c->t[slot ^ 1] = tn;
        c->dt_last = dt;
        c->steps_done += 1;
        tlog[step] = tn;
        dtlog[step] = dt;
    }
}

// ---------------------------------------------------------------- fused stage

namespace {

// Tiles are consecutive Hilbert ranges, so tiles t and t+1 are neighbours in
// space.  Workgroups are dealt round-robin to the eight XCDs, each with its
// own L2; give XCD x one contiguous run of tiles so that the halo cells
// shared by neighbouring tiles are read through the same L2.
__device__ __forceinline__ int xcd_tile(int w, int ntiles) {
    const int per = ntiles / 8, rem = ntiles % 8;
    const int x = w % 8, idx = w / 8;
    return (x < rem) ? x * (per + 1) + idx : rem * (per + 1) + (x - rem) * per + idx;
}

__device__ __forceinline__ void lds_store_face(double* lds, int stride, int slot, const Face& f) {
    lds[0 * stride + slot] = f.eta;
    lds[1 * stride + slot] = f.h;
    lds[2 * stride + slot] = f.H;
    lds[3 * stride + slot] = f.u;
    lds[4 * stride + slot] = f.v;
}

__device__ __forceinline__ Face lds_load_face(const double* lds, int stride, int slot) {
    Face f;
    f.eta = lds[0 * stride + slot];
    f.h = lds[1 * stride + slot];
    f.H = lds[2 * stride + slot];
    f.u = lds[3 * stride + slot];
    f.v = lds[4 * stride + slot];
    return f;
}

}  // namespace

// One workgroup per tile of kTile cells, one thread per cell:
//  1. reconstruct the tile's cells (Section 2.4) and store their three face
//     states in LDS; reconstruct the halo cells across the tile boundary and
//     store the face each shares with the tile;
//  2. per cell, the three face fluxes in canonical orientation from LDS (one
//     branch-free evaluation per face), the centred bed source, the residual
//     and the Runge-Kutta stage.
// Each face inside a tile is evaluated by both of its cells; a face list
// evaluated once per face (edge-parallel, with two more barriers to hand the
// terms over) measured slower on the 1M-cell basin.
template <int STAGE>
__global__ __launch_bounds__(kBlock) void stage_kernel(DevMesh m, TileMap tm, double* __restrict__ H,
                                                       double* __restrict__ HU,
                                                       double* __restrict__ HV,
                                                       double* __restrict__ H1,
                                                       double* __restrict__ HU1,
                                                       double* __restrict__ HV1, StepParams p,
                                                       Ctrl* c, int slot, int step, double* tlog,
                                                       double* dtlog) {
    extern __shared__ double lds[];
    const int stride = 3 * kTile + tm.bmax;
    double dt, tn;
    const bool active = step_dt(c, slot, p, dt, tn);
    if (!active) {
        if (STAGE == 2 && blockIdx.x == 0 && threadIdx.x == 0) {
            const double t = c->t[slot];
            c->t[slot ^ 1] = t;
            if (!c->err && t < p.t_stop) {  // no valid time step
                c->err = 2;
                c->err_step = step;
            }
        }
        return;
    }
    if (STAGE == 1 && blockIdx.x == 0 && threadIdx.x == 0) c->rmin[slot ^ 1] = 0x7FF0000000000000ull;
    // state the stage reconstructs: w^n in stage 1, w1 in stage 2
    const double* __restrict__ Hs = (STAGE == 1) ? H : H1;
    const double* __restrict__ HUs = (STAGE == 1) ? HU : HU1;
    const double* __restrict__ HVs = (STAGE == 1) ? HV : HV1;
    const int64_t nc = m.nc;
    const int t = xcd_tile(int(blockIdx.x), tm.ntiles);
    const int64_t c0 = int64_t(t) * kTile;
    const int cnt = int(min(int64_t(kTile), nc - c0));
    const int i = threadIdx.x;
    const int64_t k = c0 + i;

    // 1. reconstruction of the tile's cells and of its halo faces
    double sc[2] = {0.0, 0.0};
    bool second = false;
    if (i < cnt) {
        Recon r;
        recon_core(m, Hs, HUs, HVs, k, p.thr, r);
#pragma unroll
        for (int j = 0; j < 3; ++j) lds_store_face(lds, stride, j * kTile + i, recon_face(r, j, p.thr));
        centred_source(m, r, k, p.hg, sc);
        second = r.second;
    }
    const int b0 = tm.bstart[t], nb = tm.bstart[t + 1] - b0;
    for (int b = i; b < nb; b += kBlock) {
        const uint32_t item = tm.bitem[b0 + b];
        const int64_t n = int64_t(item >> 2);
        const int jn = int(item & 3u);
        Recon r;
        recon_core(m, Hs, HUs, HVs, n, p.thr, r);
        const Face f = (jn == 0) ? recon_face(r, 0, p.thr)
                     : (jn == 1) ? recon_face(r, 1, p.thr) : recon_face(r, 2, p.thr);
        lds_store_face(lds, stride, 3 * kTile + b, f);
    }
    __syncthreads();

    // 3. residual and Runge-Kutta stage per cell
    unsigned long long clamp = 0;
    double rr = __longlong_as_double(0x7FF0000000000000ll);
    bool bad = false;
    if (i < cnt) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const uint16_t s = tm.nloc[j * nc + k];
            const bool wall = (s == kNlocWall16);
            const Face own = lds_load_face(lds, stride, j * kTile + i);
            const Face other = lds_load_face(lds, stride, wall ? j * kTile + i : int(s & 0x7FFFu));
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
        const double R0 = a0 / ar, R1 = a1 / ar, R2 = a2 / ar;
        if (STAGE == 1) {
            double h1 = H[k] + dt * R0;
            double u1 = HU[k] + dt * R1;
            double v1 = HV[k] + dt * R2;
            if (h1 < 0.0) { h1 = 0.0; clamp = 1; }
            if (h1 < p.thr) { u1 = 0.0; v1 = 0.0; }
            H1[k] = h1;
            HU1[k] = u1;
            HV1[k] = v1;
        } else {
            double hn = 0.5 * H[k] + 0.5 * (H1[k] + dt * R0);
            double un = 0.5 * HU[k] + 0.5 * (HU1[k] + dt * R1);
            double vn = 0.5 * HV[k] + 0.5 * (HV1[k] + dt * R2);
            if (hn < 0.0) { hn = 0.0; clamp = 1; }
            if (hn < p.thr) { un = 0.0; vn = 0.0; }
            H[k] = hn;
            HU[k] = un;
            HV[k] = vn;
            bad = !isfinite(hn) || !isfinite(un) || !isfinite(vn);
            rr = cfl_ratio(hn, un, vn, ar, m.perim[k], p.g, p.thr);
        }
    }
    if (STAGE == 2 && bad) {
        atomicOr(&c->err, 1);
        atomicMin(&c->err_step, step);
    }
    block_count_atomic(clamp, &c->clamps);
    if (STAGE == 2) {
        block_min_atomic(rr, &c->rmin[slot ^ 1]);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            c->t[slot ^ 1] = tn;
            c->dt_last = dt;
            c->steps_done += 1;
            tlog[step] = tn;
            dtlog[step] = dt;
        }
    }
}

template __global__ void stage_kernel<1>(DevMesh, TileMap, double*, double*, double*, double*,
                                         double*, double*, StepParams, Ctrl*, int, int, double*,
                                         double*);
template __global__ void stage_kernel<2>(DevMesh, TileMap, double*, double*, double*, double*,
                                         double*, double*, StepParams, Ctrl*, int, int, double*,
                                         double*);

// ---------------------------------------------------------------- permutation

__global__ void gather_kernel(int64_t n, const int64_t* __restrict__ perm,
                              const double* __restrict__ src, double* __restrict__ dst) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[perm[i]];
}

__global__ void scatter_kernel(int64_t n, const int64_t* __restrict__ perm,
                               const double* __restrict__ src, double* __restrict__ dst) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) dst[perm[i]] = src[i];
}

}  // namespace vsw
