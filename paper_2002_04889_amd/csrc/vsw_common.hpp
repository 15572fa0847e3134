// Device helpers shared by the FP64 and FP32 stage kernels: time step from
// the control block, CFL ratio, block reductions, XCD-aware tile order and
// the stage-2 time bookkeeping.
#pragma once
#include "vsw_kernels.hpp"

namespace vsw {

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

struct TileInfo {
    int seg;     // scenario of the tile
    bool first;  // first tile of its scenario
    int cnt;     // cells in the tile (1..kTile)
};

__device__ __forceinline__ TileInfo tile_info(uint32_t v) {
    TileInfo t;
    t.seg = int(v >> 10);
    t.first = ((v >> 9) & 1u) != 0;
    t.cnt = int(v & 511u) + 1;
    return t;
}

// dt of the scenario's step using control slot `slot`: CFL rule (or fixed
// dt), clipped so the time lands exactly on t_stop.  False if the step is
// not taken.
__device__ __forceinline__ bool step_dt(const Ctrl* c, const Seg* sg, int slot,
                                        const StepParams& p, double& dt, double& tn) {
    if (c->err) return false;
    const double t = sg->t[slot];
    if (!(t < p.t_stop)) return false;
    const unsigned long long rb = sg->rmin[slot];
    double d = (p.dt_fixed > 0.0) ? p.dt_fixed : p.cfl * __longlong_as_double((long long)rb);
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

// The two state buffers of step `step` of the call: w^n is read from in,
// w^{n+1} written to out.
template <class T>
__device__ __forceinline__ void step_buffers(const Ctrl* c, int step, T* Wa, T* Wb, T*& in,
                                             T*& out) {
    const bool odd = ((c->par + step) & 1) != 0;
    in = odd ? Wb : Wa;
    out = odd ? Wa : Wb;
}

// A scenario whose time has reached t_stop takes no more steps in this call;
// its cells are carried into the buffer the step writes (not after an error,
// where the failing step's input stays where it is).
template <class T>
__device__ __forceinline__ void carry_state(const Ctrl* c, const Seg* sg, int slot,
                                            const StepParams& p, const T* __restrict__ in,
                                            T* __restrict__ out, int64_t c0, int cnt) {
    if (c->err || sg->t[slot] < p.t_stop) return;
    const int i = threadIdx.x;
    if (i < cnt) out[c0 + i] = in[c0 + i];
}

// CFL ratio |K| / (P_K (|u| + sqrt(g H))) of a wet cell, +inf otherwise.
// Where g H >= 2^-600, sqrt(g H) >= 2^-300 and a speed |u| below 2^-383
// does not change the sum: |u| is then taken as sqrt(max(u^2 + v^2,
// 2^-767)), which keeps sqrt_n in its range, and the sum is the same
// number.  Other cells, and momenta with tiny_num, take the plain form.
__device__ __forceinline__ double cfl_ratio(double H, double HU, double HV, double area,
                                            double perim, double g, double thr) {
    if (!(H >= thr)) return __longlong_as_double(0x7FF0000000000000ll);
    const double gH = g * H;
    const Rcp dh = rcp_of(H);
    const double u = quot(HU, dh), v = quot(HV, dh);
    const double uu = u * u + v * v;
    const double s = sqrt_n(__builtin_fmax(uu, 0x1p-767)) + sqrt_n(gH);
    const double ps = perim * s;
    double r = quot(area, rcp_of(ps));
    if (wave_any(!(gH >= 0x1p-600) || tiny_num(HU) || tiny_num(HV))) {
        const double u2 = HU / H, v2 = HV / H;
        r = area / (perim * (sqrt(u2 * u2 + v2 * v2) + sqrt(gH)));
    }
    return r;
}

// Block-wide min of a positive double over NT threads, then one atomic min
// on its bits.  The bits of positive doubles order like the values; a plain
// read first skips the atomic when the target already holds a value at
// least as small (values only decrease, so a stale read never loses one).
template <int NT = kBlock>
__device__ __forceinline__ void block_min_atomic(double v, unsigned long long* target) {
    __shared__ double part[NT / 64];
    v = wave_min(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) part[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = part[0];
#pragma unroll
        for (int i = 1; i < NT / 64; ++i) m = (part[i] < m) ? part[i] : m;
        const unsigned long long b = dbits(m);
        if (m < __longlong_as_double(0x7FF0000000000000ll) &&
            b < __hip_atomic_load(target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMin(target, b);
    }
}

template <int NT = kBlock>
__device__ __forceinline__ void block_count_atomic(unsigned long long v, unsigned long long* target) {
    __shared__ unsigned long long part[NT / 64];
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) part[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) s += part[i];
        if (s) atomicAdd(target, s);
    }
}

// block_count_atomic and block_min_atomic in one pass (one barrier).
template <int NT>
__device__ __forceinline__ void block_count_min_atomic(unsigned long long n,
                                                       unsigned long long* count, double v,
                                                       unsigned long long* target) {
    __shared__ unsigned long long pn[NT / 64];
    __shared__ double pv[NT / 64];
    n = wave_sum(n);
    v = wave_min(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        pn[wid] = n;
        pv[wid] = v;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long s = 0;
        double m = pv[0];
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) {
            s += pn[i];
            m = (pv[i] < m) ? pv[i] : m;
        }
        if (s) atomicAdd(count, s);
        const unsigned long long b = dbits(m);
        if (m < __longlong_as_double(0x7FF0000000000000ll) &&
            b < __hip_atomic_load(target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMin(target, b);
    }
}

// Stage 1: w1 = w + dt R(w), then the post-stage fix (negative depth set to
// zero and counted; velocity zero below H_thr).
// mk: bit 0 cleared when the depth is clamped, bit 1 when the momentum is
// zeroed (what the adjoint of the fix needs).
__device__ __forceinline__ Cell4 stage1_update(const Cell4& w, const double R[3], double dt,
                                               double thr, unsigned long long& clamp,
                                               uint8_t& mk) {
    Cell4 o;
    o.H = w.H + dt * R[0];
    o.HU = w.HU + dt * R[1];
    o.HV = w.HV + dt * R[2];
    o.h = w.h;
    mk = 3;
    if (o.H < 0.0) { o.H = 0.0; clamp = 1; mk &= uint8_t(~1u); }
    if (o.H < thr) { o.HU = 0.0; o.HV = 0.0; mk &= uint8_t(~2u); }
    return o;
}

// Stage 2: w^{n+1} = w/2 + (w1 + dt R(w1))/2, then the post-stage fix.
__device__ __forceinline__ Cell4 stage2_update(const Cell4& w, const Cell4& w1, const double R[3],
                                               double dt, double thr, unsigned long long& clamp,
                                               uint8_t& mk) {
    Cell4 o;
    o.H = 0.5 * w.H + 0.5 * (w1.H + dt * R[0]);
    o.HU = 0.5 * w.HU + 0.5 * (w1.HU + dt * R[1]);
    o.HV = 0.5 * w.HV + 0.5 * (w1.HV + dt * R[2]);
    o.h = w.h;
    mk = 3;
    if (o.H < 0.0) { o.H = 0.0; clamp = 1; mk &= uint8_t(~1u); }
    if (o.H < thr) { o.HU = 0.0; o.HV = 0.0; mk &= uint8_t(~2u); }
    return o;
}

// Time bookkeeping of a scenario at the end of stage 2 (thread 0 of the
// scenario's first tile) or, for a step that is not taken, the carry-over of
// the time and the no-valid-dt error.
__device__ __forceinline__ void stage2_bookkeeping(Ctrl* c, Seg* sg, const TileInfo& ti, int nseg,
                                                   int slot, int step, bool active, double dt,
                                                   double tn, double t_stop, double* log) {
    if (!ti.first || threadIdx.x != 0) return;
    if (active) {
        sg->t[slot ^ 1] = tn;
        sg->dt_last = dt;
        sg->steps_done += 1;
        const int64_t e = 2 * (int64_t(step) * nseg + ti.seg);
        log[e] = tn;
        log[e + 1] = dt;
    } else {
        const double t = sg->t[slot];
        sg->t[slot ^ 1] = t;
        if (!c->err && t < t_stop) {  // no valid time step
            atomicOr(&c->err, 2);
            atomicMin(&c->err_step, step);
        }
    }
}

// Face state j of cell k from a face buffer (two-pass organisation).
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
    const Nbr4 nb = m.nbr[k];
    const uint32_t sl[3] = {nb.s0, nb.s1, nb.s2};
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const uint32_t s = sl[j];
        const bool wall = (s == kWallSlot);
        const Face own = load_face(fb, nc, j, k);
        const Face other = wall ? own : load_face(fb, nc, int(s & 3u), int64_t(s >> 3));
        double tt[3];
        const bool left = face_term(g, hg, own, other, wall, (s & 4u) != 0, gf(m, 0, j, k),
                                    gf(m, 1, j, k), gf(m, 2, j, k), tt);
        if (left) {
            a0 = a0 - tt[0]; a1 = a1 - tt[1]; a2 = a2 - tt[2];
        } else {
            a0 = a0 + tt[0]; a1 = a1 + tt[1]; a2 = a2 + tt[2];
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

// A face state in LDS: eta, h, u, v at slot + c * stride.  The face depth H
// is read only by the cell that owns the face (its pressure correction),
// which keeps it in registers.
__device__ __forceinline__ void lds_store_face(double* lds, int stride, int slot, const Face& f) {
    lds[0 * stride + slot] = f.eta;
    lds[1 * stride + slot] = f.h;
    lds[2 * stride + slot] = f.u;
    lds[3 * stride + slot] = f.v;
}

__device__ __forceinline__ Face lds_load_face(const double* lds, int stride, int slot, double H) {
    Face f;
    f.eta = lds[0 * stride + slot];
    f.h = lds[1 * stride + slot];
    f.H = H;
    f.u = lds[2 * stride + slot];
    f.v = lds[3 * stride + slot];
    return f;
}

// First phase of the tile kernels (one workgroup per tile t of cnt cells
// starting at cell c0, one thread per cell): reconstruct the tile's cells
// (Section 2.4) and store their three face states in LDS slots j kTile + i;
// reconstruct the halo cells across the tile boundary and store the face
// each shares with the tile in slots 3 kTile + b.  Thread i keeps its own
// face depths, the centred bed source and the order.  The caller
// synchronises the workgroup before reading the LDS.
__device__ __forceinline__ void tile_faces(const DevMesh& m, const TileMap& tm,
                                           const Cell4* __restrict__ Ws, int t, int64_t c0,
                                           int cnt, double thr, double hg, double* lds,
                                           int stride, double ownH[3], double sc[2],
                                           bool& second) {
    const int i = threadIdx.x;
    const int64_t k = c0 + i;
    sc[0] = 0.0;
    sc[1] = 0.0;
    ownH[0] = ownH[1] = ownH[2] = 0.0;
    second = false;
    if (i < cnt) {
        Recon r;
        recon_core(m, Ws, k, thr, r);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const Face f = recon_face(r, j, thr);
            lds_store_face(lds, stride, j * kTile + i, f);
            ownH[j] = f.H;
        }
        centred_source(m, r, k, hg, sc);
        second = r.second;
    }
    const int b0 = tm.bstart[t], nb = tm.bstart[t + 1] - b0;
    for (int b = i; b < nb; b += kBlock) {
        const uint32_t item = tm.bitem[b0 + b];
        const int64_t n = int64_t(item >> 2);
        const int jn = int(item & 3u);
        Recon r;
        recon_core(m, Ws, n, thr, r);
        lds_store_face(lds, stride, 3 * kTile + b, recon_face_sel(r, jn, thr));
    }
}

// Tiles are consecutive Hilbert ranges, so tiles t and t+1 are neighbours in
// space.  Workgroups are dealt round-robin to the eight XCDs, each with its
// own L2; give XCD x one contiguous run of tiles so that the halo cells
// shared by neighbouring tiles are read through the same L2.
__device__ __forceinline__ int xcd_tile(int w, int ntiles) {
    const int per = ntiles / 8, rem = ntiles % 8;
    const int x = w % 8, idx = w / 8;
    return (x < rem) ? x * (per + 1) + idx : rem * (per + 1) + (x - rem) * per + idx;
}

}  // namespace vsw
