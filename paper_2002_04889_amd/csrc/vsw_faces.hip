// Face-parallel FP64 stage kernels of the SSP-RK(2,2) step (Section 2.3).
//
// One workgroup per tile of T consecutive cells (T = 128, 256 or 512, one
// thread per cell), in three phases:
//   1. reconstruct (Section 2.4, eq. (3)) the tile's cells and the halo
//      cells across its boundary into LDS face slots; the geometry (face
//      midpoint offsets, area, wall normals) comes from the cell's vertex
//      coordinates, the least-squares weights from memory;
//   2. evaluate every face of the tile once, in canonical orientation: the
//      HLL flux with the hydrostatic reconstruction (Section 2.2), the face
//      normal and length from its two vertices, and for each side of the
//      face its term l (phi + (0, p n)) and its part of the centred bed
//      source, written over the face states of that side's slot (each slot
//      belongs to one face, so no other thread reads it);
//   3. per cell: the three terms in local face order, the source, the
//      residual and the Runge-Kutta stage (and in stage 2 the next CFL
//      minimum).
// Every quantity is computed by the same expressions in the same order as
// the cell-parallel kernels on the host-computed geometry, so both give
// bitwise the same results; a face is evaluated once instead of once per
// side, and the flux geometry (face normals, lengths, midpoint offsets,
// areas) is not read from memory.
#include "vsw_common.hpp"
#include "vsw_faces.hpp"

namespace vsw {

namespace {

// Vertex coordinates of a cell in local order.
struct Tri {
    double x[3], y[3];
};

__device__ __forceinline__ Tri load_tri(const FaceMesh& m, const TopoD& tp) {
    const double2 p0 = m.vxy[tp.v0], p1 = m.vxy[tp.v1], p2 = m.vxy[tp.v2];
    return Tri{{p0.x, p1.x, p2.x}, {p0.y, p1.y, p2.y}};
}

// State records of the three neighbours of cell k (k itself across a wall,
// where the record is not used): one load each, without branches.
__device__ __forceinline__ void load_nbrs(const Cell4* __restrict__ W, const TopoD& tp, int64_t k,
                                          Cell4 cn[3]) {
    const uint32_t sl[3] = {tp.n0, tp.n1, tp.n2};
#pragma unroll
    for (int j = 0; j < 3; ++j) cn[j] = W[(sl[j] != kWallSlot) ? int64_t(sl[j] >> 3) : k];
}

__device__ __forceinline__ double tri_area(const Tri& g) {
    const double cr = (g.x[1] - g.x[0]) * (g.y[2] - g.y[0]) - (g.x[2] - g.x[0]) * (g.y[1] - g.y[0]);
    return 0.5 * cr;
}

// Reconstruction of a cell from its loaded state, neighbours, vertices and
// least-squares weights; the wall normals and face-midpoint offsets are
// computed from the vertices as the host computes its stored geometry.
__device__ __forceinline__ void recon_tri(const Cell4& ck, const Cell4 cn[3], const TopoD& tp,
                                          const Tri& g, const LsqW& w, double thr, Recon& r,
                                          int sel = -1) {
    const uint32_t sl[3] = {tp.n0, tp.n1, tp.n2};
    recon_from(
        ck, cn, sl, thr,
        [&](int j, double& nx, double& ny) {
            const int j1 = (j == 2) ? 0 : j + 1;
            const double ex = g.x[j1] - g.x[j], ey = g.y[j1] - g.y[j];
            const double l = sqrt_n(ex * ex + ey * ey);
            const Rcp d = rcp_of(l);
            nx = quot(ey, d);
            ny = quot(-ex, d);
        },
        [&](double* gw, double* gd) {
            // sums of admitted coordinates: zero or at least 2^-352
            const Rcp d3 = rcp_three();
            const double cx = quot((g.x[0] + g.x[1]) + g.x[2], d3);
            const double cy = quot((g.y[0] + g.y[1]) + g.y[2], d3);
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int j1 = (j == 2) ? 0 : j + 1;
                gw[2 * j] = w.w[2 * j];
                gw[2 * j + 1] = w.w[2 * j + 1];
                gd[2 * j] = (g.x[j] + g.x[j1]) * 0.5 - cx;
                gd[2 * j + 1] = (g.y[j] + g.y[j1]) * 0.5 - cy;
            }
        },
        r, sel);
}

// Unit normal (from vertex a to b, turned clockwise) and length of a face.
struct FaceGeo {
    double nx, ny, l;
};

// The mesh upload admits vertex coordinates that are zero or between 2^-300
// and 2^300 in magnitude, so an edge component is zero or at least 2^-352,
// the squared length at least 2^-704 and the length within [2^-352, 2^302]:
// sqrt_n and quot return the correctly rounded values without range tests.
__device__ __forceinline__ FaceGeo face_geo(const double2& pa, const double2& pb) {
    const double ex = pb.x - pa.x, ey = pb.y - pa.y;
    const double l = sqrt_n(ex * ex + ey * ey);
    const Rcp d = rcp_of(l);
    return FaceGeo{quot(ey, d), quot(-ex, d), l};
}

__device__ __forceinline__ void store_face(double* Le, double* Lh, double* LH, double* Lu,
                                           double* Lv, int s, const Face& f) {
    Le[s] = f.eta;
    Lh[s] = f.h;
    LH[s] = f.H;
    Lu[s] = f.u;
    Lv[s] = f.v;
}

}  // namespace

template <int T, int STAGE, bool TAPE>
__device__ __forceinline__ void faces_stage_body(const FaceMesh& m, const FaceTileMap& tm,
                                                 Cell4* __restrict__ Wa, Cell4* __restrict__ Wb,
                                                 Cell4* __restrict__ W1, const StepParams& p,
                                                 Ctrl* c, Seg* sg, int slot, int step_arg,
                                                 double* log, const Tape& tape) {
    extern __shared__ double lds[];
    const int S = 3 * T + tm.bmax;
    // face slots: eta, h, H, u, v of a face state; after phase 2 the face's
    // terms for the slot's cell (three components, source x, source y)
    double* __restrict__ Le = lds;
    double* __restrict__ Lh = lds + S;
    double* __restrict__ LH = lds + 2 * S;
    double* __restrict__ Lu = lds + 3 * S;
    double* __restrict__ Lv = lds + 4 * S;
    double* __restrict__ CH = lds + 5 * S;  // cell depth H_K
    double* __restrict__ Ch = CH + T;       // cell bed depth h_K
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
            carry_state(c, sgs, slot, p, W, Wout, int64_t(t) * T, ti.cnt);
            stage2_bookkeeping(c, sgs, ti, tm.nseg, slot, step, false, 0.0, 0.0, p.t_stop, log);
        }
        return;
    }
    if (STAGE == 1 && ti.first && threadIdx.x == 0) sgs->rmin[slot ^ 1] = 0x7FF0000000000000ull;
    // state the stage reconstructs: w^n in stage 1, w1 in stage 2
    const Cell4* __restrict__ Ws = (STAGE == 1) ? W : W1;
    const int64_t c0 = int64_t(t) * T;
    const int cnt = ti.cnt;
    const int i = threadIdx.x;
    const int64_t k = c0 + i;
    const bool own = i < cnt;
    const int b0 = tm.bstart[t], nb = tm.bstart[t + 1] - b0;
    const int f0 = tm.fstart[t], nf = tm.fstart[t + 1] - f0;

    // The loads are issued in dependency levels, each before the arithmetic
    // that waits for the previous one: (1) the cell's topology, weights and
    // state and the first halo item of the thread; (2) the cell's neighbours
    // and vertices and the halo cell's topology; (3) after the cell's
    // reconstruction, the halo cell's data; (4) after the halo, the first
    // two face records of the thread, their vertices and the records the
    // Runge-Kutta stage reads, all before the first barrier.  (Face records
    // held through the reconstructions would need more than the 128
    // registers of four waves per SIMD.)
    // each level's loads are issued at raised wave priority, so that a wave
    // that reaches them is not held behind the arithmetic of the other waves
    // on its SIMD before its requests are in flight
    __builtin_amdgcn_s_setprio(2);
    const int64_t ko = own ? k : c0;
    const TopoD tp = m.topo[ko];
    const LsqW lw = m.lsq[ko];
    const Cell4 ck = Ws[ko];
    uint32_t hitem = 0;
    if (i < nb) hitem = tm.bitem[b0 + i];
    const Tri tg = load_tri(m, tp);
    Cell4 cn[3];
    load_nbrs(Ws, tp, ko, cn);
    TopoD htp{0u, 0u, 0u, 0u, 0u, 0u};
    if (i < nb) htp = m.topo[hitem >> 2];
    __builtin_amdgcn_s_setprio(0);

    // phase 1: the tile's cells and the halo faces
    double area = 1.0;
    bool second = false;
    if (own) {
        Recon r;
        recon_tri(ck, cn, tp, tg, lw, p.thr, r);
        area = tri_area(tg);
#pragma unroll
        for (int j = 0; j < 3; ++j) store_face(Le, Lh, LH, Lu, Lv, j * T + i, recon_face(r, j, p.thr));
        CH[i] = r.Hk;
        Ch[i] = r.hk;
        second = r.second;
    }
    for (int b = i; b < nb; b += T) {
        const bool pre = (b == i);
        const uint32_t item = pre ? hitem : tm.bitem[b0 + b];
        const int64_t n = int64_t(item >> 2);
        const int jn = int(item & 3u);
        const TopoD tq = pre ? htp : m.topo[n];
        const LsqW lq = m.lsq[n];
        const Cell4 cq = Ws[n];
        const Tri gq = load_tri(m, tq);
        Cell4 cnq[3];
        load_nbrs(Ws, tq, n, cnq);
        Recon r;
        recon_tri(cq, cnq, tq, gq, lq, p.thr, r, jn);
        store_face(Le, Lh, LH, Lu, Lv, 3 * T + b, recon_face(r, 0, p.thr));
    }
    __builtin_amdgcn_s_setprio(2);
    FaceItemD it0{0u, 0u, 0, 0}, it1{0u, 0u, 0, 0};
    if (i < nf) it0 = tm.items[f0 + i];
    if (i + T < nf) it1 = tm.items[f0 + i + T];
    double2 a0 = make_double2(0.0, 0.0), e0 = a0, a1 = a0, e1 = a0;
    if (i < nf) {
        a0 = m.vxy[it0.va];
        e0 = m.vxy[it0.vb];
    }
    if (i + T < nf) {
        a1 = m.vxy[it1.va];
        e1 = m.vxy[it1.vb];
    }
    Cell4 wn{0.0, 0.0, 0.0, 0.0}, w1{0.0, 0.0, 0.0, 0.0};
    double per = 1.0;
    if (own) {
        wn = W[k];
        if (STAGE == 2) {
            w1 = W1[k];
            per = m.perim[k];
        }
    }
    __builtin_amdgcn_s_setprio(0);
    FaceGeo g0{0.0, 0.0, 0.0}, g1{0.0, 0.0, 0.0};
    if (i < nf) g0 = face_geo(a0, e0);
    if (i + T < nf) g1 = face_geo(a1, e1);
    __syncthreads();

    // phase 2: each face once
    for (int q = i; q < nf; q += T) {
        FaceItemD it;
        FaceGeo fg;
        if (q == i) {
            it = it0;
            fg = g0;
        } else if (q == i + T) {
            it = it1;
            fg = g1;
        } else {
            it = tm.items[f0 + q];
            fg = face_geo(m.vxy[it.va], m.vxy[it.vb]);
        }
        const int sl = it.sl;
        const bool wall = (it.sr == kFaceWall);
        const int sr = wall ? sl : int(it.sr);
        const Face L{Le[sl], Lh[sl], LH[sl], Lu[sl], Lv[sl]};
        const Face R{Le[sr], Lh[sr], LH[sr], Lu[sr], Lv[sr]};
        const double nx = fg.nx, ny = fg.ny, l = fg.l;
        double tL[3], tR[3];
        face_pair(p.g, p.hg, L, R, wall, nx, ny, l, tL, tR);
        // the left cell subtracts its term, the right cell adds its own;
        // each side's part of the centred source (Section 2.2 reading) uses
        // that cell's outward normal
        if (sl < 3 * T) {
            const int ci = sl & (T - 1);
            const double cc = (l * (CH[ci] + L.H)) * (L.h - Ch[ci]);
            Le[sl] = -tL[0];
            Lh[sl] = -tL[1];
            LH[sl] = -tL[2];
            Lu[sl] = cc * nx;
            Lv[sl] = cc * ny;
        }
        if (!wall && sr < 3 * T) {
            const int ci = sr & (T - 1);
            const double cc = (l * (CH[ci] + R.H)) * (R.h - Ch[ci]);
            Le[sr] = tR[0];
            Lh[sr] = tR[1];
            LH[sr] = tR[2];
            Lu[sr] = cc * (-nx);
            Lv[sr] = cc * (-ny);
        }
    }
    __syncthreads();

    // phase 3: residual and Runge-Kutta stage per cell
    unsigned long long clamp = 0;
    double rr = __longlong_as_double(0x7FF0000000000000ll);
    bool bad = false;
    if (own) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int sj = j * T + i;
            s0 = s0 + Le[sj];
            s1 = s1 + Lh[sj];
            s2 = s2 + LH[sj];
        }
        if (second) {
            const double sx = (Lu[i] + Lu[T + i]) + Lu[2 * T + i];
            const double sy = (Lv[i] + Lv[T + i]) + Lv[2 * T + i];
            s1 = s1 + p.hg * sx;
            s2 = s2 + p.hg * sy;
        }
        double R[3];
        div_area(s0, s1, s2, area, R);
        uint8_t mk;
        if (STAGE == 1) {
            W1[k] = stage1_update(wn, R, dt, p.thr, clamp, mk);
        } else {
            const Cell4 o = stage2_update(wn, w1, R, dt, p.thr, clamp, mk);
            Wout[k] = o;
            bad = !isfinite(o.H) || !isfinite(o.HU) || !isfinite(o.HV);
            rr = cfl_ratio(o.H, o.HU, o.HV, area, per, p.g, p.thr);
        }
        if (TAPE) {
            tape.R[3 * k] = R[0];
            tape.R[3 * k + 1] = R[1];
            tape.R[3 * k + 2] = R[2];
            tape.mask[k] = mk;
        }
    }
    if (STAGE == 2 && bad) {
        atomicOr(&c->err, 1);
        atomicMin(&c->err_step, step);
    }
    if (STAGE == 2) {
        block_count_min_atomic<T>(clamp, &c->clamps, rr, TAPE ? tape.rmin : &sgs->rmin[slot ^ 1]);
        stage2_bookkeeping(c, sgs, ti, tm.nseg, slot, step, true, dt, tn, p.t_stop, log);
    } else {
        block_count_atomic<T>(clamp, &c->clamps);
    }
}

template <int T, int STAGE>
__global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(4))) void faces_stage_kernel(
    FaceMesh m, FaceTileMap tm, Cell4* __restrict__ Wa, Cell4* __restrict__ Wb,
    Cell4* __restrict__ W1, StepParams p, Ctrl* c, Seg* sg, int slot, int step_arg, double* log) {
    faces_stage_body<T, STAGE, false>(m, tm, Wa, Wb, W1, p, c, sg, slot, step_arg, log, Tape{});
}

template <int T, int STAGE>
__global__ __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(4))) void faces_tape_kernel(
    FaceMesh m, FaceTileMap tm, Cell4* __restrict__ W, Cell4* __restrict__ Wout,
    Cell4* __restrict__ W1, StepParams p, Ctrl* c, Seg* sg, int slot, int step_arg, double* log,
    Tape tp) {
    faces_stage_body<T, STAGE, true>(m, tm, W, Wout, W1, p, c, sg, slot, step_arg, log, tp);
}

template <int T>
__global__ __launch_bounds__(T) void faces_dt_init_kernel(FaceMesh m, FaceTileMap tm,
                                                          const Cell4* __restrict__ W,
                                                          const double* __restrict__ area,
                                                          double g, double thr, Seg* sg) {
    const TileInfo ti = tile_info(tm.tinfo[blockIdx.x]);
    const int64_t k = int64_t(blockIdx.x) * T + threadIdx.x;
    double r = __longlong_as_double(0x7FF0000000000000ll);
    if (int(threadIdx.x) < ti.cnt) {
        const Cell4 q = W[k];
        r = cfl_ratio(q.H, q.HU, q.HV, area[k], m.perim[k], g, thr);
    }
    block_min_atomic<T>(r, &sg[ti.seg].rmin[0]);
}

#define VSW_FACES_INSTANCES(T)                                                                   \
    template __global__ void faces_stage_kernel<T, 1>(FaceMesh, FaceTileMap, Cell4*, Cell4*,     \
                                                      Cell4*, StepParams, Ctrl*, Seg*, int, int, \
                                                      double*);                                  \
    template __global__ void faces_stage_kernel<T, 2>(FaceMesh, FaceTileMap, Cell4*, Cell4*,     \
                                                      Cell4*, StepParams, Ctrl*, Seg*, int, int, \
                                                      double*);                                  \
    template __global__ void faces_dt_init_kernel<T>(FaceMesh, FaceTileMap, const Cell4*,        \
                                                     const double*, double, double, Seg*);
VSW_FACES_INSTANCES(128)
VSW_FACES_INSTANCES(256)
VSW_FACES_INSTANCES(512)
#undef VSW_FACES_INSTANCES

// the adjoint replays tiles of 256 cells
template __global__ void faces_tape_kernel<256, 1>(FaceMesh, FaceTileMap, Cell4*, Cell4*, Cell4*,
                                                   StepParams, Ctrl*, Seg*, int, int, double*,
                                                   Tape);
template __global__ void faces_tape_kernel<256, 2>(FaceMesh, FaceTileMap, Cell4*, Cell4*, Cell4*,
                                                   StepParams, Ctrl*, Seg*, int, int, double*,
                                                   Tape);

}  // namespace vsw
