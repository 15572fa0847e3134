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

// Reconstruction of cell k from its vertices and least-squares weights.
// area (may be null) receives |K|.
__device__ __forceinline__ void recon_geo(const FaceMesh& m, const Cell4* __restrict__ W,
                                          int64_t k, double thr, Recon& r, double* area) {
    const TopoD tp = m.topo[k];
    const double2 p0 = m.vxy[tp.v0], p1 = m.vxy[tp.v1], p2 = m.vxy[tp.v2];
    const double x[3] = {p0.x, p1.x, p2.x}, y[3] = {p0.y, p1.y, p2.y};
    if (area) {
        const double cr = (x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0]);
        *area = 0.5 * cr;
    }
    const uint32_t sl[3] = {tp.n0, tp.n1, tp.n2};
    recon_with(
        W, k, sl, thr,
        [&](int j, double& nx, double& ny) {
            const int j1 = (j == 2) ? 0 : j + 1;
            const double ex = x[j1] - x[j], ey = y[j1] - y[j];
            const double l = sqrt(ex * ex + ey * ey);
            nx = ey / l;
            ny = (-ex) / l;
        },
        [&](double* gw, double* gd) {
            const LsqW w = m.lsq[k];
            const double cx = ((x[0] + x[1]) + x[2]) / 3.0;
            const double cy = ((y[0] + y[1]) + y[2]) / 3.0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int j1 = (j == 2) ? 0 : j + 1;
                gw[2 * j] = w.w[2 * j];
                gw[2 * j + 1] = w.w[2 * j + 1];
                gd[2 * j] = (x[j] + x[j1]) * 0.5 - cx;
                gd[2 * j + 1] = (y[j] + y[j1]) * 0.5 - cy;
            }
        },
        r);
}

}  // namespace

template <int T, int STAGE>
__global__ __launch_bounds__(T) void faces_stage_kernel(FaceMesh m, FaceTileMap tm,
                                                        Cell4* __restrict__ Wa,
                                                        Cell4* __restrict__ Wb,
                                                        Cell4* __restrict__ W1, StepParams p,
                                                        Ctrl* c, Seg* sg, int slot, int step_arg,
                                                        double* log) {
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

    // phase 1: the tile's cells and the halo faces
    double area = 1.0;
    bool second = false;
    if (i < cnt) {
        Recon r;
        recon_geo(m, Ws, k, p.thr, r, &area);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const Face f = recon_face(r, j, p.thr);
            const int sj = j * T + i;
            Le[sj] = f.eta;
            Lh[sj] = f.h;
            LH[sj] = f.H;
            Lu[sj] = f.u;
            Lv[sj] = f.v;
        }
        CH[i] = r.Hk;
        Ch[i] = r.hk;
        second = r.second;
    }
    const int b0 = tm.bstart[t], nb = tm.bstart[t + 1] - b0;
    for (int b = i; b < nb; b += T) {
        const uint32_t item = tm.bitem[b0 + b];
        const int64_t n = int64_t(item >> 2);
        const int jn = int(item & 3u);
        Recon r;
        recon_geo(m, Ws, n, p.thr, r, nullptr);
        const Face f = (jn == 0) ? recon_face(r, 0, p.thr)
                     : (jn == 1) ? recon_face(r, 1, p.thr) : recon_face(r, 2, p.thr);
        const int sb = 3 * T + b;
        Le[sb] = f.eta;
        Lh[sb] = f.h;
        LH[sb] = f.H;
        Lu[sb] = f.u;
        Lv[sb] = f.v;
    }
    __syncthreads();

    // phase 2: each face once
    const int f0 = tm.fstart[t], nf = tm.fstart[t + 1] - f0;
    for (int q = i; q < nf; q += T) {
        const FaceItemD it = tm.items[f0 + q];
        const int sl = it.sl;
        const bool wall = (it.sr == kFaceWall);
        const int sr = wall ? sl : int(it.sr);
        const Face L{Le[sl], Lh[sl], LH[sl], Lu[sl], Lv[sl]};
        const Face R{Le[sr], Lh[sr], LH[sr], Lu[sr], Lv[sr]};
        const double2 pa = m.vxy[it.va], pb = m.vxy[it.vb];
        const double ex = pb.x - pa.x, ey = pb.y - pa.y;
        const double l = sqrt(ex * ex + ey * ey);
        const double nx = ey / l, ny = (-ex) / l;
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
    if (i < cnt) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const int sj = j * T + i;
            a0 = a0 + Le[sj];
            a1 = a1 + Lh[sj];
            a2 = a2 + LH[sj];
        }
        if (second) {
            const double sx = (Lu[i] + Lu[T + i]) + Lu[2 * T + i];
            const double sy = (Lv[i] + Lv[T + i]) + Lv[2 * T + i];
            a1 = a1 + p.hg * sx;
            a2 = a2 + p.hg * sy;
        }
        const double R[3] = {a0 / area, a1 / area, a2 / area};
        uint8_t mk;
        if (STAGE == 1) {
            W1[k] = stage1_update(W[k], R, dt, p.thr, clamp, mk);
        } else {
            const Cell4 o = stage2_update(W[k], W1[k], R, dt, p.thr, clamp, mk);
            Wout[k] = o;
            bad = !isfinite(o.H) || !isfinite(o.HU) || !isfinite(o.HV);
            rr = cfl_ratio(o.H, o.HU, o.HV, area, m.perim[k], p.g, p.thr);
        }
    }
    if (STAGE == 2 && bad) {
        atomicOr(&c->err, 1);
        atomicMin(&c->err_step, step);
    }
    block_count_atomic<T>(clamp, &c->clamps);
    if (STAGE == 2) {
        block_min_atomic<T>(rr, &sgs->rmin[slot ^ 1]);
        stage2_bookkeeping(c, sgs, ti, tm.nseg, slot, step, true, dt, tn, p.t_stop, log);
    }
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

}  // namespace vsw
