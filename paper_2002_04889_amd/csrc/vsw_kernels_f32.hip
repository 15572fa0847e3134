// Mixed-precision (FP32) variant of the fused stage kernel.
//
// Same scheme as the FP64 kernel (Sections 2.2-2.5), evaluated with FP32
// state and FP32 arithmetic wherever the quantities are small:
//   FP32: the prognostic free surface eta and momentum (Hu, Hv) in memory,
//         the least-squares gradients and Barth-Jespersen limiter, face
//         values of eta, Hu, Hv, face velocities, wave speeds, the mass and
//         tangential-momentum fluxes.
//   FP64: depths (H = eta + h with h ~ 4000 m cannot be held to 1e-4 m in
//         FP32), the hydrostatic reconstruction h* = min(h_L, h_R),
//         H* = max(0, eta + h*), the normal-momentum flux that carries
//         g H*^2 / 2, the hydrostatic and centred bed-source terms, the
//         accumulation of each cell's residual, the stage update and the CFL
//         reduction.
// At rest (eta = 0, u = 0) every FP32 quantity is exactly zero, so the lake
// at rest is kept to FP64 round-off as in the FP64 kernel.  A cell set dry
// by the post-stage fix stores eta = -h rounded upward, so its depth
// eta + h is never negative.
#include "vsw_common.hpp"
#include "vsw_faces.hpp"
#include "vsw_kernels_f32.hpp"

namespace vsw {

namespace {

struct ReconF {
    float fe[3], fu[3], fv[3];   // face eta, Hu, Hv
    double fh[3], fH[3];         // face bed depth and total depth
    double Hk, hk;
    bool second;
};

__device__ __forceinline__ float fminf_(float a, float b) { return (b < a) ? b : a; }
__device__ __forceinline__ float fmaxf_(float a, float b) { return (b > a) ? b : a; }

// pick3 of the FP64 kernel for FP32 values.
__device__ __forceinline__ float pick3f(int j, float a, float b, float c) {
    asm volatile("" : "+v"(a), "+v"(b), "+v"(c));
    return (j == 0) ? a : (j == 1) ? b : c;
}

// Reciprocal of a positive normal double to about one ulp: the hardware
// estimate and two Newton steps e = 1 - b r, r = r + r e with fused
// multiply-adds (quadratic convergence from the estimate).
__device__ __forceinline__ double recip_f64(double b) {
    double r = __builtin_amdgcn_rcp(b);
    double e = __builtin_fma(-b, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-b, r, 1.0);
    return __builtin_fma(r, e, r);
}

// FP32 reconstruction of cell k.  Geometry from callbacks as in recon_with:
// wall_n(j, nx, ny) in FP64 (rounded here), geo(w, d) as FP32 values.
// recon_from_f32 takes the records already loaded: ck, hk of the cell,
// cnb[j], hnb[j] of the neighbour across face j (not read on a wall).
template <class WallN, class Geo>
__device__ __forceinline__ void recon_from_f32(const CellF& ck, double hk, const CellF cnb[3],
                                               const double hnb[3], const uint32_t sl[3],
                                               double thr, WallN wall_n, Geo geo, ReconF& r,
                                               int sel = -1) {
    const float ek = ck.eta, uk = ck.hu, vk = ck.hv;
    const double Hk = double(ek) + hk;
    float qe[3], qu[3], qv[3], dh[3];
    bool cand = (Hk >= thr);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const uint32_t s = sl[j];
        if (s != kWallSlot) {
            const CellF& cn = cnb[j];
            const double hn = hnb[j];
            const double Hn = double(cn.eta) + hn;
            qe[j] = cn.eta;
            qu[j] = cn.hu;
            qv[j] = cn.hv;
            dh[j] = float(hn - hk);
            if (!(Hn >= thr)) cand = false;
        } else {
            // wall ghost: same depth and surface, mirrored momentum
            double nxd, nyd;
            wall_n(j, nxd, nyd);
            const float nx = float(nxd), ny = float(nyd);
            const float mn = uk * nx + vk * ny;
            qe[j] = ek;
            qu[j] = uk - (2.0f * mn) * nx;
            qv[j] = vk - (2.0f * mn) * ny;
            dh[j] = 0.0f;
        }
    }
    r.Hk = Hk;
    r.hk = hk;
    if (cand) {
        float gw[6], gd[6];
        geo(gw, gd);
        const float wx0 = gw[0], wx1 = gw[2], wx2 = gw[4];
        const float wy0 = gw[1], wy1 = gw[3], wy2 = gw[5];
        const float dxs[3] = {gd[0], gd[2], gd[4]};
        const float dys[3] = {gd[1], gd[3], gd[5]};
        auto project = [&](const float* qs, float q0, float* pj) {
            const float d0 = qs[0] - q0, d1 = qs[1] - q0, d2 = qs[2] - q0;
            const float gx = wx0 * d0 + wx1 * d1 + wx2 * d2;
            const float gy = wy0 * d0 + wy1 * d1 + wy2 * d2;
#pragma unroll
            for (int j = 0; j < 3; ++j) pj[j] = gx * dxs[j] + gy * dys[j];
        };
        float pe[3], pu[3], pv[3], ph[3];
        project(qe, ek, pe);
        project(qu, uk, pu);
        project(qv, vk, pv);
        project(dh, 0.0f, ph);
        // Barth-Jespersen, as in the FP64 kernel, with the two ratios taken
        // by the hardware reciprocal (1 ulp) and capped at one
        auto limiter = [](float q0, const float* qs, const float* pj) -> float {
            float qmax = q0, qmin = q0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                qmax = fmaxf_(qmax, qs[j]);
                qmin = fminf_(qmin, qs[j]);
            }
            const float up = qmax - q0, dn = qmin - q0;
            float dpos_max = 0.0f, dneg_min = 0.0f;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                dpos_max = fmaxf_(dpos_max, pj[j]);
                dneg_min = fminf_(dneg_min, pj[j]);
            }
            float a = 1.0f;
            if (dpos_max > 0.0f && up < dpos_max)
                a = fminf_(1.0f, up * __builtin_amdgcn_rcpf(dpos_max));
            if (dneg_min < 0.0f && dn > dneg_min)
                a = fminf_(a, dn * __builtin_amdgcn_rcpf(dneg_min));
            return a;
        };
        const float ae = limiter(ek, qe, pe);
        const float au = limiter(uk, qu, pu);
        const float av = limiter(vk, qv, pv);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            r.fe[j] = ek + ae * pe[j];
            r.fh[j] = hk + double(ph[j]);
            r.fH[j] = double(r.fe[j]) + r.fh[j];
            if (r.fH[j] < thr) cand = false;
        }
        if (sel < 0) {
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                r.fu[j] = uk + au * pu[j];
                r.fv[j] = vk + av * pv[j];
            }
        } else {
            // one face in slot 0 (see recon_from)
            r.fu[0] = uk + au * pick3f(sel, pu[0], pu[1], pu[2]);
            r.fv[0] = vk + av * pick3f(sel, pv[0], pv[1], pv[2]);
            r.fe[0] = pick3f(sel, r.fe[0], r.fe[1], r.fe[2]);
            r.fh[0] = pick3(sel, r.fh[0], r.fh[1], r.fh[2]);
            r.fH[0] = pick3(sel, r.fH[0], r.fH[1], r.fH[2]);
        }
    }
    if (!cand) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            r.fe[j] = ek; r.fu[j] = uk; r.fv[j] = vk; r.fh[j] = hk; r.fH[j] = Hk;
        }
    }
    r.second = cand;
}

template <class WallN, class Geo>
__device__ __forceinline__ void recon_with_f32(const CellF* __restrict__ W,
                                               const double* __restrict__ hc, int64_t k,
                                               const uint32_t sl[3], double thr, WallN wall_n,
                                               Geo geo, ReconF& r) {
    const CellF ck = W[k];
    const double hk = hc[k];
    CellF cn[3];
    double hn[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int64_t n = (sl[j] != kWallSlot) ? int64_t(sl[j] >> 3) : k;
        cn[j] = W[n];
        hn[j] = hc[n];
    }
    recon_from_f32(ck, hk, cn, hn, sl, thr, wall_n, geo, r);
}

__device__ __forceinline__ void recon_core_f32(const DevMesh& m, const CellF* __restrict__ W,
                                               int64_t k, double thr, ReconF& r) {
    const Nbr4 nb = m.nbr[k];
    const uint32_t sl[3] = {nb.s0, nb.s1, nb.s2};
    recon_with_f32(
        W, m.hcell, k, sl, thr,
        [&](int j, double& nx, double& ny) {
            nx = gf(m, 0, j, k);
            ny = gf(m, 1, j, k);
        },
        [&](float* gw, float* gd) {
            const RGeomF rg = m.rgeomf[k];
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                gw[q] = rg.w[q];
                gd[q] = rg.d[q];
            }
        },
        r);
}

__device__ __forceinline__ FaceF recon_face_f32(const ReconF& r, int j, double thr) {
    FaceF f;
    f.eta = r.fe[j];
    f.h = r.fh[j];
    f.H = r.fH[j];
    if (r.fH[j] >= thr) {
        // hardware reciprocal (1 ulp; this path is held to a tolerance):
        // the face depth is at least H_thr here
        const float rH = __builtin_amdgcn_rcpf(float(r.fH[j]));
        f.u = r.fu[j] * rH;
        f.v = r.fv[j] * rH;
    } else {
        f.u = 0.0f;
        f.v = 0.0f;
    }
    return f;
}

// recon_face_f32(r, j) for a face index j known only at run time: the face
// values are selected first (among registers, see pick3), then one face
// state is formed.
__device__ __forceinline__ FaceF recon_face_sel_f32(const ReconF& r, int j, double thr) {
    ReconF s;
    s.fe[0] = pick3f(j, r.fe[0], r.fe[1], r.fe[2]);
    s.fu[0] = pick3f(j, r.fu[0], r.fu[1], r.fu[2]);
    s.fv[0] = pick3f(j, r.fv[0], r.fv[1], r.fv[2]);
    s.fh[0] = pick3(j, r.fh[0], r.fh[1], r.fh[2]);
    s.fH[0] = pick3(j, r.fH[0], r.fH[1], r.fH[2]);
    return recon_face_f32(s, 0, thr);
}

// HLL flux in the face frame (Section 2.2) with FP64 depths HL, HR: the
// mass and tangential fluxes in FP32, the normal-momentum flux (which holds
// g H^2 / 2) in FP64.
__device__ __forceinline__ void hll_face_f32(double g, double hg, double HL, float unL, float utL,
                                             double HR, float unR, float utR, float& f0,
                                             double& f1, float& f2) {
    if (HL == 0.0 && HR == 0.0) {
        f0 = 0.0f; f1 = 0.0; f2 = 0.0f;
        return;
    }
    // hardware square root (1 ulp) of non-negative arguments
    const float cL = __builtin_amdgcn_sqrtf(float(g * HL)), cR = __builtin_amdgcn_sqrtf(float(g * HR));
    float sL, sR;
    if (HL == 0.0) {
        sL = unR - 2.0f * cR;
        sR = unR + cR;
    } else if (HR == 0.0) {
        sL = unL - cL;
        sR = unL + 2.0f * cL;
    } else {
        const float us = 0.5f * (unL + unR) + (cL - cR);
        const float cs = 0.5f * (cL + cR) - 0.25f * (unR - unL);
        sL = fminf_(unL - cL, us - cs);
        sR = fmaxf_(us + cs, unR + cR);
    }
    const float HLf = float(HL), HRf = float(HR);
    const float qL = HLf * unL, qR = HRf * unR;
    const float fL0 = qL, fL2 = qL * utL;
    const float fR0 = qR, fR2 = qR * utR;
    const double fL1 = double(qL * unL) + hg * (HL * HL);
    const double fR1 = double(qR * unR) + hg * (HR * HR);
    if (sL >= 0.0f) {
        f0 = fL0; f1 = fL1; f2 = fL2;
    } else if (sR < 0.0f) {
        f0 = fR0; f1 = fR1; f2 = fR2;
    } else {
        // The speeds are FP32; the denominator is their exact difference in
        // FP64, so F* of a uniform state returns that state's flux (an FP32
        // rounded sR - sL would bias the g H^2 / 2 part, ~1e8, by ~1e-7
        // relative on every face).  Mass and normal-momentum star fluxes are
        // formed in FP64 from the FP32 terms; the tangential one in FP32.
        // One reciprocal for the three components (this path is held to a
        // tolerance, not to the FP64 path's bits); den > 0 here.
        const double dR = double(sR), dL = double(sL), den = dR - dL, sLR = dL * dR;
        const double rden = recip_f64(den);
        f0 = float(((dR * double(fL0) - dL * double(fR0)) + sLR * (HR - HL)) * rden);
        f1 = ((dR * fL1 - dL * fR1) + sLR * (double(qR) - double(qL))) * rden;
        f2 = ((sR * fL2 - sL * fR2) + float(sLR) * (HRf * utR - HLf * utL)) * float(rden);
    }
}

// One face seen from a cell, canonical orientation, no divergent branches
// (see face_term of the FP64 kernel).  Returns l (phi + (0, p n)) in FP64.
__device__ __forceinline__ bool face_term_f32(double g, double hg, const FaceF& own,
                                              const FaceF& other, bool wall, bool own_left,
                                              double nx_out, double ny_out, double l, double t[3]) {
    const bool left = wall || own_left;
    const float eL = left ? own.eta : other.eta, eR = left ? other.eta : own.eta;
    const double hL = left ? own.h : other.h, hR = left ? other.h : own.h;
    const double HL = left ? own.H : other.H, HR = left ? other.H : own.H;
    const float uL = left ? own.u : other.u, uR = left ? other.u : own.u;
    const float vL = left ? own.v : other.v, vR = left ? other.v : own.v;
    const double nx = left ? nx_out : -nx_out, ny = left ? ny_out : -ny_out;
    const float nxf = float(nx), nyf = float(ny);
    const float unL = uL * nxf + vL * nyf, utL = vL * nxf - uL * nyf;
    float unR = uR * nxf + vR * nyf;
    const float utR = vR * nxf - uR * nyf;
    const double hs = dmin(hL, hR);
    const double HsL = dpos(double(eL) + hs), HsR = dpos(double(eR) + hs);
    if (wall) unR = -unL;
    float f0, f2;
    double f1;
    hll_face_f32(g, hg, HsL, unL, utL, HsR, unR, utR, f0, f1, f2);
    const double pc = left ? hg * (HL * HL - HsL * HsL) : hg * (HR * HR - HsR * HsR);
    const double phi1 = f1 * nx - double(f2) * ny;
    const double phi2 = f1 * ny + double(f2) * nx;
    t[0] = l * double(f0);
    t[1] = l * (phi1 + pc * nx);
    t[2] = l * (phi2 + pc * ny);
    return left;
}

// A face evaluated once for both of its cells, canonical orientation (the
// numbers face_term_f32 gives each side).  On a wall R is L itself.
__device__ __forceinline__ void face_pair_f32(double g, double hg, const FaceF& L, const FaceF& R,
                                              bool wall, double nx, double ny, double l,
                                              double tL[3], double tR[3]) {
    const float nxf = float(nx), nyf = float(ny);
    const float unL = L.u * nxf + L.v * nyf, utL = L.v * nxf - L.u * nyf;
    float unR = R.u * nxf + R.v * nyf;
    const float utR = R.v * nxf - R.u * nyf;
    const double hs = dmin(L.h, R.h);
    const double HsL = dpos(double(L.eta) + hs), HsR = dpos(double(R.eta) + hs);
    if (wall) unR = -unL;
    float f0, f2;
    double f1;
    hll_face_f32(g, hg, HsL, unL, utL, HsR, unR, utR, f0, f1, f2);
    const double pcL = hg * (L.H * L.H - HsL * HsL);
    const double pcR = hg * (R.H * R.H - HsR * HsR);
    const double phi1 = f1 * nx - double(f2) * ny;
    const double phi2 = f1 * ny + double(f2) * nx;
    tL[0] = l * double(f0);
    tL[1] = l * (phi1 + pcL * nx);
    tL[2] = l * (phi2 + pcL * ny);
    tR[0] = tL[0];
    tR[1] = l * (phi1 + pcR * nx);
    tR[2] = l * (phi2 + pcR * ny);
}

// FP32 reconstruction of a cell from its loaded records, vertices (geometry
// in FP64 as the host computes it, rounded to FP32 where the FP32 terms use
// it) and FP32 least-squares weights.
__device__ __forceinline__ void recon_tri_f32(const CellF& ck, double hk, const CellF cn[3],
                                              const double hn[3], const TopoD& tp,
                                              const double x[3], const double y[3],
                                              const LsqWF& w, double thr, ReconF& r,
                                              int sel = -1) {
    const uint32_t sl[3] = {tp.n0, tp.n1, tp.n2};
    recon_from_f32(
        ck, hk, cn, hn, sl, thr,
        [&](int j, double& nx, double& ny) {
            const int j1 = (j == 2) ? 0 : j + 1;
            const double ex = x[j1] - x[j], ey = y[j1] - y[j];
            const double l = sqrt_n(ex * ex + ey * ey);
            const Rcp d = rcp_of(l);
            nx = quot(ey, d);
            ny = quot(-ex, d);
        },
        [&](float* gw, float* gd) {
            const Rcp d3 = rcp_three();
            const double cx = quot((x[0] + x[1]) + x[2], d3);
            const double cy = quot((y[0] + y[1]) + y[2], d3);
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int j1 = (j == 2) ? 0 : j + 1;
                gw[2 * j] = w.w[2 * j];
                gw[2 * j + 1] = w.w[2 * j + 1];
                gd[2 * j] = float((x[j] + x[j1]) * 0.5 - cx);
                gd[2 * j + 1] = float((y[j] + y[j1]) * 0.5 - cy);
            }
        },
        r, sel);
}

// The records recon_tri_f32 reads for cell k: state, still-water depth,
// neighbours (k itself across a wall, not used), vertices.
struct CellInF {
    CellF ck;
    double hk;
    CellF cn[3];
    double hn[3];
    double x[3], y[3];
};

__device__ __forceinline__ void load_cell_f32(const FaceMesh& m, const CellF* __restrict__ W,
                                              const double* __restrict__ hc, const TopoD& tp,
                                              int64_t k, CellInF& in) {
    const uint32_t sl[3] = {tp.n0, tp.n1, tp.n2};
    in.ck = W[k];
    in.hk = hc[k];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int64_t n = (sl[j] != kWallSlot) ? int64_t(sl[j] >> 3) : k;
        in.cn[j] = W[n];
        in.hn[j] = hc[n];
    }
    const double2 p0 = m.vxy[tp.v0], p1 = m.vxy[tp.v1], p2 = m.vxy[tp.v2];
    in.x[0] = p0.x; in.x[1] = p1.x; in.x[2] = p2.x;
    in.y[0] = p0.y; in.y[1] = p1.y; in.y[2] = p2.y;
}

// Store a stage result: eta rounded to nearest, or, for a cell set dry,
// eta = -h rounded upward so that eta + h >= 0.
__device__ __forceinline__ CellF store_state(double h, double eta, double hu, double hv, bool dry) {
    CellF o;
    o.eta = dry ? __double2float_ru(-h) : float(eta);
    if (double(o.eta) + h < 0.0) o.eta = __double2float_ru(dry ? -h : eta);
    o.hu = float(hu);
    o.hv = float(hv);
    return o;
}

__device__ __forceinline__ double cfl_ratio_f32(const CellF& q, double h, double area,
                                                double perim, double g, double thr) {
    const double H = double(q.eta) + h;
    return cfl_ratio(H, double(q.hu), double(q.hv), area, perim, g, thr);
}

__device__ __forceinline__ void lds_store_face_f32(double* ld, float* lf, int stride, int slot,
                                                   const FaceF& f) {
    ld[0 * stride + slot] = f.h;
    ld[1 * stride + slot] = f.H;
    lf[0 * stride + slot] = f.eta;
    lf[1 * stride + slot] = f.u;
    lf[2 * stride + slot] = f.v;
}

__device__ __forceinline__ FaceF lds_load_face_f32(const double* ld, const float* lf, int stride,
                                                   int slot) {
    FaceF f;
    f.h = ld[0 * stride + slot];
    f.H = ld[1 * stride + slot];
    f.eta = lf[0 * stride + slot];
    f.u = lf[1 * stride + slot];
    f.v = lf[2 * stride + slot];
    return f;
}

}  // namespace

__global__ __launch_bounds__(kBlock) void dt_init_f32_kernel(DevMesh m, TileMap tm,
                                                             const CellF* __restrict__ W,
                                                             double g, double thr, Seg* sg) {
    const TileInfo ti = tile_info(tm.tinfo[blockIdx.x]);
    const int64_t k = int64_t(blockIdx.x) * kTile + threadIdx.x;
    double r = __longlong_as_double(0x7FF0000000000000ll);
    if (int(threadIdx.x) < ti.cnt)
        r = cfl_ratio_f32(W[k], m.hcell[k], m.area[k], m.perim[k], g, thr);
    block_min_atomic(r, &sg[ti.seg].rmin[0]);
}

// Same three phases as the FP64 stage kernel; LDS holds per face slot the
// FP64 (h, H) and FP32 (eta, u, v) of the face state.  TAPE adds the
// outputs the discrete adjoint records (TapeF) and leaves the arithmetic as
// it is.
template <int STAGE, bool TAPE>
__device__ __forceinline__ void stage_f32_body(const DevMesh& m, const TileMap& tm,
                                               CellF* __restrict__ Wa, CellF* __restrict__ Wb,
                                               CellF* __restrict__ W1, const StepParams& p,
                                               Ctrl* c, Seg* sg, int slot, int step_arg,
                                               double* log, const TapeF& tp) {
    extern __shared__ double lds[];
    const int stride = 3 * kTile + tm.bmax;
    double* ld = lds;
    float* lf = reinterpret_cast<float*>(lds + 2 * stride);
    const int t = tm.xcd_order ? xcd_tile(int(blockIdx.x), tm.ntiles) : int(blockIdx.x);
    const TileInfo ti = tile_info(tm.tinfo[t]);
    Seg* sgs = sg + ti.seg;
    const int step = c->kbase + step_arg;
    CellF *W, *Wout;
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
    const CellF* __restrict__ Ws = (STAGE == 1) ? W : W1;
    const int64_t nc = m.nc;
    const int64_t c0 = int64_t(t) * kTile;
    const int cnt = ti.cnt;
    const int i = threadIdx.x;
    const int64_t k = c0 + i;

    bool second = false;
    if (i < cnt) {
        ReconF r;
        recon_core_f32(m, Ws, k, p.thr, r);
#pragma unroll
        for (int j = 0; j < 3; ++j)
            lds_store_face_f32(ld, lf, stride, j * kTile + i, recon_face_f32(r, j, p.thr));
        second = r.second;
    }
    const int b0 = tm.bstart[t], nb = tm.bstart[t + 1] - b0;
    for (int b = i; b < nb; b += kBlock) {
        const uint32_t item = tm.bitem[b0 + b];
        const int64_t n = int64_t(item >> 2);
        const int jn = int(item & 3u);
        ReconF r;
        recon_core_f32(m, Ws, n, p.thr, r);
        lds_store_face_f32(ld, lf, stride, 3 * kTile + b, recon_face_sel_f32(r, jn, p.thr));
    }
    __syncthreads();

    unsigned long long clamp = 0;
    double rr = __longlong_as_double(0x7FF0000000000000ll);
    bool bad = false;
    if (i < cnt) {
        double fH[3], fh[3], fnx[3], fny[3], fl[3];
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const uint16_t s = tm.nloc[j * nc + k];
            const bool wall = (s == kNlocWall16);
            const FaceF own = lds_load_face_f32(ld, lf, stride, j * kTile + i);
            const FaceF other =
                lds_load_face_f32(ld, lf, stride, wall ? j * kTile + i : int(s & 0x7FFFu));
            fnx[j] = gf(m, 0, j, k);
            fny[j] = gf(m, 1, j, k);
            fl[j] = gf(m, 2, j, k);
            fH[j] = own.H;
            fh[j] = own.h;
            double tt[3];
            const bool left = face_term_f32(p.g, p.hg, own, other, wall, (s & 0x8000u) != 0,
                                            fnx[j], fny[j], fl[j], tt);
            if (left) {
                a0 = a0 - tt[0]; a1 = a1 - tt[1]; a2 = a2 - tt[2];
            } else {
                a0 = a0 + tt[0]; a1 = a1 + tt[1]; a2 = a2 + tt[2];
            }
        }
        const double hk = m.hcell[k];
        if (second) {
            const CellF q = Ws[k];
            double c3[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) c3[j] = (fl[j] * ((double(q.eta) + hk) + fH[j])) * (fh[j] - hk);
            const double sx = c3[0] * fnx[0] + c3[1] * fnx[1] + c3[2] * fnx[2];
            const double sy = c3[0] * fny[0] + c3[1] * fny[1] + c3[2] * fny[2];
            a1 = a1 + p.hg * sx;
            a2 = a2 + p.hg * sy;
        }
        const double ar = m.area[k];
        const double rar = recip_f64(ar);
        const double R0 = a0 * rar, R1 = a1 * rar, R2 = a2 * rar;
        const CellF w = W[k];
        double e, u, v;
        if (STAGE == 1) {
            e = double(w.eta) + dt * R0;
            u = double(w.hu) + dt * R1;
            v = double(w.hv) + dt * R2;
        } else {
            const CellF w1 = W1[k];
            e = 0.5 * double(w.eta) + 0.5 * (double(w1.eta) + dt * R0);
            u = 0.5 * double(w.hu) + 0.5 * (double(w1.hu) + dt * R1);
            v = 0.5 * double(w.hv) + 0.5 * (double(w1.hv) + dt * R2);
        }
        const double Hn = e + hk;
        bool dry = false;
        uint8_t mk = 3;
        if (Hn < 0.0) { dry = true; clamp = 1; mk &= uint8_t(~1u); }
        if (Hn < p.thr) { u = 0.0; v = 0.0; mk &= uint8_t(~2u); }
        const CellF o = store_state(hk, e, u, v, dry);
        if (STAGE == 1) {
            W1[k] = o;
        } else {
            Wout[k] = o;
            bad = !isfinite(e) || !isfinite(u) || !isfinite(v);
            rr = cfl_ratio_f32(o, hk, ar, m.perim[k], p.g, p.thr);
        }
        if (TAPE) {
            // the state this stage reconstructed, in FP64 as the FP32 terms
            // of the stage see it (H = eta + h rounded once)
            const CellF q = Ws[k];
            tp.win[k] = Cell4{double(q.eta) + hk, double(q.hu), double(q.hv), hk};
            tp.R[3 * k] = R0;
            tp.R[3 * k + 1] = R1;
            tp.R[3 * k + 2] = R2;
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
__global__ __launch_bounds__(kBlock) void stage_f32_kernel(DevMesh m, TileMap tm,
                                                           CellF* __restrict__ Wa,
                                                           CellF* __restrict__ Wb,
                                                           CellF* __restrict__ W1, StepParams p,
                                                           Ctrl* c, Seg* sg, int slot,
                                                           int step_arg, double* log) {
    stage_f32_body<STAGE, false>(m, tm, Wa, Wb, W1, p, c, sg, slot, step_arg, log, TapeF{});
}

template <int STAGE>
__global__ __launch_bounds__(kBlock) void stage_f32_tape_kernel(DevMesh m, TileMap tm,
                                                                CellF* __restrict__ W,
                                                                CellF* __restrict__ Wout,
                                                                CellF* __restrict__ W1,
                                                                StepParams p, Ctrl* c, Seg* sg,
                                                                int slot, int step_arg,
                                                                double* log, TapeF tp) {
    stage_f32_body<STAGE, true>(m, tm, W, Wout, W1, p, c, sg, slot, step_arg, log, tp);
}

template __global__ void stage_f32_kernel<1>(DevMesh, TileMap, CellF*, CellF*, CellF*,
                                             StepParams, Ctrl*, Seg*, int, int, double*);
template __global__ void stage_f32_kernel<2>(DevMesh, TileMap, CellF*, CellF*, CellF*,
                                             StepParams, Ctrl*, Seg*, int, int, double*);
template __global__ void stage_f32_tape_kernel<1>(DevMesh, TileMap, CellF*, CellF*, CellF*,
                                                  StepParams, Ctrl*, Seg*, int, int, double*,
                                                  TapeF);
template __global__ void stage_f32_tape_kernel<2>(DevMesh, TileMap, CellF*, CellF*, CellF*,
                                                  StepParams, Ctrl*, Seg*, int, int, double*,
                                                  TapeF);

// Face-parallel FP32 stage kernel: the phases of faces_stage_kernel, the
// arithmetic of stage_f32_kernel.  LDS planes hold doubles (FP32 values are
// stored exactly as doubles).
// TAPE records what stage_f32_tape_kernel records (TapeF), with the same
// arithmetic.
template <int T, int STAGE, bool TAPE>
__device__ __forceinline__ void faces_stage_f32_body(const FaceMesh& m, const FaceTileMap& tm,
                                                     const double* __restrict__ hc,
                                                     CellF* __restrict__ Wa,
                                                     CellF* __restrict__ Wb,
                                                     CellF* __restrict__ W1, const StepParams& p,
                                                     Ctrl* c, Seg* sg, int slot, int step_arg,
                                                     double* log, const TapeF& tape) {
    extern __shared__ double lds[];
    const int S = 3 * T + tm.bmax;
    double* __restrict__ Le = lds;
    double* __restrict__ Lh = lds + S;
    double* __restrict__ LH = lds + 2 * S;
    double* __restrict__ Lu = lds + 3 * S;
    double* __restrict__ Lv = lds + 4 * S;
    double* __restrict__ CH = lds + 5 * S;
    double* __restrict__ Ch = CH + T;
    const int t = tm.xcd_order ? xcd_tile(int(blockIdx.x), tm.ntiles) : int(blockIdx.x);
    const TileInfo ti = tile_info(tm.tinfo[t]);
    Seg* sgs = sg + ti.seg;
    const int step = c->kbase + step_arg;
    CellF *W, *Wout;
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
    const CellF* __restrict__ Ws = (STAGE == 1) ? W : W1;
    const int64_t c0 = int64_t(t) * T;
    const int cnt = ti.cnt;
    const int i = threadIdx.x;
    const int64_t k = c0 + i;

    const bool own = i < cnt;
    const int b0 = tm.bstart[t], nb = tm.bstart[t + 1] - b0;
    const int f0 = tm.fstart[t], nf = tm.fstart[t + 1] - f0;
    // loads in dependency levels, as in faces_stage_kernel; the FP32 records
    // leave the registers to fetch the thread's first two face records with
    // the first level and their vertices after the cell's reconstruction
    const int64_t ko = own ? k : c0;
    const TopoD tp = m.topo[ko];
    const LsqWF lw = m.lsqf[ko];
    uint32_t hitem = 0;
    if (i < nb) hitem = tm.bitem[b0 + i];
    CellInF in;
    load_cell_f32(m, Ws, hc, tp, ko, in);
    TopoD htp{0u, 0u, 0u, 0u, 0u, 0u};
    if (i < nb) htp = m.topo[hitem >> 2];
    FaceItemD it0{0u, 0u, 0, 0}, it1{0u, 0u, 0, 0};
    if (i < nf) it0 = tm.items[f0 + i];
    if (i + T < nf) it1 = tm.items[f0 + i + T];

    double area = 1.0;
    bool second = false;
    if (own) {
        ReconF r;
        recon_tri_f32(in.ck, in.hk, in.cn, in.hn, tp, in.x, in.y, lw, p.thr, r);
        const double cr = (in.x[1] - in.x[0]) * (in.y[2] - in.y[0]) -
                          (in.x[2] - in.x[0]) * (in.y[1] - in.y[0]);
        area = 0.5 * cr;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const FaceF f = recon_face_f32(r, j, p.thr);
            const int sj = j * T + i;
            Le[sj] = double(f.eta);
            Lh[sj] = f.h;
            LH[sj] = f.H;
            Lu[sj] = double(f.u);
            Lv[sj] = double(f.v);
        }
        CH[i] = r.Hk;
        Ch[i] = r.hk;
        second = r.second;
    }
    double2 a0 = make_double2(0.0, 0.0), e0 = a0, a1 = a0, e1 = a0;
    if (i < nf) {
        a0 = m.vxy[it0.va];
        e0 = m.vxy[it0.vb];
    }
    if (i + T < nf) {
        a1 = m.vxy[it1.va];
        e1 = m.vxy[it1.vb];
    }
    for (int b = i; b < nb; b += T) {
        const bool pre = (b == i);
        const uint32_t item = pre ? hitem : tm.bitem[b0 + b];
        const int64_t n = int64_t(item >> 2);
        const int jn = int(item & 3u);
        const TopoD tq = pre ? htp : m.topo[n];
        const LsqWF lq = m.lsqf[n];
        CellInF iq;
        load_cell_f32(m, Ws, hc, tq, n, iq);
        ReconF r;
        recon_tri_f32(iq.ck, iq.hk, iq.cn, iq.hn, tq, iq.x, iq.y, lq, p.thr, r, jn);
        const FaceF f = recon_face_f32(r, 0, p.thr);
        const int sb = 3 * T + b;
        Le[sb] = double(f.eta);
        Lh[sb] = f.h;
        LH[sb] = f.H;
        Lu[sb] = double(f.u);
        Lv[sb] = double(f.v);
    }
    CellF wn{0.0f, 0.0f, 0.0f}, w1{0.0f, 0.0f, 0.0f};
    double hk = 0.0, per = 1.0;
    if (own) {
        wn = W[k];
        hk = hc[k];
        if (STAGE == 2) {
            w1 = W1[k];
            per = m.perim[k];
        }
    }
    auto fgeo = [](const double2& pa, const double2& pb, double g[3]) {
        const double ex = pb.x - pa.x, ey = pb.y - pa.y;
        const double l = sqrt_n(ex * ex + ey * ey);
        const Rcp d = rcp_of(l);
        g[0] = quot(ey, d);
        g[1] = quot(-ex, d);
        g[2] = l;
    };
    double g0[3] = {0.0, 0.0, 0.0}, g1[3] = {0.0, 0.0, 0.0};
    if (i < nf) fgeo(a0, e0, g0);
    if (i + T < nf) fgeo(a1, e1, g1);
    __syncthreads();

    for (int q = i; q < nf; q += T) {
        FaceItemD it;
        double fg[3];
        if (q == i) {
            it = it0;
            fg[0] = g0[0]; fg[1] = g0[1]; fg[2] = g0[2];
        } else if (q == i + T) {
            it = it1;
            fg[0] = g1[0]; fg[1] = g1[1]; fg[2] = g1[2];
        } else {
            it = tm.items[f0 + q];
            fgeo(m.vxy[it.va], m.vxy[it.vb], fg);
        }
        const int sl = it.sl;
        const bool wall = (it.sr == kFaceWall);
        const int sr = wall ? sl : int(it.sr);
        FaceF L, R;
        L.eta = float(Le[sl]); L.h = Lh[sl]; L.H = LH[sl]; L.u = float(Lu[sl]); L.v = float(Lv[sl]);
        R.eta = float(Le[sr]); R.h = Lh[sr]; R.H = LH[sr]; R.u = float(Lu[sr]); R.v = float(Lv[sr]);
        const double nx = fg[0], ny = fg[1], l = fg[2];
        double tL[3], tR[3];
        face_pair_f32(p.g, p.hg, L, R, wall, nx, ny, l, tL, tR);
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
        const double rar = recip_f64(area);
        const double R0 = s0 * rar, R1 = s1 * rar, R2 = s2 * rar;
        const CellF w = wn;
        double e, u, v;
        if (STAGE == 1) {
            e = double(w.eta) + dt * R0;
            u = double(w.hu) + dt * R1;
            v = double(w.hv) + dt * R2;
        } else {
            e = 0.5 * double(w.eta) + 0.5 * (double(w1.eta) + dt * R0);
            u = 0.5 * double(w.hu) + 0.5 * (double(w1.hu) + dt * R1);
            v = 0.5 * double(w.hv) + 0.5 * (double(w1.hv) + dt * R2);
        }
        const double Hn = e + hk;
        bool dry = false;
        uint8_t mk = 3;
        if (Hn < 0.0) { dry = true; clamp = 1; mk &= uint8_t(~1u); }
        if (Hn < p.thr) { u = 0.0; v = 0.0; mk &= uint8_t(~2u); }
        const CellF o = store_state(hk, e, u, v, dry);
        if (STAGE == 1) {
            W1[k] = o;
        } else {
            Wout[k] = o;
            bad = !isfinite(e) || !isfinite(u) || !isfinite(v);
            rr = cfl_ratio_f32(o, hk, area, per, p.g, p.thr);
        }
        if (TAPE) {
            // the state this stage reconstructed, in FP64 as the FP32 terms
            // of the stage see it (H = eta + h rounded once)
            const CellF q = Ws[k];
            tape.win[k] = Cell4{double(q.eta) + hk, double(q.hu), double(q.hv), hk};
            tape.R[3 * k] = R0;
            tape.R[3 * k + 1] = R1;
            tape.R[3 * k + 2] = R2;
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
__global__ __launch_bounds__(T) void faces_stage_f32_kernel(FaceMesh m, FaceTileMap tm,
                                                            const double* __restrict__ hc,
                                                            CellF* __restrict__ Wa,
                                                            CellF* __restrict__ Wb,
                                                            CellF* __restrict__ W1, StepParams p,
                                                            Ctrl* c, Seg* sg, int slot,
                                                            int step_arg, double* log) {
    faces_stage_f32_body<T, STAGE, false>(m, tm, hc, Wa, Wb, W1, p, c, sg, slot, step_arg, log,
                                          TapeF{});
}

// faces_stage_f32_kernel with a tape: reads w^n from W and writes w^{n+1}
// to Wout (control par and step index 0).
template <int T, int STAGE>
__global__ __launch_bounds__(T) void faces_tape_f32_kernel(FaceMesh m, FaceTileMap tm,
                                                           const double* __restrict__ hc,
                                                           CellF* __restrict__ W,
                                                           CellF* __restrict__ Wout,
                                                           CellF* __restrict__ W1, StepParams p,
                                                           Ctrl* c, Seg* sg, int slot,
                                                           int step_arg, double* log, TapeF tp) {
    faces_stage_f32_body<T, STAGE, true>(m, tm, hc, W, Wout, W1, p, c, sg, slot, step_arg, log, tp);
}

template <int T>
__global__ __launch_bounds__(T) void faces_dt_init_f32_kernel(FaceMesh m, FaceTileMap tm,
                                                              const CellF* __restrict__ W,
                                                              const double* __restrict__ hc,
                                                              const double* __restrict__ area,
                                                              double g, double thr, Seg* sg) {
    const TileInfo ti = tile_info(tm.tinfo[blockIdx.x]);
    const int64_t k = int64_t(blockIdx.x) * T + threadIdx.x;
    double r = __longlong_as_double(0x7FF0000000000000ll);
    if (int(threadIdx.x) < ti.cnt) r = cfl_ratio_f32(W[k], hc[k], area[k], m.perim[k], g, thr);
    block_min_atomic<T>(r, &sg[ti.seg].rmin[0]);
}

#define VSW_FACES_F32_INSTANCES(T)                                                              \
    template __global__ void faces_stage_f32_kernel<T, 1>(FaceMesh, FaceTileMap, const double*, \
                                                          CellF*, CellF*, CellF*, StepParams,   \
                                                          Ctrl*, Seg*, int, int, double*);      \
    template __global__ void faces_stage_f32_kernel<T, 2>(FaceMesh, FaceTileMap, const double*, \
                                                          CellF*, CellF*, CellF*, StepParams,   \
                                                          Ctrl*, Seg*, int, int, double*);      \
    template __global__ void faces_dt_init_f32_kernel<T>(FaceMesh, FaceTileMap, const CellF*,   \
                                                         const double*, const double*, double,  \
                                                         double, Seg*);
VSW_FACES_F32_INSTANCES(128)
VSW_FACES_F32_INSTANCES(256)
VSW_FACES_F32_INSTANCES(512)
#undef VSW_FACES_F32_INSTANCES

// the adjoint replays tiles of 256 cells
template __global__ void faces_tape_f32_kernel<256, 1>(FaceMesh, FaceTileMap, const double*,
                                                       CellF*, CellF*, CellF*, StepParams, Ctrl*,
                                                       Seg*, int, int, double*, TapeF);
template __global__ void faces_tape_f32_kernel<256, 2>(FaceMesh, FaceTileMap, const double*,
                                                       CellF*, CellF*, CellF*, StepParams, Ctrl*,
                                                       Seg*, int, int, double*, TapeF);

// Free surface at the gauge cells after step `step` (see gauge_kernel).
__global__ void gauge_f32_kernel(const CellF* __restrict__ Wa, const CellF* __restrict__ Wb,
                                 const double* __restrict__ h, const int64_t* __restrict__ cells,
                                 int ng,
                                 const int32_t* __restrict__ gseg, const Seg* sg,
                                 const Ctrl* c, int step_arg, double* __restrict__ log) {
    const int gi = int(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gi >= ng) return;
    const int step = c->kbase + step_arg;
    const CellF *Win, *W;
    step_buffers(c, step, Wa, Wb, Win, W);
    const int64_t k = cells[gi];
    if (sg[gseg[gi]].steps_done <= step) return;
    const CellF q = W[k];
    const double hk = h[k];
    log[int64_t(step) * ng + gi] = (double(q.eta) + hk) - hk;
}

// Caller-order FP64 (H, HU, HV) into FP32 state records: eta = H - h rounded
// to nearest (upward for a dry cell so that eta + h >= 0).
__global__ void pack_state_f32_kernel(int64_t n, const int64_t* __restrict__ perm,
                                      const double* __restrict__ H, const double* __restrict__ HU,
                                      const double* __restrict__ HV, const double* __restrict__ h,
                                      CellF* __restrict__ W, CellF* __restrict__ W1) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t k = perm[i];
    if (k < 0) return;
    const CellF q = store_state(h[i], H[k] - h[i], HU[k], HV[k], !(H[k] > 0.0));
    W[i] = q;
    W1[i] = q;
}

// FP32 state records into caller-order FP64 arrays, H = eta + h.
__global__ void unpack_state_f32_kernel(int64_t n, const int64_t* __restrict__ perm,
                                        const CellF* __restrict__ W,
                                        const double* __restrict__ h, double* __restrict__ H,
                                        double* __restrict__ HU, double* __restrict__ HV) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t k = perm[i];
    if (k < 0) return;
    const CellF q = W[i];
    if (H) H[k] = double(q.eta) + h[i];
    if (HU) HU[k] = double(q.hu);
    if (HV) HV[k] = double(q.hv);
}

}  // namespace vsw
