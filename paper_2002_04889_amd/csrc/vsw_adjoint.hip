// Discrete adjoint of the SSP-RK(2,2) step of the shallow-water scheme
// (Sections 2.2-2.5), FP64, for gradients of a loss of the state with
// respect to the initial state and the bed depth h.
//
// Reverse of one step w^{n+1} = fix(w/2 + (w1 + dt R(w1))/2),
// w1 = fix(w + dt R(w)), dt = CFL min_K ratio_K(w):
//   lt2 = mask2 lam;  lam_w = lt2/2;  lam_w1 = lt2/2 + J_R(w1)^T (dt/2 lt2)
//   lt1 = mask1 lam_w1;  lam_w += lt1 + J_R(w)^T (dt lt1)
//   lam_dt = sum lt2/2 . R(w1) + sum lt1 . R(w);  lam_w[K*] += lam_dt CFL d ratio_K*/d w
// with the masks the post-stage fix applied (a clamped depth or a zeroed
// momentum passes no derivative) and K* the cell that set the CFL minimum.
// The bed depth h enters R through eta = H - h, its reconstruction, the
// hydrostatic reconstruction and the bed source; its adjoint accumulates
// over all steps.
//
// The stages' residuals, fix masks and intermediate states are recorded by
// the stage kernels while they replay a checkpoint segment (Tape).  J_R^T mu
// is taken in two passes, each cell-centric and free of atomics (the
// contributions between cells of one tile handed over through LDS in the
// first, those between tiles through memory to the second):
//   vjp     per tile, the face states reconstructed into LDS as in the
//           forward; per cell, the adjoint of its face states from the face
//           terms of both cells that share each face (the forward evaluates
//           each face once from each side, in canonical orientation) and
//           from the bed source, then the reverse of the cell's
//           reconstruction (least-squares gradient, Barth-Jespersen limiter
//           with its branch recomputed, eq. (3), face velocity), giving the
//           cell's own adjoint and one contribution per stencil member;
//           a member in the same tile adds it to its own adjoint, in face
//           order, after a barrier;
//   gather  each cell adds the contributions its face neighbours in other
//           tiles made to it, in face order.
// Branches (wet/dry, upwind side, limiter case, min/max) are taken as the
// forward takes them; the derivative is that of the taken branch.  Values
// that decide a branch are formed bit for bit as the forward forms them;
// reciprocals that only scale a derivative are the refined hardware
// reciprocal (within an ulp of the quotient).
#include "vsw_adjoint.hpp"
#include "vsw_common.hpp"

namespace vsw {

namespace {

// Reverse of hll_face: adds the adjoint of (HL, unL, utL, HR, unR, utR)
// for the flux adjoint fb.
__device__ __forceinline__ void hll_face_rev(double g, double hg, double HL, double unL,
                                             double utL, double HR, double unR, double utR,
                                             const double fb[3], double& HLb, double& unLb,
                                             double& utLb, double& HRb, double& unRb,
                                             double& utRb) {
    if (HL == 0.0 && HR == 0.0) return;
    // the forward's wave speeds, bit for bit (its branches are taken again)
    const double xL = g * HL, xR = g * HR;
    double cL = sqrt_n(xL), cR = sqrt_n(xR);
    if (wave_any(!(xL >= 0x1p-767) || !(xR >= 0x1p-767))) {
        cL = sqrt(xL);
        cR = sqrt(xR);
    }
    double sL, sR, us = 0.0, cs = 0.0;
    bool selL = false, selR = false;  // sL = us - cs, sR = unR + cR chosen
    if (HL == 0.0) {
        sL = unR - 2.0 * cR;
        sR = unR + cR;
    } else if (HR == 0.0) {
        sL = unL - cL;
        sR = unL + 2.0 * cL;
    } else {
        us = 0.5 * (unL + unR) + (cL - cR);
        cs = 0.5 * (cL + cR) - 0.25 * (unR - unL);
        const double a = unL - cL, b = us - cs;
        selL = b < a;
        sL = selL ? b : a;
        const double c = us + cs, d = unR + cR;
        selR = d > c;
        sR = selR ? d : c;
    }
    const double qL = HL * unL, qR = HR * unR;
    const double fL[3] = {qL, qL * unL + hg * (HL * HL), qL * utL};
    const double fR[3] = {qR, qR * unR + hg * (HR * HR), qR * utR};
    double fLb[3] = {0.0, 0.0, 0.0}, fRb[3] = {0.0, 0.0, 0.0}, dUb[3] = {0.0, 0.0, 0.0};
    double sLb = 0.0, sRb = 0.0;
    if (sL >= 0.0) {
        fLb[0] = fb[0]; fLb[1] = fb[1]; fLb[2] = fb[2];
    } else if (sR < 0.0) {
        fRb[0] = fb[0]; fRb[1] = fb[1]; fRb[2] = fb[2];
    } else {
        const double den = sR - sL, sLR = sL * sR, rd = rcp_of(den).r;
        const double dU[3] = {HR - HL, qR - qL, HR * utR - HL * utL};
        double rdb = 0.0, sLRb = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            // f_c = N_c * rd
            const double N = (sR * fL[c] - sL * fR[c]) + sLR * dU[c];
            const double nb = fb[c] * rd;
            rdb += fb[c] * N;
            sRb += nb * fL[c];
            fLb[c] += nb * sR;
            sLb -= nb * fR[c];
            fRb[c] -= nb * sL;
            sLRb += nb * dU[c];
            dUb[c] += nb * sLR;
        }
        sLb += sLRb * sR;
        sRb += sLRb * sL;
        const double denb = -rdb * rd * rd;  // rd = 1 / den
        sRb += denb;
        sLb -= denb;
    }
    // jumps of the conserved variables
    HRb += dUb[0];
    HLb -= dUb[0];
    double qLb = -dUb[1], qRb = dUb[1];
    HRb += dUb[2] * utR;
    utRb += dUb[2] * HR;
    HLb -= dUb[2] * utL;
    utLb -= dUb[2] * HL;
    // physical fluxes
    qLb += fLb[0] + fLb[1] * unL + fLb[2] * utL;
    unLb += fLb[1] * qL;
    HLb += fLb[1] * (hg * 2.0 * HL);
    utLb += fLb[2] * qL;
    qRb += fRb[0] + fRb[1] * unR + fRb[2] * utR;
    unRb += fRb[1] * qR;
    HRb += fRb[1] * (hg * 2.0 * HR);
    utRb += fRb[2] * qR;
    HLb += qLb * unL;
    unLb += qLb * HL;
    HRb += qRb * unR;
    unRb += qRb * HR;
    // wave speeds
    double cLb = 0.0, cRb = 0.0;
    if (HL == 0.0) {
        unRb += sLb + sRb;
        cRb += -2.0 * sLb + sRb;
    } else if (HR == 0.0) {
        unLb += sLb + sRb;
        cLb += -sLb + 2.0 * sRb;
    } else {
        double usb = 0.0, csb = 0.0;
        if (selL) { usb += sLb; csb -= sLb; } else { unLb += sLb; cLb -= sLb; }
        if (selR) { unRb += sRb; cRb += sRb; } else { usb += sRb; csb += sRb; }
        unLb += 0.5 * usb;
        unRb += 0.5 * usb;
        cLb += usb;
        cRb -= usb;
        cLb += 0.5 * csb;
        cRb += 0.5 * csb;
        unRb -= 0.25 * csb;
        unLb += 0.25 * csb;
    }
    if (HL > 0.0) HLb += cLb * g * rcp_of(2.0 * cL).r;
    if (HR > 0.0) HRb += cRb * g * rcp_of(2.0 * cR).r;
}

__device__ __forceinline__ void face_add(Face& a, const double eta, double h, double H, double u,
                                         double v) {
    a.eta += eta; a.h += h; a.H += H; a.u += u; a.v += v;
}

// Reverse of the two terms of one face for the adjoint of this cell's face
// state: this cell's term (adjoint tb) and, on an interior face, the
// neighbour's term (adjoint tbn).  Both terms come from one flux in the
// face's canonical orientation (they differ in sign and in the side whose
// pressure correction they carry), so the flux is reversed once for the
// combined adjoint.  On a wall the ghost is the mirror of own, and its
// derivatives fold back into own.
__device__ __forceinline__ void face_pair_rev(double g, double hg, const Face& own,
                                              const Face& other, bool wall, bool own_left,
                                              double nx_out, double ny_out, double l,
                                              const double tb[3], const double tbn[3],
                                              Face& ownb) {
    const bool left = wall || own_left;
    const Face& L = left ? own : other;
    const Face& R = left ? other : own;
    const double nx = left ? nx_out : -nx_out, ny = left ? ny_out : -ny_out;
    const double unL = L.u * nx + L.v * ny, utL = L.v * nx - L.u * ny;
    double unR = R.u * nx + R.v * ny;
    const double utR = R.v * nx - R.u * ny;
    const bool hsR = R.h < L.h;  // hs = dmin(hL, hR) takes hR
    const double hs = hsR ? R.h : L.h;
    const double aL = L.eta + hs, aR = R.eta + hs;
    const double HsL = (aL > 0.0) ? aL : 0.0, HsR = (aR > 0.0) ? aR : 0.0;
    if (wall) unR = -unL;
    // a term is l (f0, phi1 + pc nx, phi2 + pc ny), phi the rotated flux f
    const double p0b = l * (tb[0] + tbn[0]), p1b = l * (tb[1] + tbn[1]),
                 p2b = l * (tb[2] + tbn[2]);
    const double pcob = l * (tb[1] * nx + tb[2] * ny);    // this cell's correction
    const double pcnb = l * (tbn[1] * nx + tbn[2] * ny);  // the neighbour's
    const double fb[3] = {p0b, p1b * nx + p2b * ny, -p1b * ny + p2b * nx};
    double HLb = 0.0, HRb = 0.0, HsLb = 0.0, HsRb = 0.0;
    if (left) {
        HLb += pcob * hg * 2.0 * L.H;
        HsLb -= pcob * hg * 2.0 * HsL;
        HsRb -= pcnb * hg * 2.0 * HsR;
    } else {
        HRb += pcob * hg * 2.0 * R.H;
        HsRb -= pcob * hg * 2.0 * HsR;
        HsLb -= pcnb * hg * 2.0 * HsL;
    }
    double unLb = 0.0, utLb = 0.0, unRb = 0.0, utRb = 0.0;
    hll_face_rev(g, hg, HsL, unL, utL, HsR, unR, utR, fb, HsLb, unLb, utLb, HsRb, unRb, utRb);
    if (wall) {
        unLb -= unRb;
        unRb = 0.0;
    }
    double eLb = 0.0, eRb = 0.0, hsb = 0.0;
    if (aL > 0.0) { eLb += HsLb; hsb += HsLb; }
    if (aR > 0.0) { eRb += HsRb; hsb += HsRb; }
    const double hLb = hsR ? 0.0 : hsb, hRb = hsR ? hsb : 0.0;
    const double uLb = unLb * nx - utLb * ny, vLb = unLb * ny + utLb * nx;
    const double uRb = unRb * nx - utRb * ny, vRb = unRb * ny + utRb * nx;
    if (left) face_add(ownb, eLb, hLb, HLb, uLb, vLb);
    if (!left || wall) face_add(ownb, eRb, hRb, HRb, uRb, vRb);
}

struct LimInfo {
    int br;       // 0: alpha = 1, 1: (max - q0) / max_j d_j, 2: (min - q0) / min_j d_j
    int iq;       // stencil member giving the max (br 1) or min (br 2); -1 = the cell
    int jd;       // face giving max_j d_j (br 1) or min_j d_j (br 2)
    double den;   // that d_j
};

// Barth-Jespersen factor as in recon_core, with the branch taken.
__device__ __forceinline__ double limiter_fwd(double q0, const double qs[3], const double pj[3],
                                              LimInfo& li) {
    double qmax = q0, qmin = q0;
    int imax = -1, imin = -1;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        if (qs[j] > qmax) { qmax = qs[j]; imax = j; }
        if (qs[j] < qmin) { qmin = qs[j]; imin = j; }
    }
    const double up = qmax - q0, dn = qmin - q0;
    double dpm = 0.0, dnm = 0.0;
    int jp = -1, jn = -1;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        if (pj[j] > dpm) { dpm = pj[j]; jp = j; }
        if (pj[j] < dnm) { dnm = pj[j]; jn = j; }
    }
    double a = 1.0;
    li.br = 0;
    if (dpm > 0.0 && up < dpm) {
        a = up / dpm;
        li.br = 1; li.iq = imax; li.jd = jp; li.den = dpm;
    }
    if (dnm < 0.0 && dn > dnm) {
        const double r = dn / dnm;
        if (r < a) {
            a = r;
            li.br = 2; li.iq = imin; li.jd = jn; li.den = dnm;
        }
    }
    return a;
}

__device__ __forceinline__ void limiter_rev(double a, double ab, const LimInfo& li, double& q0b,
                                            double qsb[3], double pjb[3]) {
    if (li.br == 0) return;
    const double rd = rcp_of(li.den).r;
    const double nb = ab * rd;              // adjoint of (q_ext - q0)
    pjb[li.jd] -= (ab * a) * rd;            // adjoint of the denominator
    q0b -= nb;
    if (li.iq < 0) q0b += nb; else qsb[li.iq] += nb;
}

}  // namespace

namespace {

// Block sum in a fixed order (wavefront butterflies, then the four waves);
// every thread of the block must call it.
__device__ __forceinline__ double block_sum(double v) {
    __shared__ double part[kBlock / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) part[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < kBlock / 64; ++i) s += part[i];
    return s;
}

}  // namespace

// ---------------------------------------------------------------- forward pieces

__global__ __launch_bounds__(kBlock) void adj_xin_kernel(TileMap tm, int64_t nc,
                                                         int32_t* __restrict__ xin) {
    const int t = int(blockIdx.x);
    const int b0 = tm.bstart[t], nb = tm.bstart[t + 1] - b0;
    for (int b = int(threadIdx.x); b < nb; b += kBlock) {
        const uint32_t item = tm.bitem[b0 + b];
        xin[int64_t(item & 3u) * nc + int64_t(item >> 2)] = b0 + b;
    }
}

__global__ __launch_bounds__(kBlock) void adj_rmin_kernel(DevMesh m, TileMap tm,
                                                          const Cell4* __restrict__ W, double g,
                                                          double thr, unsigned long long* rmin) {
    const TileInfo ti = tile_info(tm.tinfo[blockIdx.x]);
    const int64_t k = int64_t(blockIdx.x) * kTile + threadIdx.x;
    double r = __longlong_as_double(0x7FF0000000000000ll);
    if (int(threadIdx.x) < ti.cnt) {
        const Cell4 q = W[k];
        r = cfl_ratio(q.H, q.HU, q.HV, m.area[k], m.perim[k], g, thr);
    }
    block_min_atomic(r, rmin);
}

__global__ __launch_bounds__(kBlock) void adj_start_kernel(DevMesh m, TileMap tm,
                                                           const Adj4* __restrict__ lam,
                                                           const uint8_t* __restrict__ mask2,
                                                           const double* __restrict__ R1,
                                                           double dt, double* __restrict__ mua,
                                                           Adj4* __restrict__ lamn,
                                                           double* __restrict__ part) {
    const TileInfo ti = tile_info(tm.tinfo[blockIdx.x]);
    const int64_t k = int64_t(blockIdx.x) * kTile + threadIdx.x;
    double d = 0.0;
    if (int(threadIdx.x) < ti.cnt) {
        const uint8_t mk = mask2[k];
        const Adj4 l = lam[k];
        const double l0 = (mk & 1) ? l.H : 0.0, l1 = (mk & 2) ? l.HU : 0.0,
                     l2 = (mk & 2) ? l.HV : 0.0;
        const double ra = rcp_of(m.area[k]).r;
        mua[3 * k] = (0.5 * dt * l0) * ra;
        mua[3 * k + 1] = (0.5 * dt * l1) * ra;
        mua[3 * k + 2] = (0.5 * dt * l2) * ra;
        lamn[k] = Adj4{0.5 * l0, 0.5 * l1, 0.5 * l2, l.h};
        d = 0.5 * (l0 * R1[3 * k] + l1 * R1[3 * k + 1] + l2 * R1[3 * k + 2]);
    }
    const double s = block_sum(d);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// ---------------------------------------------------------------- J_R^T mu

// One workgroup per tile.  Phase 1 is the stage kernel's: the face states of
// the tile's cells and of its halo faces, reconstructed into LDS.  Phase 2,
// per cell k (no exchange between threads):
//  a. the adjoint of each of k's three face states from the two terms of
//     the face, k's own (weight mua_k) and its neighbour's (weight mua_n),
//     plus the bed source of a second-order cell;
//  b. the reverse of k's reconstruction, its branches recomputed: the
//     adjoint of k's own variables and one contribution per stencil member,
//     handed to the member through LDS (same tile) or AdjC (other tiles).
__global__ __launch_bounds__(kBlock) void adj_vjp_kernel(DevMesh m, TileMap tm,
                                                         const Cell4* __restrict__ W,
                                                         const double* __restrict__ mua,
                                                         double g, double hg, double thr,
                                                         AdjC c,
                                                         unsigned long long* argmin_reset) {
    extern __shared__ double lds[];
    const int stride = 3 * kTile + tm.bmax;
    const int t = int(blockIdx.x);
    const TileInfo ti = tile_info(tm.tinfo[t]);
    const int64_t nc = m.nc, c0 = int64_t(t) * kTile;
    const int i = threadIdx.x;
    const int64_t k = c0 + i;
    double sc[2], ownH[3];
    bool second;
    // clears the minimising-cell word the next gather fills (the previous
    // step's turn kernel, its last reader, has finished)
    if (argmin_reset && t == 0 && i == 0) *argmin_reset = ~0ull;
    // phase 1, mostly dependent gathers, at raised wave priority: a wave in
    // it issues its loads ahead of waves in the arithmetic of phase 2
    __builtin_amdgcn_s_setprio(2);
    tile_faces(m, tm, W, t, c0, ti.cnt, thr, hg, lds, stride, ownH, sc, second);
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();
    const bool own = i < ti.cnt;
    // the cell's own adjoint and its contribution to the stencil member
    // across each face (zero on a wall)
    double ownv[4] = {0.0, 0.0, 0.0, 0.0};
    double con[3][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
    uint32_t sl[3] = {kWallSlot, kWallSlot, kWallSlot};
    if (own) {
    // ---- a. face-state adjoints
    const double ab[3] = {mua[3 * k], mua[3 * k + 1], mua[3 * k + 2]};
    const Nbr4 nb = m.nbr[k];
    sl[0] = nb.s0;
    sl[1] = nb.s1;
    sl[2] = nb.s2;
    Face F[3];
    double fhs[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        F[j] = Face{0.0, 0.0, 0.0, 0.0, 0.0};
        const uint32_t s = sl[j];
        const bool wall = (s == kWallSlot);
        const bool own_left = wall || (s & 4u);
        const Face own = lds_load_face(lds, stride, j * kTile + i, ownH[j]);
        fhs[j] = own.h;
        const double nx = gf(m, 0, j, k), ny = gf(m, 1, j, k), l = gf(m, 2, j, k);
        // this cell's term enters its accumulator with - (left) or + (right),
        // the neighbour's with the opposite sign
        const double sg = own_left ? -1.0 : 1.0;
        const double tb[3] = {sg * ab[0], sg * ab[1], sg * ab[2]};
        if (wall) {
            const double zero[3] = {0.0, 0.0, 0.0};
            face_pair_rev(g, hg, own, own, true, true, nx, ny, l, tb, zero, F[j]);
        } else {
            const int64_t n = int64_t(s >> 3);
            // the neighbour's face depth enters only the neighbour's own
            // pressure correction, whose adjoint is not needed here
            const Face other = lds_load_face(
                lds, stride, int(tm.nloc[j * nc + k] & 0x7FFFu), 0.0);
            const double tbn[3] = {-sg * mua[3 * n], -sg * mua[3 * n + 1], -sg * mua[3 * n + 2]};
            face_pair_rev(g, hg, own, other, false, own_left, nx, ny, l, tb, tbn, F[j]);
        }
    }
    const Cell4 ck = W[k];
    double DH = 0.0, Dh = 0.0;
    if (second) {
        // bed source (g/2) sum_j l_j (H_K + H_Kj)(h_Kj - h_K) n_j added to the momentum rows
        const double sxb = hg * ab[1], syb = hg * ab[2];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double nx = gf(m, 0, j, k), ny = gf(m, 1, j, k), l = gf(m, 2, j, k);
            const double cb = sxb * nx + syb * ny;
            const double dHj = cb * (l * (fhs[j] - ck.h)), dhj = cb * (l * (ck.H + ownH[j]));
            F[j].H += dHj;
            F[j].h += dhj;
            DH += dHj;
            Dh -= dhj;
        }
    }

    // ---- b. reverse of the reconstruction (forward recomputed as in recon_core)
    const double Hk = ck.H, hk = ck.h, ek = Hk - hk, uk = ck.HU, vk = ck.HV;
    double qe[3], qu[3], qv[3], qh[3];
    bool cand = (Hk >= thr);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const uint32_t s = sl[j];
        if (s != kWallSlot) {
            const Cell4 cn = W[int64_t(s >> 3)];
            qe[j] = cn.H - cn.h;
            qu[j] = cn.HU;
            qv[j] = cn.HV;
            qh[j] = cn.h;
            if (!(cn.H >= thr)) cand = false;
        } else {
            const double nx = gf(m, 0, j, k), ny = gf(m, 1, j, k);
            const double mn = uk * nx + vk * ny;
            qe[j] = ek;
            qu[j] = uk - (2.0 * mn) * nx;
            qv[j] = vk - (2.0 * mn) * ny;
            qh[j] = hk;
        }
    }
    double pe[3], pu[3], pv[3], ph[3], fe[3], fu[3], fv[3], fH[3];
    double ae = 1.0, au = 1.0, av = 1.0;
    LimInfo le{0, -1, 0, 1.0}, lu{0, -1, 0, 1.0}, lv{0, -1, 0, 1.0};
    const RGeom rg = m.rgeom[k];
    const double wx[3] = {rg.w[0], rg.w[2], rg.w[4]}, wy[3] = {rg.w[1], rg.w[3], rg.w[5]};
    const double dxs[3] = {rg.d[0], rg.d[2], rg.d[4]}, dys[3] = {rg.d[1], rg.d[3], rg.d[5]};
    auto project = [&](const double* qs, double q0, double* pj) {
        const double d0 = qs[0] - q0, d1 = qs[1] - q0, d2 = qs[2] - q0;
        const double gx = wx[0] * d0 + wx[1] * d1 + wx[2] * d2;
        const double gy = wy[0] * d0 + wy[1] * d1 + wy[2] * d2;
#pragma unroll
        for (int j = 0; j < 3; ++j) pj[j] = gx * dxs[j] + gy * dys[j];
    };
    if (cand) {
        project(qe, ek, pe);
        project(qu, uk, pu);
        project(qv, vk, pv);
        project(qh, hk, ph);
        ae = limiter_fwd(ek, qe, pe, le);
        au = limiter_fwd(uk, qu, pu, lu);
        av = limiter_fwd(vk, qv, pv, lv);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            fe[j] = ek + ae * pe[j];
            fu[j] = uk + au * pu[j];
            fv[j] = vk + av * pv[j];
            fH[j] = fe[j] + (hk + ph[j]);
            if (fH[j] < thr) cand = false;
        }
    }
    if (!cand) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            fe[j] = ek; fu[j] = uk; fv[j] = vk; fH[j] = Hk;
        }
    }
    double feb[3], fub[3], fvb[3], fhb[3], fHb[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        feb[j] = F[j].eta;
        fhb[j] = F[j].h;
        fHb[j] = F[j].H;
        fub[j] = 0.0;
        fvb[j] = 0.0;
        if (fH[j] >= thr) {
            // u = fu * rH, v = fv * rH, rH = 1 / fH
            const double ub = F[j].u, vb = F[j].v;
            const double rH = rcp_of(fH[j]).r;
            fub[j] = ub * rH;
            fvb[j] = vb * rH;
            fHb[j] -= (ub * fu[j] + vb * fv[j]) * rH * rH;
        }
    }
    double Hkb = DH, hkb = Dh, ekb = 0.0, ukb = 0.0, vkb = 0.0;
    double qeb[3] = {0.0, 0.0, 0.0}, qub[3] = {0.0, 0.0, 0.0}, qvb[3] = {0.0, 0.0, 0.0},
           qhb[3] = {0.0, 0.0, 0.0};
    if (!cand) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            ekb += feb[j]; ukb += fub[j]; vkb += fvb[j]; hkb += fhb[j]; Hkb += fHb[j];
        }
    } else {
        double peb[3], pub[3], pvb[3], phb[3], aeb = 0.0, aub = 0.0, avb = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double e_b = feb[j] + fHb[j], h_b = fhb[j] + fHb[j];
            ekb += e_b;
            aeb += e_b * pe[j];
            peb[j] = e_b * ae;
            ukb += fub[j];
            aub += fub[j] * pu[j];
            pub[j] = fub[j] * au;
            vkb += fvb[j];
            avb += fvb[j] * pv[j];
            pvb[j] = fvb[j] * av;
            hkb += h_b;
            phb[j] = h_b;
        }
        limiter_rev(ae, aeb, le, ekb, qeb, peb);
        limiter_rev(au, aub, lu, ukb, qub, pub);
        limiter_rev(av, avb, lv, vkb, qvb, pvb);
        auto project_rev = [&](const double* pjb, double& q0b, double* qsb) {
            const double gxb = pjb[0] * dxs[0] + pjb[1] * dxs[1] + pjb[2] * dxs[2];
            const double gyb = pjb[0] * dys[0] + pjb[1] * dys[1] + pjb[2] * dys[2];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const double db = wx[q] * gxb + wy[q] * gyb;
                qsb[q] += db;
                q0b -= db;
            }
        };
        project_rev(peb, ekb, qeb);
        project_rev(pub, ukb, qub);
        project_rev(pvb, vkb, qvb);
        project_rev(phb, hkb, qhb);
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const uint32_t s = sl[j];
        if (s != kWallSlot) {
            con[j][0] = qeb[j];
            con[j][1] = qub[j];
            con[j][2] = qvb[j];
            con[j][3] = qhb[j] - qeb[j];
        } else {
            const double nx = gf(m, 0, j, k), ny = gf(m, 1, j, k);
            ekb += qeb[j];
            ukb += qub[j];
            vkb += qvb[j];
            const double mnb = -2.0 * (qub[j] * nx + qvb[j] * ny);
            ukb += mnb * nx;
            vkb += mnb * ny;
            hkb += qhb[j];
        }
    }
    ownv[0] = Hkb + ekb;
    ownv[1] = ukb;
    ownv[2] = vkb;
    ownv[3] = hkb - ekb;
    }
    // Hand the contributions over: to a stencil member in this tile through
    // the LDS slot of its face state (the slot of the face it shares with
    // this cell; every reader of face states is past the barrier), to one in
    // another tile through c.x for the gather kernels.
    __syncthreads();
    if (own) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const uint32_t s = sl[j];
            if (s == kWallSlot) continue;
            if (int64_t(s >> 3) / kTile == int64_t(t)) {
                const int slot = int(tm.nloc[j * nc + k] & 0x7FFFu);
#pragma unroll
                for (int q = 0; q < 4; ++q) lds[q * stride + slot] = con[j][q];
            } else {
                // slot 3 kTile + b: halo item b of this tile names the member
                const int b = int(tm.nloc[j * nc + k] & 0x7FFFu) - 3 * kTile;
                c.x[tm.bstart[t] + b] = Adj4{con[j][0], con[j][1], con[j][2], con[j][3]};
            }
        }
    }
    __syncthreads();
    if (own) {
        // own + the contributions of the stencil members in this tile, in
        // face order; those from other tiles follow in the gather
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const uint32_t s = sl[j];
            if (s == kWallSlot || int64_t(s >> 3) / kTile != int64_t(t)) continue;
            const int slot = j * kTile + i;
#pragma unroll
            for (int q = 0; q < 4; ++q) ownv[q] += lds[q * stride + slot];
        }
        c.own[k] = Adj4{ownv[0], ownv[1], ownv[2], ownv[3]};
    }
}

namespace {

// own (with the contributions from its own tile) + the stencil contributions
// the face neighbours in other tiles made to cell k, in face order
__device__ __forceinline__ Adj4 gather_cell(const DevMesh& m, const AdjC& c, int64_t k) {
    Adj4 a = c.own[k];
    const int32_t x[3] = {c.xin[k], c.xin[m.nc + k], c.xin[2 * m.nc + k]};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        if (x[j] < 0) continue;
        const Adj4 v = c.x[x[j]];
        a.H += v.H; a.HU += v.HU; a.HV += v.HV; a.h += v.h;
    }
    return a;
}

}  // namespace

__global__ __launch_bounds__(kBlock) void adj_gather_rk2_kernel(
    DevMesh m, TileMap tm, AdjC c, const Adj4* __restrict__ lam,
    const uint8_t* __restrict__ mask2, const uint8_t* __restrict__ mask1,
    const double* __restrict__ R0, double dt, double* __restrict__ mua, Adj4* __restrict__ lamn,
    double* __restrict__ part, const Cell4* __restrict__ W, double g, double thr,
    const unsigned long long* rmin, unsigned long long* argmin) {
    const TileInfo ti = tile_info(tm.tinfo[blockIdx.x]);
    const int64_t k = int64_t(blockIdx.x) * kTile + threadIdx.x;
    double d = 0.0;
    if (int(threadIdx.x) < ti.cnt) {
        if (argmin) {
            // the cell that set dt: the lowest index whose CFL ratio has the
            // bits of the minimum
            const Cell4 q = W[k];
            const double rr = cfl_ratio(q.H, q.HU, q.HV, m.area[k], m.perim[k], g, thr);
            if (rr < __longlong_as_double(0x7FF0000000000000ll) && dbits(rr) == *rmin)
                atomicMin(argmin, (unsigned long long)k);
        }
        const Adj4 w = gather_cell(m, c, k);
        const uint8_t m2 = mask2[k], m1 = mask1[k];
        const Adj4 l = lam[k];
        const double a0 = ((m2 & 1) ? 0.5 * l.H : 0.0) + w.H;
        const double a1 = ((m2 & 2) ? 0.5 * l.HU : 0.0) + w.HU;
        const double a2 = ((m2 & 2) ? 0.5 * l.HV : 0.0) + w.HV;
        const double t0 = (m1 & 1) ? a0 : 0.0, t1 = (m1 & 2) ? a1 : 0.0, t2 = (m1 & 2) ? a2 : 0.0;
        const double ra = rcp_of(m.area[k]).r;
        mua[3 * k] = (dt * t0) * ra;
        mua[3 * k + 1] = (dt * t1) * ra;
        mua[3 * k + 2] = (dt * t2) * ra;
        Adj4 n = lamn[k];
        n.H += t0; n.HU += t1; n.HV += t2;
        n.h += w.h;
        lamn[k] = n;
        d = t0 * R0[3 * k] + t1 * R0[3 * k + 1] + t2 * R0[3 * k + 2];
    }
    const double s = block_sum(d);
    if (threadIdx.x == 0) part[blockIdx.x] += s;
}

__global__ __launch_bounds__(kBlock) void adj_turn_kernel(
    DevMesh m, TileMap tm, AdjC c, const Cell4* __restrict__ W, double g,
    double thr, double cfl, const unsigned long long* argmin, const double* __restrict__ part,
    const int64_t* cells, int ng, const double* r, Adj4* __restrict__ lamn,
    const uint8_t* __restrict__ mask2p,
    const double* __restrict__ R1p, double dtp, double* __restrict__ mua,
    Adj4* __restrict__ lamp, double* __restrict__ partp) {
    const TileInfo ti = tile_info(tm.tinfo[blockIdx.x]);
    const int64_t k = int64_t(blockIdx.x) * kTile + threadIdx.x;
    double d = 0.0;
    // the adjoint of dt, sum of part[] in fixed order, formed by the block
    // that holds the minimising cell
    double lamdt = 0.0;
    if (argmin && *argmin / kTile == (unsigned long long)blockIdx.x) {
        __shared__ double tot;
        double sp = 0.0;
        for (int i = threadIdx.x; i < int(gridDim.x); i += kBlock) sp += part[i];
        const double t = block_sum(sp);
        if (threadIdx.x == 0) tot = t;
        __syncthreads();
        lamdt = tot;
    }
    if (int(threadIdx.x) < ti.cnt) {
        // after J_R(w)^T: the contributions gathered in fixed order
        const Adj4 w = gather_cell(m, c, k);
        Adj4 n = lamn[k];
        n.H += w.H; n.HU += w.HU; n.HV += w.HV;
        double hb = n.h + w.h;
        if (argmin && (unsigned long long)k == *argmin) {
            // dt = CFL ratio of the minimising cell (the first in the
            // internal order among cells of equal ratio)
            const Cell4 q = W[k];
            const double rr = cfl_ratio(q.H, q.HU, q.HV, m.area[k], m.perim[k], g, thr);
            {
                const double u = q.HU / q.H, v = q.HV / q.H;
                const double m2 = u * u + v * v, mm = sqrt(m2), c = sqrt(g * q.H), sp = mm + c;
                const double sb = -(lamdt * cfl) * rr / sp;
                const double ub = (m2 > 0.0) ? sb * u / mm : 0.0;
                const double vb = (m2 > 0.0) ? sb * v / mm : 0.0;
                n.H += sb * g / (2.0 * c) - (ub * u + vb * v) / q.H;
                n.HU += ub / q.H;
                n.HV += vb / q.H;
            }
        }
        if (r) {
            // gauge misfit of w^k, in gauge order (gauges may share a cell)
            for (int gi = 0; gi < ng; ++gi)
                if (cells[gi] == k) {
                    n.H += 2.0 * r[gi];
                    hb -= 2.0 * r[gi];
                }
        }
        n.h = hb;
        lamn[k] = n;
        if (mask2p) {
            // the start of the reverse of step k-1 (as adj_start_kernel)
            const uint8_t mk = mask2p[k];
            const double l0 = (mk & 1) ? n.H : 0.0, l1 = (mk & 2) ? n.HU : 0.0,
                         l2 = (mk & 2) ? n.HV : 0.0;
            const double ra = rcp_of(m.area[k]).r;
            mua[3 * k] = (0.5 * dtp * l0) * ra;
            mua[3 * k + 1] = (0.5 * dtp * l1) * ra;
            mua[3 * k + 2] = (0.5 * dtp * l2) * ra;
            lamp[k] = Adj4{0.5 * l0, 0.5 * l1, 0.5 * l2, hb};
            d = 0.5 * (l0 * R1p[3 * k] + l1 * R1p[3 * k + 1] + l2 * R1p[3 * k + 2]);
        }
    }
    if (mask2p) {
        const double s = block_sum(d);
        if (threadIdx.x == 0) partp[blockIdx.x] = s;
    }
}


// ---------------------------------------------------------------- loss and output

__global__ void adj_gauge_kernel(const int64_t* cells, int ng, const double* r, Adj4* lam) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    for (int i = 0; i < ng; ++i) {  // one thread: gauges may share a cell
        const int64_t k = cells[i];
        lam[k].H += 2.0 * r[i];
        lam[k].h -= 2.0 * r[i];
    }
}

__global__ void adj_unpack_kernel(int64_t n, const int64_t* perm, const Adj4* lam, double* gH,
                                  double* gHU, double* gHV, double* gh) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t k = perm[i];
    if (k < 0) return;
    gH[k] = lam[i].H;
    gHU[k] = lam[i].HU;
    gHV[k] = lam[i].HV;
    gh[k] = lam[i].h;
}

}  // namespace vsw
