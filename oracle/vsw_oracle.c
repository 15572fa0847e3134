/*
 * Plain FP64 CPU oracle of the shallow-water finite-volume stage.
 * TEST INFRASTRUCTURE ONLY (see vsw_oracle.h).  Parity for the numerical
 * scheme is pinned by the tests in tests/test_oracle_*.py against closed
 * forms (Thacker, Ritter), invariants (lake at rest, mass, symmetry) and
 * textbook identities of the HLL flux; no oracle value comes from the GPU.
 *
 * Paper: Giles, Kashdan, Salmanidou, Guillas, Dias, "Performance analysis of
 * Volna-OP2 -- massively parallel code for tsunami modelling" (2020).
 *   Section 2.1  the NSWE, w = (H, Hu, Hv), H = h + eta
 *   Section 2.2  cell-centred FV, HLL flux, wave speeds after Zhou et al.
 *   Section 2.3  SSP-RK(2,2), CFL condition
 *   Section 2.4  MUSCL: least-squares gradient, Barth-Jespersen limiter,
 *                reconstruction eq. (3), threshold depth H_thr
 *   Section 2.5  wall boundary by ghost cells
 * Where the paper is silent the readings used are listed in the design notes
 * of the repository; each one is named at its use below (hydrostatic
 * reconstruction, dry-bed speeds, CFL formula, ...).
 *
 * Build: gcc -O3 -fopenmp -ffp-contract=off -fno-fast-math (no FMA
 * contraction, so every operation is one IEEE-754 rounding in the order
 * written).  OpenMP splits only loops whose iterations are independent (one
 * cell or one face per iteration, each writing its own outputs), plus the
 * exact min and integer-count reductions, so every result is bitwise the
 * same for any thread count.
 */
#include "vsw_oracle.h"

#include <math.h>
#include <omp.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

struct orc_mesh {
    int64_t nc, nv, ne, nw;
    double *vx, *vy;   /* vertex coordinates */
    int32_t *tri;      /* 3*nc, counter-clockwise */
    double *h;         /* still-water depth at centroids (h = -z) */
    int32_t *nbr;      /* 3*nc, neighbour across face j, -1 = wall */
    int32_t *isl;      /* 3*nc, 1 if the cell is the canonical left side */
    double *cx, *cy, *area, *perim;
    double *len, *nx, *ny, *dx, *dy, *wx, *wy; /* 3*nc */
    int32_t *ecell;    /* 2*ne: left cell, right cell (-1 = wall) */
    int32_t *eface;    /* 2*ne: local face index in left / right cell */
};

/* ---------------------------------------------------------------- helpers */

static double mind(double a, double b) { return (b < a) ? b : a; }
static double maxd(double a, double b) { return (b > a) ? b : a; }
static double pos(double a) { return (a > 0.0) ? a : 0.0; }

static void set_err(char *err, int errlen, const char *fmt, ...) {
    if (!err || errlen <= 0) return;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(err, (size_t)errlen, fmt, ap);
    va_end(ap);
}

typedef struct {
    uint64_t key;
    int32_t cell;
    int32_t face;
} half_edge;

static int cmp_half(const void *pa, const void *pb) {
    const half_edge *a = (const half_edge *)pa, *b = (const half_edge *)pb;
    if (a->key != b->key) return (a->key < b->key) ? -1 : 1;
    if (a->cell != b->cell) return (a->cell < b->cell) ? -1 : 1;
    return (a->face < b->face) ? -1 : (a->face > b->face);
}

void orc_mesh_free(orc_mesh *m) {
    if (!m) return;
    free(m->vx); free(m->vy); free(m->tri); free(m->h); free(m->nbr);
    free(m->isl); free(m->cx); free(m->cy); free(m->area); free(m->perim);
    free(m->len); free(m->nx); free(m->ny); free(m->dx); free(m->dy);
    free(m->wx); free(m->wy); free(m->ecell); free(m->eface);
    free(m);
}

/* Lexicographic (x, y) order of two vertices: the canonical left side of an
 * interior face is the cell that runs along it from the smaller vertex. */
static int vertex_less(const orc_mesh *m, int32_t a, int32_t b) {
    if (m->vx[a] != m->vx[b]) return m->vx[a] < m->vx[b];
    return m->vy[a] < m->vy[b];
}

/* ------------------------------------------------------------ mesh build */

orc_mesh *orc_mesh_build(int64_t nv, const double *vx, const double *vy,
                         int64_t nc, const int32_t *tri, const double *h,
                         char *err, int errlen) {
    if (nv <= 0 || nc <= 0) {
        set_err(err, errlen, "empty mesh (nv=%lld, nc=%lld)", (long long)nv, (long long)nc);
        return NULL;
    }
    orc_mesh *m = (orc_mesh *)calloc(1, sizeof(orc_mesh));
    m->nc = nc;
    m->nv = nv;
    m->vx = (double *)malloc(sizeof(double) * nv);
    m->vy = (double *)malloc(sizeof(double) * nv);
    memcpy(m->vx, vx, sizeof(double) * nv);
    memcpy(m->vy, vy, sizeof(double) * nv);
    m->tri = (int32_t *)malloc(sizeof(int32_t) * 3 * nc);
    m->h = (double *)malloc(sizeof(double) * nc);
    memcpy(m->h, h, sizeof(double) * nc);
    m->nbr = (int32_t *)malloc(sizeof(int32_t) * 3 * nc);
    m->isl = (int32_t *)malloc(sizeof(int32_t) * 3 * nc);
    double **arrs3[] = {&m->len, &m->nx, &m->ny, &m->dx, &m->dy, &m->wx, &m->wy};
    for (int i = 0; i < 7; ++i) *arrs3[i] = (double *)malloc(sizeof(double) * 3 * nc);
    m->cx = (double *)malloc(sizeof(double) * nc);
    m->cy = (double *)malloc(sizeof(double) * nc);
    m->area = (double *)malloc(sizeof(double) * nc);
    m->perim = (double *)malloc(sizeof(double) * nc);

    /* Orientation: counter-clockwise, swapping local vertices 1 and 2 of a
     * clockwise triangle; zero area is an error. */
    for (int64_t k = 0; k < nc; ++k) {
        int32_t a = tri[3 * k], b = tri[3 * k + 1], c = tri[3 * k + 2];
        if (a < 0 || a >= nv || b < 0 || b >= nv || c < 0 || c >= nv) {
            set_err(err, errlen, "triangle %lld has a vertex index out of range (nv=%lld)", (long long)k, (long long)nv);
            orc_mesh_free(m);
            return NULL;
        }
        double cr = (vx[b] - vx[a]) * (vy[c] - vy[a]) - (vx[c] - vx[a]) * (vy[b] - vy[a]);
        if (!(cr != 0.0) || !isfinite(cr)) {
            set_err(err, errlen, "triangle %lld is degenerate (zero area)", (long long)k);
            orc_mesh_free(m);
            return NULL;
        }
        if (cr < 0.0) { int32_t t = b; b = c; c = t; }
        m->tri[3 * k] = a;
        m->tri[3 * k + 1] = b;
        m->tri[3 * k + 2] = c;
    }

    /* Faces: sort the 3*nc directed faces by their undirected vertex pair. */
    int64_t nh = 3 * nc;
    half_edge *he = (half_edge *)malloc(sizeof(half_edge) * nh);
    for (int64_t k = 0; k < nc; ++k)
        for (int j = 0; j < 3; ++j) {
            uint32_t a = (uint32_t)m->tri[3 * k + j];
            uint32_t b = (uint32_t)m->tri[3 * k + (j + 1) % 3];
            uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
            he[3 * k + j].key = ((uint64_t)lo << 32) | hi;
            he[3 * k + j].cell = (int32_t)k;
            he[3 * k + j].face = j;
        }
    qsort(he, (size_t)nh, sizeof(half_edge), cmp_half);
    int64_t ne = 0, nw = 0;
    for (int64_t i = 0; i < nh;) {
        int64_t r = i + 1;
        while (r < nh && he[r].key == he[i].key) ++r;
        if (r - i > 2) {
            set_err(err, errlen, "edge shared by more than two triangles (cell %lld)",
                    (long long)he[i].cell);
            free(he);
            orc_mesh_free(m);
            return NULL;
        }
        ++ne;
        if (r - i == 1) ++nw;
        i = r;
    }
    m->ne = ne;
    m->nw = nw;
    m->ecell = (int32_t *)malloc(sizeof(int32_t) * 2 * ne);
    m->eface = (int32_t *)malloc(sizeof(int32_t) * 2 * ne);
    int64_t e = 0;
    for (int64_t i = 0; i < nh;) {
        int64_t r = i + 1;
        while (r < nh && he[r].key == he[i].key) ++r;
        int32_t k1 = he[i].cell, j1 = he[i].face;
        int32_t a1 = m->tri[3 * k1 + j1], b1 = m->tri[3 * k1 + (j1 + 1) % 3];
        if (r - i == 1) {
            m->nbr[3 * k1 + j1] = -1;
            m->isl[3 * k1 + j1] = 1;
            m->ecell[2 * e] = k1; m->eface[2 * e] = j1;
            m->ecell[2 * e + 1] = -1; m->eface[2 * e + 1] = -1;
        } else {
            int32_t k2 = he[i + 1].cell, j2 = he[i + 1].face;
            int32_t a2 = m->tri[3 * k2 + j2];
            if (a2 == a1 || k1 == k2) {
                set_err(err, errlen, "triangles %lld and %lld overlap (same edge direction)",
                        (long long)k1, (long long)k2);
                free(he);
                orc_mesh_free(m);
                return NULL;
            }
            if (m->vx[a1] == m->vx[b1] && m->vy[a1] == m->vy[b1]) {
                set_err(err, errlen, "duplicate vertex coordinates in cell %lld", (long long)k1);
                free(he);
                orc_mesh_free(m);
                return NULL;
            }
            int first_left = vertex_less(m, a1, b1);
            int32_t kl = first_left ? k1 : k2, jl = first_left ? j1 : j2;
            int32_t kr = first_left ? k2 : k1, jr = first_left ? j2 : j1;
            m->nbr[3 * kl + jl] = kr; m->isl[3 * kl + jl] = 1;
            m->nbr[3 * kr + jr] = kl; m->isl[3 * kr + jr] = 0;
            m->ecell[2 * e] = kl; m->eface[2 * e] = jl;
            m->ecell[2 * e + 1] = kr; m->eface[2 * e + 1] = jr;
        }
        ++e;
        i = r;
    }
    free(he);

    /* Geometry (Section 2.4: cell centre x_0, face centre x_f). */
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nc; ++k) {
        const int32_t *t = m->tri + 3 * k;
        double x0 = m->vx[t[0]], x1 = m->vx[t[1]], x2 = m->vx[t[2]];
        double y0 = m->vy[t[0]], y1 = m->vy[t[1]], y2 = m->vy[t[2]];
        double cr = (x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0);
        m->area[k] = 0.5 * cr;
        m->cx[k] = (x0 + x1 + x2) / 3.0;
        m->cy[k] = (y0 + y1 + y2) / 3.0;
        for (int j = 0; j < 3; ++j) {
            double xa = m->vx[t[j]], ya = m->vy[t[j]];
            double xb = m->vx[t[(j + 1) % 3]], yb = m->vy[t[(j + 1) % 3]];
            double ex = xb - xa, ey = yb - ya;
            double l = sqrt(ex * ex + ey * ey);
            m->len[3 * k + j] = l;
            m->nx[3 * k + j] = ey / l;     /* outward unit normal */
            m->ny[3 * k + j] = -ex / l;
            m->dx[3 * k + j] = (xa + xb) * 0.5 - m->cx[k];
            m->dy[3 * k + j] = (ya + yb) * 0.5 - m->cy[k];
        }
        m->perim[k] = m->len[3 * k] + m->len[3 * k + 1] + m->len[3 * k + 2];
    }
    /* Least-squares weights: grad q = M^-1 sum_j delta_j (q_Sj - q_K) with
     * M = sum_j delta_j delta_j^T, written as sum_j w_j (q_Sj - q_K),
     * w_j = M^-1 delta_j.  delta_j runs from the centroid to the neighbour
     * centroid, or to the wall ghost: the centroid mirrored in the face. */
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nc; ++k) {
        double ddx[3], ddy[3];
        for (int j = 0; j < 3; ++j) {
            int32_t n = m->nbr[3 * k + j];
            if (n >= 0) {
                ddx[j] = m->cx[n] - m->cx[k];
                ddy[j] = m->cy[n] - m->cy[k];
            } else {
                double fnx = m->nx[3 * k + j], fny = m->ny[3 * k + j];
                double dn = m->dx[3 * k + j] * fnx + m->dy[3 * k + j] * fny;
                ddx[j] = (2.0 * dn) * fnx;
                ddy[j] = (2.0 * dn) * fny;
            }
        }
        double mxx = ddx[0] * ddx[0] + ddx[1] * ddx[1] + ddx[2] * ddx[2];
        double mxy = ddx[0] * ddy[0] + ddx[1] * ddy[1] + ddx[2] * ddy[2];
        double myy = ddy[0] * ddy[0] + ddy[1] * ddy[1] + ddy[2] * ddy[2];
        double det = mxx * myy - mxy * mxy;
        for (int j = 0; j < 3; ++j) {
            m->wx[3 * k + j] = (myy * ddx[j] - mxy * ddy[j]) / det;
            m->wy[3 * k + j] = (mxx * ddy[j] - mxy * ddx[j]) / det;
        }
    }
    return m;
}

int64_t orc_mesh_ncells(const orc_mesh *m) { return m->nc; }
int64_t orc_mesh_nedges(const orc_mesh *m) { return m->ne; }
int64_t orc_mesh_nwalls(const orc_mesh *m) { return m->nw; }

void orc_mesh_geometry(const orc_mesh *m, double *cx, double *cy,
                       double *area, double *perim, double *len, double *nx,
                       double *ny, double *dx, double *dy, double *wx,
                       double *wy, int32_t *nbr, int32_t *is_left,
                       int32_t *tri_oriented) {
    size_t n1 = sizeof(double) * m->nc, n3 = 3 * n1;
    if (cx) memcpy(cx, m->cx, n1);
    if (cy) memcpy(cy, m->cy, n1);
    if (area) memcpy(area, m->area, n1);
    if (perim) memcpy(perim, m->perim, n1);
    if (len) memcpy(len, m->len, n3);
    if (nx) memcpy(nx, m->nx, n3);
    if (ny) memcpy(ny, m->ny, n3);
    if (dx) memcpy(dx, m->dx, n3);
    if (dy) memcpy(dy, m->dy, n3);
    if (wx) memcpy(wx, m->wx, n3);
    if (wy) memcpy(wy, m->wy, n3);
    if (nbr) memcpy(nbr, m->nbr, sizeof(int32_t) * 3 * m->nc);
    if (is_left) memcpy(is_left, m->isl, sizeof(int32_t) * 3 * m->nc);
    if (tri_oriented) memcpy(tri_oriented, m->tri, sizeof(int32_t) * 3 * m->nc);
}

/* ------------------------------------------------------------ HLL flux */

/* HLL flux (Section 2.2) in the face frame: states (H, u_n, u_t), flux of
 * the 1D system (H u_n, H u_n^2 + g H^2 / 2, H u_n u_t).
 * Wave speeds: two-rarefaction estimate u*, c* of Zhou et al. when both
 * sides are wet; when one side is dry the dry-bed speeds u - c / u + 2c
 * (reading of the shoreline Riemann problem the paper cites). */
static void hll_face_frame(double g, double HL, double unL, double utL,
                           double HR, double unR, double utR, double *f,
                           double *speeds) {
    const double hg = 0.5 * g;
    if (HL == 0.0 && HR == 0.0) {
        f[0] = 0.0; f[1] = 0.0; f[2] = 0.0;
        if (speeds) { speeds[0] = 0.0; speeds[1] = 0.0; speeds[2] = NAN; speeds[3] = NAN; }
        return;
    }
    double cL = sqrt(g * HL), cR = sqrt(g * HR);
    double sL, sR, us = NAN, cs = NAN;
    if (HL == 0.0) {
        sL = unR - 2.0 * cR;
        sR = unR + cR;
    } else if (HR == 0.0) {
        sL = unL - cL;
        sR = unL + 2.0 * cL;
    } else {
        us = 0.5 * (unL + unR) + (cL - cR);
        cs = 0.5 * (cL + cR) - 0.25 * (unR - unL);
        sL = mind(unL - cL, us - cs);
        sR = maxd(us + cs, unR + cR);
    }
    if (speeds) { speeds[0] = sL; speeds[1] = sR; speeds[2] = us; speeds[3] = cs; }
    double qL = HL * unL, qR = HR * unR;
    double wL[3] = {HL, qL, HL * utL};
    double wR[3] = {HR, qR, HR * utR};
    double fL[3] = {qL, qL * unL + hg * (HL * HL), qL * utL};
    double fR[3] = {qR, qR * unR + hg * (HR * HR), qR * utR};
    if (sL >= 0.0) {
        f[0] = fL[0]; f[1] = fL[1]; f[2] = fL[2];
    } else if (sR < 0.0) {
        f[0] = fR[0]; f[1] = fR[1]; f[2] = fR[2];
    } else {
        /* the star flux of Section 2.2 over (s_R - s_L) */
        double den = sR - sL, sLR = sL * sR;
        for (int c = 0; c < 3; ++c)
            f[c] = ((sR * fL[c] - sL * fR[c]) + sLR * (wR[c] - wL[c])) / den;
    }
}

void orc_hll(double g, const double *wl, const double *wr, double nx,
             double ny, double *phi, double *speeds) {
    /* wl, wr = (H, u, v) */
    double unL = wl[1] * nx + wl[2] * ny, utL = wl[2] * nx - wl[1] * ny;
    double unR = wr[1] * nx + wr[2] * ny, utR = wr[2] * nx - wr[1] * ny;
    double f[3];
    hll_face_frame(g, wl[0], unL, utL, wr[0], unR, utR, f, speeds);
    phi[0] = f[0];
    phi[1] = f[1] * nx - f[2] * ny;
    phi[2] = f[1] * ny + f[2] * nx;
}

/* Face flux with the hydrostatic reconstruction of Audusse et al. (the
 * reading of the bathymetry source, which the paper does not discretise):
 * h* = min(h_L, h_R), H*_s = max(0, eta_s + h*).  A wall face (right ==
 * NULL) takes the mirror of the left state in the face frame: same depth,
 * normal velocity reversed, tangential kept (Section 2.5). */
void orc_face_flux(const orc_params *p, const double *left,
                   const double *right, double nx, double ny, double *phi,
                   double *pcorr) {
    const double hg = 0.5 * p->g;
    double etaL = left[0], hL = left[1], HL = left[2], uL = left[3], vL = left[4];
    double unL = uL * nx + vL * ny, utL = vL * nx - uL * ny;
    double f[3];
    if (right == NULL) {
        double hs = hL;
        double HsL = pos(etaL + hs);
        hll_face_frame(p->g, HsL, unL, utL, HsL, -unL, utL, f, NULL);
        pcorr[0] = hg * (HL * HL - HsL * HsL);
        pcorr[1] = 0.0;
    } else {
        double etaR = right[0], hR = right[1], HR = right[2], uR = right[3], vR = right[4];
        double unR = uR * nx + vR * ny, utR = vR * nx - uR * ny;
        double hs = mind(hL, hR);
        double HsL = pos(etaL + hs), HsR = pos(etaR + hs);
        hll_face_frame(p->g, HsL, unL, utL, HsR, unR, utR, f, NULL);
        pcorr[0] = hg * (HL * HL - HsL * HsL);
        pcorr[1] = hg * (HR * HR - HsR * HsR);
    }
    phi[0] = f[0];
    phi[1] = f[1] * nx - f[2] * ny;
    phi[2] = f[1] * ny + f[2] * nx;
}

/* ------------------------------------------------------------ reconstruction */

/* Reconstruction of cell k (Section 2.4, eq. (3)).
 * Variables: eta = H - h, Hu, Hv limited by Barth-Jespersen; h
 * reconstructed with its unlimited gradient.  Second order only when the
 * cell, its three stencil members and its three reconstructed face depths
 * all reach H_thr; otherwise every face takes the cell value. */
static void recon_cell(const orc_mesh *m, const orc_params *p, const double *H,
                       const double *HU, const double *HV, int64_t k,
                       double *face, double *grad, double *alpha, int *order,
                       double *sc) {
    const double thr = p->h_threshold;
    const double Hk = H[k], hk = m->h[k], ek = Hk - hk, uk = HU[k], vk = HV[k];
    double qs[4][3]; /* stencil values of eta, Hu, Hv, h */
    int cand = (Hk >= thr);
    for (int j = 0; j < 3; ++j) {
        int32_t n = m->nbr[3 * k + j];
        double Hs;
        if (n >= 0) {
            Hs = H[n];
            qs[0][j] = H[n] - m->h[n];
            qs[1][j] = HU[n];
            qs[2][j] = HV[n];
            qs[3][j] = m->h[n];
        } else {
            /* wall ghost: mirrored momentum, same depth and surface */
            double fnx = m->nx[3 * k + j], fny = m->ny[3 * k + j];
            double mn = uk * fnx + vk * fny;
            Hs = Hk;
            qs[0][j] = ek;
            qs[1][j] = uk - (2.0 * mn) * fnx;
            qs[2][j] = vk - (2.0 * mn) * fny;
            qs[3][j] = hk;
        }
        if (!(Hs >= thr)) cand = 0;
    }
    const double qk[4] = {ek, uk, vk, hk};
    double g[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    double al[3] = {0, 0, 0};
    double fq[4][3]; /* face values of eta, Hu, Hv, h */
    double fH[3];
    if (cand) {
        const double *wx = m->wx + 3 * k, *wy = m->wy + 3 * k;
        for (int q = 0; q < 4; ++q) {
            double d0 = qs[q][0] - qk[q], d1 = qs[q][1] - qk[q], d2 = qs[q][2] - qk[q];
            g[q][0] = wx[0] * d0 + wx[1] * d1 + wx[2] * d2;
            g[q][1] = wy[0] * d0 + wy[1] * d1 + wy[2] * d2;
        }
        double proj[4][3];
        for (int q = 0; q < 4; ++q)
            for (int j = 0; j < 3; ++j)
                proj[q][j] = g[q][0] * m->dx[3 * k + j] + g[q][1] * m->dy[3 * k + j];
        /* Barth-Jespersen: the largest alpha in [0,1] that keeps every face
         * value inside the range of the cell and its stencil members. */
        for (int q = 0; q < 3; ++q) {
            double qmax = qk[q], qmin = qk[q];
            for (int j = 0; j < 3; ++j) {
                qmax = maxd(qmax, qs[q][j]);
                qmin = mind(qmin, qs[q][j]);
            }
            double a = 1.0;
            for (int j = 0; j < 3; ++j) {
                double d = proj[q][j], phi = 1.0;
                if (d > 0.0) phi = mind(1.0, (qmax - qk[q]) / d);
                else if (d < 0.0) phi = mind(1.0, (qmin - qk[q]) / d);
                a = mind(a, phi);
            }
            al[q] = a;
        }
        for (int j = 0; j < 3; ++j) {
            for (int q = 0; q < 3; ++q) fq[q][j] = qk[q] + al[q] * proj[q][j];
            fq[3][j] = hk + proj[3][j];
            fH[j] = fq[0][j] + fq[3][j];
            if (fH[j] < thr) cand = 0;
        }
    }
    if (!cand) {
        for (int j = 0; j < 3; ++j) {
            for (int q = 0; q < 4; ++q) fq[q][j] = qk[q];
            fH[j] = Hk;
        }
    }
    if (face) {
        for (int j = 0; j < 3; ++j) {
            double *f = face + 15 * k + 5 * j;
            f[0] = fq[0][j];
            f[1] = fq[3][j];
            f[2] = fH[j];
            if (fH[j] >= thr) {
                f[3] = fq[1][j] / fH[j];
                f[4] = fq[2][j] / fH[j];
            } else {
                f[3] = 0.0;
                f[4] = 0.0;
            }
        }
    }
    if (grad)
        for (int q = 0; q < 4; ++q) {
            grad[8 * k + 2 * q] = g[q][0];
            grad[8 * k + 2 * q + 1] = g[q][1];
        }
    if (alpha)
        for (int q = 0; q < 3; ++q) alpha[3 * k + q] = cand ? al[q] : 0.0;
    if (order) *order = cand ? 2 : 1;
    if (sc) {
        /* Centred part of the bathymetry source for second-order cells:
         * (g/2) sum_j l_j (H_K + H_Kj)(h_Kj - h_K) n_j. */
        sc[0] = 0.0;
        sc[1] = 0.0;
        if (cand) {
            const double hg = 0.5 * p->g;
            double c[3];
            for (int j = 0; j < 3; ++j)
                c[j] = (m->len[3 * k + j] * (Hk + fH[j])) * (fq[3][j] - hk);
            const double *fnx = m->nx + 3 * k, *fny = m->ny + 3 * k;
            double sx = c[0] * fnx[0] + c[1] * fnx[1] + c[2] * fnx[2];
            double sy = c[0] * fny[0] + c[1] * fny[1] + c[2] * fny[2];
            sc[0] = hg * sx;
            sc[1] = hg * sy;
        }
    }
}

void orc_reconstruct(const orc_mesh *m, const orc_params *p, const double *H,
                     const double *HU, const double *HV, double *grad,
                     double *alpha, int32_t *order, double *face) {
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < m->nc; ++k) {
        int o;
        recon_cell(m, p, H, HU, HV, k, face, grad, alpha, &o, NULL);
        if (order) order[k] = o;
    }
}

/* ------------------------------------------------------------ residual */

void orc_residual(const orc_mesh *m, const orc_params *p, const double *H,
                  const double *HU, const double *HV, double *RH, double *RHU,
                  double *RHV) {
    const int64_t nc = m->nc;
    double *face = (double *)malloc(sizeof(double) * 15 * nc);
    double *sc = (double *)malloc(sizeof(double) * 2 * nc);
    int *ord = (int *)malloc(sizeof(int) * nc);
    double *term = (double *)malloc(sizeof(double) * 9 * nc); /* per face side */

    /* 1. cell loop: reconstruction */
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nc; ++k)
        recon_cell(m, p, H, HU, HV, k, face, NULL, NULL, &ord[k], sc + 2 * k);

    /* 2. edge loop: one flux per face in canonical orientation; each side
     *    keeps l * (phi + (0, p_side n)) */
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m->ne; ++e) {
        int32_t kl = m->ecell[2 * e], jl = m->eface[2 * e];
        int32_t kr = m->ecell[2 * e + 1], jr = m->eface[2 * e + 1];
        double fnx = m->nx[3 * kl + jl], fny = m->ny[3 * kl + jl];
        double l = m->len[3 * kl + jl];
        double phi[3], pc[2];
        const double *fl = face + 15 * kl + 5 * jl;
        const double *fr = (kr >= 0) ? face + 15 * kr + 5 * jr : NULL;
        orc_face_flux(p, fl, fr, fnx, fny, phi, pc);
        double *tl = term + 9 * kl + 3 * jl;
        tl[0] = l * phi[0];
        tl[1] = l * (phi[1] + pc[0] * fnx);
        tl[2] = l * (phi[2] + pc[0] * fny);
        if (kr >= 0) {
            double *tr = term + 9 * kr + 3 * jr;
            tr[0] = l * phi[0];
            tr[1] = l * (phi[1] + pc[1] * fnx);
            tr[2] = l * (phi[2] + pc[1] * fny);
        }
    }

    /* 3. cell loop: gather the three faces in local order, add the source,
     *    divide by the area */
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nc; ++k) {
        double acc[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j < 3; ++j) {
            const double *t = term + 9 * k + 3 * j;
            if (m->isl[3 * k + j]) {
                acc[0] = acc[0] - t[0];
                acc[1] = acc[1] - t[1];
                acc[2] = acc[2] - t[2];
            } else {
                acc[0] = acc[0] + t[0];
                acc[1] = acc[1] + t[1];
                acc[2] = acc[2] + t[2];
            }
        }
        if (ord[k] == 2) {
            acc[1] = acc[1] + sc[2 * k];
            acc[2] = acc[2] + sc[2 * k + 1];
        }
        RH[k] = acc[0] / m->area[k];
        RHU[k] = acc[1] / m->area[k];
        RHV[k] = acc[2] / m->area[k];
    }
    free(face); free(sc); free(ord); free(term);
}

/* ------------------------------------------------------------ time step */

/* CFL rule (reading of Section 2.3): dt = CFL * min over cells with
 * H >= H_thr of |K| / (P_K (|u_K| + sqrt(g H_K))). */
double orc_dt(const orc_mesh *m, const orc_params *p, const double *H,
              const double *HU, const double *HV) {
    double rmin = INFINITY;
    /* the minimum of a set does not depend on the order it is taken in */
#pragma omp parallel for schedule(static) reduction(min : rmin)
    for (int64_t k = 0; k < m->nc; ++k) {
        if (!(H[k] >= p->h_threshold)) continue;
        double u = HU[k] / H[k], v = HV[k] / H[k];
        double s = sqrt(u * u + v * v) + sqrt(p->g * H[k]);
        double r = m->area[k] / (m->perim[k] * s);
        rmin = mind(rmin, r);
    }
    return p->cfl * rmin;
}

static void post_fix(const orc_params *p, double *H, double *HU, double *HV,
                     int64_t k, int64_t *clamps) {
    if (H[k] < 0.0) {
        H[k] = 0.0;
        ++*clamps;
    }
    if (H[k] < p->h_threshold) {
        HU[k] = 0.0;
        HV[k] = 0.0;
    }
}

int orc_run(const orc_mesh *m, const orc_params *p, double *H, double *HU,
            double *HV, double *t, int64_t nsteps, double t_stop,
            int64_t *steps_done, double *dts, int64_t *clamps) {
    const int64_t nc = m->nc;
    double *H1 = (double *)malloc(sizeof(double) * nc);
    double *U1 = (double *)malloc(sizeof(double) * nc);
    double *V1 = (double *)malloc(sizeof(double) * nc);
    double *RH = (double *)malloc(sizeof(double) * nc);
    double *RU = (double *)malloc(sizeof(double) * nc);
    double *RV = (double *)malloc(sizeof(double) * nc);
    int rc = 0;
    int64_t done = 0, ncl = 0;
    for (int64_t s = 0; s < nsteps; ++s) {
        if (!(*t < t_stop)) break;
        double dt = (p->dt_fixed > 0.0) ? p->dt_fixed : orc_dt(m, p, H, HU, HV);
        double rem = t_stop - *t, tn;
        if (dt >= rem) {
            dt = rem;
            tn = t_stop;
        } else {
            tn = *t + dt;
        }
        if (!(dt > 0.0) || !isfinite(dt)) { rc = -1; break; }
        /* stage 1: w1 = w + dt L(w) */
        orc_residual(m, p, H, HU, HV, RH, RU, RV);
#pragma omp parallel for schedule(static) reduction(+ : ncl)
        for (int64_t k = 0; k < nc; ++k) {
            H1[k] = H[k] + dt * RH[k];
            U1[k] = HU[k] + dt * RU[k];
            V1[k] = HV[k] + dt * RV[k];
            post_fix(p, H1, U1, V1, k, &ncl);
        }
        /* stage 2: w^{n+1} = w/2 + (w1 + dt L(w1))/2 */
        orc_residual(m, p, H1, U1, V1, RH, RU, RV);
        int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : ncl) reduction(| : bad)
        for (int64_t k = 0; k < nc; ++k) {
            H[k] = 0.5 * H[k] + 0.5 * (H1[k] + dt * RH[k]);
            HU[k] = 0.5 * HU[k] + 0.5 * (U1[k] + dt * RU[k]);
            HV[k] = 0.5 * HV[k] + 0.5 * (V1[k] + dt * RV[k]);
            post_fix(p, H, HU, HV, k, &ncl);
            if (!isfinite(H[k]) || !isfinite(HU[k]) || !isfinite(HV[k])) bad = 1;
        }
        if (bad) { rc = -1; break; }
        if (dts) dts[done] = dt;
        *t = tn;
        ++done;
    }
    if (steps_done) *steps_done = done;
    if (clamps) *clamps = ncl;
    free(H1); free(U1); free(V1); free(RH); free(RU); free(RV);
    return rc;
}

void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

int orc_max_threads(void) { return omp_get_max_threads(); }
