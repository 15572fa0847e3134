// Host-side mesh preparation for the GPU solver.
//
// Geometry follows the cell-centred finite-volume discretisation of
// Section 2.2 and the reconstruction of Section 2.4 (cell centre x_0, face
// centre x_f, least-squares stencil of the three face neighbours, wall ghost
// cells of Section 2.5).  The arithmetic of every geometric quantity is
// written out operation by operation and the file is compiled without
// floating-point contraction, so the values are the IEEE-754 results of the
// expressions as written.
#include "vsw_mesh.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <numeric>

#include "../../include/vsw.h"

namespace vsw {
namespace {

// Hilbert index of (x, y) on a 2^16 x 2^16 grid (classic rotate-and-flip
// walk, most significant level first).
uint64_t hilbert16(uint32_t x, uint32_t y) {
    uint64_t d = 0;
    for (uint32_t s = 1u << 15; s > 0; s >>= 1) {
        uint32_t rx = (x & s) ? 1u : 0u;
        uint32_t ry = (y & s) ? 1u : 0u;
        d += uint64_t(s) * uint64_t(s) * ((3u * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) {
                x = (s - 1) - (x & (s - 1)) + (x & ~(s - 1));
                y = (s - 1) - (y & (s - 1)) + (y & ~(s - 1));
            }
            std::swap(x, y);
        }
    }
    return d;
}

// Recursive coordinate bisection of the cells idx[lo, hi) by their
// centroids: split at the median along the longer side of their bounding
// box into floor(nt / 2) whole tiles and the rest (nt = tiles needed),
// recursively, down to single tiles; the leaves in tree order (left first)
// are the tiles, compact patches with fewer faces on their boundary than
// runs of a space-filling curve.  Inside a leaf the cells follow `key`.
void bisect(std::vector<int64_t>& idx, int64_t lo, int64_t hi, const std::vector<double>& cx,
            const std::vector<double>& cy, const std::vector<uint64_t>& key, int64_t tile) {
    const int64_t n = hi - lo;
    if (n <= tile) {
        std::sort(idx.begin() + lo, idx.begin() + hi,
                  [&](int64_t a, int64_t b) { return key[a] < key[b]; });
        return;
    }
    const int64_t nt = (n + tile - 1) / tile;
    const int64_t nl = (nt / 2) * tile;
    double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
    for (int64_t i = lo; i < hi; ++i) {
        const int64_t k = idx[i];
        x0 = std::min(x0, cx[k]); x1 = std::max(x1, cx[k]);
        y0 = std::min(y0, cy[k]); y1 = std::max(y1, cy[k]);
    }
    const std::vector<double>& c = (x1 - x0 >= y1 - y0) ? cx : cy;
    // ties broken by the cell index: a strict order, so the split is unique
    std::nth_element(idx.begin() + lo, idx.begin() + lo + nl, idx.begin() + hi,
                     [&](int64_t a, int64_t b) { return c[a] < c[b] || (c[a] == c[b] && a < b); });
    bisect(idx, lo, lo + nl, cx, cy, key, tile);
    bisect(idx, lo + nl, hi, cx, cy, key, tile);
}

uint64_t splitmix64(uint64_t& st) {
    uint64_t z = (st += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

int build_host_mesh(int64_t nv, const double* vx, const double* vy, int64_t nc,
                    const int32_t* tri_in, const double* h_in, int ordering,
                    uint64_t seed, int tile, HostMesh& out, std::string& err) {
    char buf[256];
    if (nv <= 0 || nc <= 0 || !vx || !vy || !tri_in || !h_in) {
        err = "empty mesh or NULL array";
        return VSW_EINVAL;
    }
    if (nc > kMaxCells || nv > INT32_MAX) {
        err = "mesh too large for 29-bit cell indices";
        return VSW_EINVAL;
    }
    // vertex coordinates zero or within [2^-300, 2^300] in magnitude: edge
    // components are then zero or at least 2^-352 and every edge length,
    // normal and area a normal number far from both ends of the range,
    // which the stage kernels' face geometry relies on
    for (int64_t i = 0; i < nv; ++i)
        for (const double c : {vx[i], vy[i]}) {
            const double a = std::fabs(c);
            if (!(a == 0.0 || (a >= 0x1p-300 && a <= 0x1p300))) {
                snprintf(buf, sizeof buf,
                         "vertex %lld: coordinate %g not 0 or within [2^-300, 2^300] in magnitude",
                         (long long)i, c);
                err = buf;
                return VSW_EINVAL;
            }
        }
    // 1. counter-clockwise vertex order (swap local vertices 1 and 2 of a
    //    clockwise triangle)
    std::vector<int32_t> tri(3 * nc);
    for (int64_t k = 0; k < nc; ++k) {
        int32_t a = tri_in[3 * k], b = tri_in[3 * k + 1], c = tri_in[3 * k + 2];
        if (a < 0 || a >= nv || b < 0 || b >= nv || c < 0 || c >= nv) {
            snprintf(buf, sizeof buf, "triangle %lld: vertex index out of range", (long long)k);
            err = buf;
            return VSW_EMESH;
        }
        double cr = (vx[b] - vx[a]) * (vy[c] - vy[a]) - (vx[c] - vx[a]) * (vy[b] - vy[a]);
        if (!(cr != 0.0) || !std::isfinite(cr)) {
            snprintf(buf, sizeof buf, "triangle %lld: zero area", (long long)k);
            err = buf;
            return VSW_EMESH;
        }
        if (cr < 0.0) std::swap(b, c);
        tri[3 * k] = a;
        tri[3 * k + 1] = b;
        tri[3 * k + 2] = c;
    }
    for (int64_t i = 0; i < nc; ++i)
        if (!std::isfinite(h_in[i])) {
            err = "non-finite depth";
            return VSW_EINVAL;
        }

    // 2. internal order
    std::vector<int64_t> perm(nc);
    std::iota(perm.begin(), perm.end(), int64_t(0));
    if (ordering == VSW_ORDER_HILBERT || ordering == VSW_ORDER_BISECTION) {
        std::vector<double> cx(nc), cy(nc);
        double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
        for (int64_t k = 0; k < nc; ++k) {
            const int32_t* t = &tri[3 * k];
            cx[k] = (vx[t[0]] + vx[t[1]] + vx[t[2]]) / 3.0;
            cy[k] = (vy[t[0]] + vy[t[1]] + vy[t[2]]) / 3.0;
            x0 = std::min(x0, cx[k]); x1 = std::max(x1, cx[k]);
            y0 = std::min(y0, cy[k]); y1 = std::max(y1, cy[k]);
        }
        double span = std::max(x1 - x0, y1 - y0);
        double sc = span > 0 ? 65535.0 / span : 0.0;
        std::vector<uint64_t> key(nc);
        for (int64_t k = 0; k < nc; ++k) {
            uint32_t qx = uint32_t(std::min(65535.0, std::max(0.0, (cx[k] - x0) * sc)));
            uint32_t qy = uint32_t(std::min(65535.0, std::max(0.0, (cy[k] - y0) * sc)));
            key[k] = (hilbert16(qx, qy) << 32) | uint64_t(k);
        }
        if (ordering == VSW_ORDER_BISECTION && tile > 0) {
            bisect(perm, 0, nc, cx, cy, key, tile);
        } else {
            std::sort(key.begin(), key.end());
            for (int64_t i = 0; i < nc; ++i) perm[i] = int64_t(key[i] & 0xFFFFFFFFull);
        }
    } else if (ordering == VSW_ORDER_RANDOM) {
        uint64_t st = seed;
        for (int64_t i = nc - 1; i > 0; --i) {
            int64_t j = int64_t(splitmix64(st) % uint64_t(i + 1));
            std::swap(perm[i], perm[j]);
        }
    } else if (ordering != VSW_ORDER_NONE) {
        err = "unknown ordering";
        return VSW_EINVAL;
    }
    std::vector<int64_t> inv(nc);
    for (int64_t i = 0; i < nc; ++i) inv[perm[i]] = i;

    // 3. face matching: bucket directed faces by their smaller vertex, then
    //    pair equal larger vertices inside a bucket
    std::vector<int64_t> start(nv + 1, 0);
    for (int64_t k = 0; k < nc; ++k)
        for (int j = 0; j < 3; ++j) {
            int32_t a = tri[3 * k + j], b = tri[3 * k + (j + 1) % 3];
            start[std::min(a, b) + 1]++;
        }
    for (int64_t v = 0; v < nv; ++v) start[v + 1] += start[v];
    std::vector<int64_t> fill(start.begin(), start.end() - 1);
    std::vector<int64_t> slot(3 * nc);  // directed face id = 3k + j
    for (int64_t k = 0; k < nc; ++k)
        for (int j = 0; j < 3; ++j) {
            int32_t a = tri[3 * k + j], b = tri[3 * k + (j + 1) % 3];
            slot[fill[std::min(a, b)]++] = 3 * k + j;
        }
    std::vector<int64_t> mate(3 * nc, -1);
    int64_t ne = 0, nw = 0;
    for (int64_t v = 0; v < nv; ++v) {
        for (int64_t p = start[v]; p < start[v + 1]; ++p) {
            int64_t f = slot[p];
            if (mate[f] != -1) continue;
            int64_t k = f / 3;
            int j = int(f % 3);
            int32_t a = tri[3 * k + j], b = tri[3 * k + (j + 1) % 3];
            int32_t hi = std::max(a, b);
            int64_t found = -1;
            for (int64_t q = p + 1; q < start[v + 1]; ++q) {
                int64_t f2 = slot[q];
                int64_t k2 = f2 / 3;
                int j2 = int(f2 % 3);
                int32_t a2 = tri[3 * k2 + j2], b2 = tri[3 * k2 + (j2 + 1) % 3];
                if (std::max(a2, b2) != hi) continue;
                if (found != -1 || mate[f2] != -1) {
                    snprintf(buf, sizeof buf, "face of triangle %lld is shared by more than two triangles",
                             (long long)k);
                    err = buf;
                    return VSW_EMESH;
                }
                if (a2 == a) {
                    snprintf(buf, sizeof buf, "triangles %lld and %lld lie on the same side of a face",
                             (long long)k, (long long)k2);
                    err = buf;
                    return VSW_EMESH;
                }
                found = f2;
            }
            ++ne;
            if (found == -1) {
                mate[f] = -2;  // wall
                ++nw;
            } else {
                if (vx[a] == vx[b] && vy[a] == vy[b]) {
                    err = "duplicate vertex coordinates on a face";
                    return VSW_EMESH;
                }
                mate[f] = found;
                mate[found] = f;
            }
        }
    }

    // 4. packed neighbour slots in internal order; the canonical left side
    //    of an interior face is the cell that walks it from its
    //    lexicographically smaller (x, y) vertex
    out.nc = nc;
    out.nv = nv;
    out.ne = ne;
    out.nw = nw;
    out.nbr.assign(3 * nc, kWall);
    for (int64_t i = 0; i < nc; ++i) {
        int64_t k = perm[i];
        for (int j = 0; j < 3; ++j) {
            int64_t f = 3 * k + j;
            if (mate[f] < 0) continue;
            int64_t k2 = mate[f] / 3;
            int j2 = int(mate[f] % 3);
            int32_t a = tri[3 * k + j], b = tri[3 * k + (j + 1) % 3];
            bool left = (vx[a] < vx[b]) || (vx[a] == vx[b] && vy[a] < vy[b]);
            out.nbr[size_t(j) * nc + i] =
                (uint32_t(inv[k2]) << 3) | (left ? 4u : 0u) | uint32_t(j2);
        }
    }

    // 5. geometry in internal order
    out.face_geom.assign(size_t(G_NFACE) * 3 * nc, 0.0);
    out.area.assign(nc, 0.0);
    out.perim.assign(nc, 0.0);
    out.h.assign(nc, 0.0);
    auto G = [&](int field, int j, int64_t i) -> double& {
        return out.face_geom[(size_t(field) * 3 + j) * nc + i];
    };
    std::vector<double> ccx(nc), ccy(nc);
    for (int64_t i = 0; i < nc; ++i) {
        const int32_t* t = &tri[3 * perm[i]];
        double xa0 = vx[t[0]], xa1 = vx[t[1]], xa2 = vx[t[2]];
        double ya0 = vy[t[0]], ya1 = vy[t[1]], ya2 = vy[t[2]];
        double cr = (xa1 - xa0) * (ya2 - ya0) - (xa2 - xa0) * (ya1 - ya0);
        out.area[i] = 0.5 * cr;
        ccx[i] = ((xa0 + xa1) + xa2) / 3.0;
        ccy[i] = ((ya0 + ya1) + ya2) / 3.0;
        double l[3];
        for (int j = 0; j < 3; ++j) {
            double xs = vx[t[j]], ys = vy[t[j]];
            double xe = vx[t[(j + 1) % 3]], ye = vy[t[(j + 1) % 3]];
            double ex = xe - xs, ey = ye - ys;
            l[j] = std::sqrt(ex * ex + ey * ey);
            G(G_LEN, j, i) = l[j];
            G(G_NX, j, i) = ey / l[j];
            G(G_NY, j, i) = (-ex) / l[j];
            G(G_DX, j, i) = (xs + xe) * 0.5 - ccx[i];
            G(G_DY, j, i) = (ys + ye) * 0.5 - ccy[i];
        }
        out.perim[i] = (l[0] + l[1]) + l[2];
        out.h[i] = h_in[perm[i]];
    }
    // least-squares weights w_j = M^-1 delta_j, M = sum_j delta_j delta_j^T;
    // delta_j points to the neighbour centroid or to the wall ghost (the
    // centroid reflected in the wall face)
    for (int64_t i = 0; i < nc; ++i) {
        double ex[3], ey[3];
        for (int j = 0; j < 3; ++j) {
            uint32_t s = out.nbr[size_t(j) * nc + i];
            if (s != kWall) {
                int64_t n = int64_t(s >> 3);
                ex[j] = ccx[n] - ccx[i];
                ey[j] = ccy[n] - ccy[i];
            } else {
                double nx = G(G_NX, j, i), ny = G(G_NY, j, i);
                double dn = G(G_DX, j, i) * nx + G(G_DY, j, i) * ny;
                ex[j] = (2.0 * dn) * nx;
                ey[j] = (2.0 * dn) * ny;
            }
        }
        double sxx = (ex[0] * ex[0] + ex[1] * ex[1]) + ex[2] * ex[2];
        double sxy = (ex[0] * ey[0] + ex[1] * ey[1]) + ex[2] * ey[2];
        double syy = (ey[0] * ey[0] + ey[1] * ey[1]) + ey[2] * ey[2];
        double det = sxx * syy - sxy * sxy;
        for (int j = 0; j < 3; ++j) {
            G(G_WX, j, i) = (syy * ex[j] - sxy * ey[j]) / det;
            G(G_WY, j, i) = (sxx * ey[j] - sxy * ex[j]) / det;
        }
    }
    // vertices in the order the internal cells first use them
    std::vector<int64_t> vnew(nv, -1);
    int64_t nvu = 0;
    out.tri.assign(3 * size_t(nc), 0u);
    for (int64_t i = 0; i < nc; ++i)
        for (int j = 0; j < 3; ++j) {
            const int32_t v = tri[3 * perm[i] + j];
            if (vnew[v] < 0) vnew[v] = nvu++;
            out.tri[3 * size_t(i) + j] = uint32_t(vnew[v]);
        }
    out.vxy.assign(2 * size_t(nvu), 0.0);
    for (int64_t v = 0; v < nv; ++v)
        if (vnew[v] >= 0) {
            out.vxy[2 * size_t(vnew[v])] = vx[v];
            out.vxy[2 * size_t(vnew[v]) + 1] = vy[v];
        }
    out.perm = std::move(perm);
    return VSW_OK;
}

void build_face_tiles(const HostMesh& hm, int tile, FaceTilesHost& out) {
    const int64_t nc = hm.nc;
    out.tile = tile;
    out.ntiles = int((nc + tile - 1) / tile);
    out.topo.assign(size_t(nc), TopoRec{{kWall, kWall, kWall}, {0u, 0u, 0u}});
    out.bstart.assign(size_t(out.ntiles) + 1, 0);
    out.fstart.assign(size_t(out.ntiles) + 1, 0);
    out.bitem.clear();
    out.items.clear();
    out.bmax = 0;
    out.fmax = 0;
    for (int64_t i = 0; i < nc; ++i)
        for (int j = 0; j < 3; ++j) {
            const uint32_t s = hm.nbr[size_t(j) * nc + i];
            out.topo[i].n[j] = (s == kWall) ? kWall : (s & ~7u);
            out.topo[i].v[j] = hm.tri[3 * size_t(i) + j];
        }
    for (int t = 0; t < out.ntiles; ++t) {
        const int64_t c0 = int64_t(t) * tile, c1 = std::min(nc, c0 + tile);
        out.bstart[t] = int32_t(out.bitem.size());
        out.fstart[t] = int32_t(out.items.size());
        int nb = 0;
        for (int64_t i = c0; i < c1; ++i) {
            if (hm.perm[i] < 0) continue;  // padding of an ensemble scenario
            const uint32_t* v = &hm.tri[3 * size_t(i)];
            for (int j = 0; j < 3; ++j) {
                const uint32_t s = hm.nbr[size_t(j) * nc + i];
                const uint32_t va = v[j], vb = v[(j + 1) % 3];
                const uint16_t own = uint16_t(j * tile + (i - c0));
                if (s == kWall) {
                    out.items.push_back(FaceItem{va, vb, own, kSlotWall});
                    continue;
                }
                const int64_t n = int64_t(s >> 3);
                const uint32_t jn = s & 3u;
                const bool left = (s & 4u) != 0;
                if (n >= c0 && n < c1) {
                    // inside the tile: listed once, by the left cell
                    if (left)
                        out.items.push_back(
                            FaceItem{va, vb, own, uint16_t(jn * tile + (n - c0))});
                } else {
                    const uint16_t halo = uint16_t(3 * tile + nb++);
                    out.bitem.push_back((uint32_t(n) << 2) | jn);
                    out.items.push_back(left ? FaceItem{va, vb, own, halo}
                                             : FaceItem{vb, va, halo, own});
                }
            }
        }
        out.bmax = std::max(out.bmax, nb);
        out.fmax = std::max(out.fmax, int(out.items.size()) - out.fstart[t]);
    }
    out.bstart[out.ntiles] = int32_t(out.bitem.size());
    out.fstart[out.ntiles] = int32_t(out.items.size());
}

void build_tiles(const HostMesh& hm, int tile, TileMapHost& out) {
    const int64_t nc = hm.nc;
    out.tile = tile;
    out.ntiles = int((nc + tile - 1) / tile);
    out.nloc.assign(3 * size_t(nc), kNlocWall);
    out.bstart.assign(size_t(out.ntiles) + 1, 0);
    out.bitem.clear();
    out.bmax = 0;
    for (int t = 0; t < out.ntiles; ++t) {
        const int64_t c0 = int64_t(t) * tile, c1 = std::min(nc, c0 + tile);
        out.bstart[t] = int32_t(out.bitem.size());
        int nb = 0;
        for (int64_t i = c0; i < c1; ++i)
            for (int j = 0; j < 3; ++j) {
                const uint32_t s = hm.nbr[size_t(j) * nc + i];
                if (s == kWall) continue;
                const int64_t n = int64_t(s >> 3);
                const uint32_t jn = s & 3u;
                uint32_t slot;
                if (n >= c0 && n < c1) {
                    slot = jn * uint32_t(tile) + uint32_t(n - c0);
                } else {
                    slot = 3u * uint32_t(tile) + uint32_t(nb++);
                    out.bitem.push_back((uint32_t(n) << 2) | jn);
                }
                out.nloc[size_t(j) * nc + i] = uint16_t(slot | ((s & 4u) ? 0x8000u : 0u));
            }
        out.bmax = std::max(out.bmax, nb);
    }
    out.bstart[out.ntiles] = int32_t(out.bitem.size());
}

int build_ensemble(int nseg, const int64_t* nv, const double* vx, const double* vy,
                   const int64_t* nc, const int32_t* tri, const double* h, int ordering,
                   uint64_t seed, int tile, EnsembleMesh& out, std::string& err) {
    if (nseg <= 0 || !nv || !nc) {
        err = "empty ensemble or NULL count array";
        return VSW_EINVAL;
    }
    out = EnsembleMesh();
    out.nseg = nseg;
    out.off.assign(size_t(nseg) + 1, 0);
    out.coff.assign(size_t(nseg) + 1, 0);
    for (int s = 0; s < nseg; ++s) {
        if (nc[s] <= 0 || nv[s] <= 0 || nc[s] > kMaxCells) {
            err = "scenario " + std::to_string(s) + ": empty or oversized mesh";
            return VSW_EINVAL;
        }
        out.coff[s + 1] = out.coff[s] + nc[s];
        out.off[s + 1] = out.off[s] + (nc[s] + tile - 1) / tile * tile;
        if (out.off[s + 1] > kMaxCells) {
            err = "ensemble too large for 29-bit cell indices";
            return VSW_EINVAL;
        }
    }
    out.ncell = out.coff[nseg];
    const int64_t N = out.off[nseg];
    const int ntiles = int(N / tile);
    HostMesh& hm = out.hm;
    TileMapHost& tm = out.tiles;
    if (tile != 128 && tile != 256 && tile != 512) {
        err = "tile size must be 128, 256 or 512";
        return VSW_EINVAL;
    }
    if (nseg == 1) {  // one mesh: no copy
        int rc = build_host_mesh(nv[0], vx, vy, nc[0], tri, h, ordering, seed, tile, hm, err);
        if (rc) return rc;
        if (tile == 256) build_tiles(hm, tile, tm);
    } else {
        hm.nc = N;
        hm.perm.assign(size_t(N), -1);
        hm.nbr.assign(3 * size_t(N), kWall);
        hm.face_geom.assign(size_t(G_NFACE) * 3 * size_t(N), 0.0);
        hm.area.assign(size_t(N), 0.0);
        hm.perim.assign(size_t(N), 0.0);
        hm.h.assign(size_t(N), 0.0);
        hm.tri.assign(3 * size_t(N), 0u);
        hm.vxy.clear();
        tm.tile = tile;
        tm.ntiles = ntiles;
        tm.nloc.assign(3 * size_t(N), kNlocWall);
        tm.bstart.assign(size_t(ntiles) + 1, 0);
        tm.bmax = 0;
        int64_t vo = 0;
        for (int s = 0; s < nseg; ++s) {
            HostMesh p;
            int rc = build_host_mesh(nv[s], vx + vo, vy + vo, nc[s], tri + 3 * out.coff[s],
                                     h + out.coff[s], ordering, seed + uint64_t(s), tile, p,
                                     err);
            if (rc) {
                err = "scenario " + std::to_string(s) + ": " + err;
                return rc;
            }
            TileMapHost pt;
            if (tile == 256) build_tiles(p, tile, pt);
            vo += nv[s];
            const int64_t o = out.off[s], n = p.nc;
            const uint32_t v0 = uint32_t(hm.vxy.size() / 2);
            hm.vxy.insert(hm.vxy.end(), p.vxy.begin(), p.vxy.end());
            for (int64_t i = 0; i < 3 * n; ++i) hm.tri[3 * size_t(o) + i] = p.tri[i] + v0;
            hm.ne += p.ne;
            hm.nw += p.nw;
            hm.nv += p.nv;
            for (int64_t i = 0; i < n; ++i) {
                hm.perm[o + i] = out.coff[s] + p.perm[i];
                hm.area[o + i] = p.area[i];
                hm.perim[o + i] = p.perim[i];
                hm.h[o + i] = p.h[i];
                for (int j = 0; j < 3; ++j) {
                    const uint32_t sl = p.nbr[size_t(j) * n + i];
                    hm.nbr[size_t(j) * N + o + i] =
                        sl == kWall ? kWall : (uint32_t((sl >> 3) + o) << 3) | (sl & 7u);
                    if (tile == 256) tm.nloc[size_t(j) * N + o + i] = pt.nloc[size_t(j) * n + i];
                    for (int f = 0; f < G_NFACE; ++f)
                        hm.face_geom[(size_t(f) * 3 + j) * N + o + i] =
                            p.face_geom[(size_t(f) * 3 + j) * n + i];
                }
            }
            if (tile == 256) {
                const int t0 = int(o / tile);
                const int32_t b0 = int32_t(tm.bitem.size());
                for (int t = 0; t < pt.ntiles; ++t) tm.bstart[t0 + t] = b0 + pt.bstart[t];
                for (uint32_t it : pt.bitem)
                    tm.bitem.push_back((uint32_t((it >> 2) + o) << 2) | (it & 3u));
                tm.bmax = std::max(tm.bmax, pt.bmax);
            }
            // padding tiles cannot occur: each scenario's tiles end at off[s + 1]
        }
        if (tile == 256)
            tm.bstart[ntiles] = int32_t(tm.bitem.size());
        else
            tm = TileMapHost();
    }
    // padding cells: no neighbours, their own three (first) vertices, never read
    build_face_tiles(hm, tile, out.ftiles);
    out.tinfo.assign(size_t(ntiles), 0u);
    for (int s = 0; s < nseg; ++s) {
        const int t0 = int(out.off[s] / tile), t1 = int(out.off[s + 1] / tile);
        const int64_t cend = out.off[s] + nc[s];
        for (int t = t0; t < t1; ++t) {
            const int64_t c0 = int64_t(t) * tile;
            const int cnt = int(std::min<int64_t>(tile, cend - c0));
            out.tinfo[t] = (uint32_t(s) << 10) | (t == t0 ? 0x200u : 0u) | uint32_t(cnt - 1);
        }
    }
    return VSW_OK;
}

}  // namespace vsw
