// Host-side mesh preparation for the GPU solver: orientation, face
// matching, canonical face orientation, internal cell order and geometry.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace vsw {

// Neighbour slot encoding (uint32 per cell face):
//   wall face      : kWall
//   interior face  : (neighbour << 3) | (is_left << 2) | neighbour_face
// where is_left says whether this cell is the canonical left side of the
// face and neighbour_face is the face's local index inside the neighbour.
constexpr uint32_t kWall = 0xFFFFFFFFu;
constexpr int64_t kMaxCells = (int64_t(1) << 29) - 1;

// Geometry fields, each stored as [face j][cell] (3 * nc doubles) or [cell].
enum GeomField : int {
    G_NX = 0,   // outward unit normal x of face j
    G_NY,       // outward unit normal y
    G_LEN,      // face length
    G_DX,       // face midpoint minus centroid, x
    G_DY,       // face midpoint minus centroid, y
    G_WX,       // least-squares weight x of stencil member j
    G_WY,       // least-squares weight y
    G_NFACE     // number of per-face fields
};

struct HostMesh {
    int64_t nc = 0, nv = 0, ne = 0, nw = 0;
    std::vector<int64_t> perm;      // internal cell i -> caller's cell perm[i]
    std::vector<uint32_t> nbr;      // [3][nc] packed neighbour slots
    std::vector<double> face_geom;  // [G_NFACE][3][nc]
    std::vector<double> area;       // [nc]
    std::vector<double> perim;      // [nc]
    std::vector<double> h;          // [nc] still-water depth
    // Vertices renumbered in the order the internal cells first use them
    // (so a tile's vertices lie together); unused vertices dropped.
    std::vector<uint32_t> tri;      // [nc][3] counter-clockwise, caller's first vertex first
    std::vector<double> vxy;        // [nvu][2] coordinates
};

// Face-parallel stage kernels.  Per cell: the neighbour across each face
// (its internal index shifted left by 3, kWall on a wall) and the vertices
// in local order (face j joins local vertices j and j + 1).  Per tile of `tile` cells: the halo faces to
// reconstruct (as in TileMapHost) and the list of the faces the tile
// evaluates, each once, in canonical orientation: vertices a -> b as the
// canonical left cell walks the face, and the LDS slots of the left and
// right face states (slot convention of TileMapHost; sr = kSlotWall on a
// wall).  An interior face inside the tile is listed once, a face to a
// halo cell once per tile that owns one of its cells.
struct TopoRec {
    uint32_t n[3];
    uint32_t v[3];
};
struct FaceItem {
    uint32_t va, vb;
    uint16_t sl, sr;
};
constexpr uint16_t kSlotWall = 0xFFFFu;

struct FaceTilesHost {
    int tile = 0, ntiles = 0, bmax = 0, fmax = 0;
    std::vector<TopoRec> topo;      // [nc]
    std::vector<int32_t> bstart;    // [ntiles + 1]
    std::vector<uint32_t> bitem;    // halo faces: (cell << 2) | face
    std::vector<int32_t> fstart;    // [ntiles + 1]
    std::vector<FaceItem> items;
};

void build_face_tiles(const HostMesh& hm, int tile, FaceTilesHost& out);

// Tiles of the fused stage kernel: tile t owns internal cells
// [t * tile, (t + 1) * tile).  Every face of an owned cell gets an LDS slot:
//   owned neighbour n with face jn : jn * tile + (n - t * tile)
//   neighbour outside the tile     : 3 * tile + b, b-th boundary face of t
// nloc[j][k] = slot | 0x8000 if cell k is the canonical left side; a wall is
// kNlocWall.  bitem[bstart[t] + b] = (neighbour << 2) | face of the
// neighbour, i.e. the halo face to reconstruct into boundary slot b.
constexpr uint16_t kNlocWall = 0xFFFFu;

struct TileMapHost {
    int tile = 0, ntiles = 0, bmax = 0;
    std::vector<uint16_t> nloc;     // [3][nc]
    std::vector<int32_t> bstart;    // [ntiles + 1]
    std::vector<uint32_t> bitem;    // [bstart[ntiles]]
};

void build_tiles(const HostMesh& hm, int tile, TileMapHost& out);

// Several independent meshes (an ensemble of scenarios) in one internal
// numbering: scenario s owns the internal cells [off[s], off[s] + nc_s),
// with off[s] a multiple of the tile size, so no tile spans two scenarios;
// the cells between one scenario's end and the next tile are padding
// (perm = -1, never read).  The caller numbers cells by concatenating the
// scenarios: caller index coff[s] + k for cell k of scenario s.
struct EnsembleMesh {
    int nseg = 0;
    int64_t ncell = 0;              // caller cells, sum of nc_s
    std::vector<int64_t> off;       // [nseg + 1] internal offsets; off[nseg] = internal count
    std::vector<int64_t> coff;      // [nseg + 1] caller offsets
    HostMesh hm;                    // over all internal cells; perm = caller index or -1
    TileMapHost tiles;              // tile map of the cell-parallel kernels (tile 256)
    FaceTilesHost ftiles;           // face lists of the face-parallel kernels
    std::vector<uint32_t> tinfo;    // [ntiles] (scenario << 10) | (first << 9) | (cells - 1)
};

// nv[s], nc[s]: vertex and cell counts of scenario s; vx, vy, tri, h hold
// the scenarios' arrays one after the other, tri indexing the scenario's own
// vertices.  Scenario s is renumbered with seed + s.  Scenarios start on
// whole tiles of `tile` cells (a multiple of 256, or 128); the cell-parallel
// tile map is built when tile is 256.
int build_ensemble(int nseg, const int64_t* nv, const double* vx, const double* vy,
                   const int64_t* nc, const int32_t* tri, const double* h, int ordering,
                   uint64_t seed, int tile, EnsembleMesh& out, std::string& err);

// Returns 0 or a VSW_E* code with a message in err.  tile: the tile size the
// bisection ordering cuts the mesh into.
int build_host_mesh(int64_t nv, const double* vx, const double* vy, int64_t nc,
                    const int32_t* tri, const double* h, int ordering, uint64_t seed,
                    int tile, HostMesh& out, std::string& err);

}  // namespace vsw
