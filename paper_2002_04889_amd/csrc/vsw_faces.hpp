// Face-parallel stage kernels: one workgroup per tile of T cells (T = 128,
// 256 or 512, one thread per cell), geometry computed from the vertex
// coordinates, every face of the tile evaluated once.
#pragma once
#include "vsw_kernels.hpp"

namespace vsw {

// Per cell: the neighbour across each face (its index shifted left by 3,
// kWallSlot on a wall) and the vertices in local counter-clockwise order
// (face j joins local vertices j and j + 1); 24 bytes.
struct alignas(8) TopoD {
    uint32_t n0, n1, n2, v0, v1, v2;
};

// One face of a tile: vertices a -> b as the canonical left cell walks it,
// LDS slots of its left and right face states (sr = kFaceWall on a wall).
struct FaceItemD {
    uint32_t va, vb;
    uint16_t sl, sr;
};
constexpr uint16_t kFaceWall = 0xFFFFu;

// Least-squares weights (w_x, w_y) of stencil members 0..2; 48 bytes, and
// the same rounded to FP32 for the mixed-precision kernel (24 bytes).
struct alignas(16) LsqW {
    double w[6];
};
struct alignas(8) LsqWF {
    float w[6];
};

struct FaceMesh {
    int64_t nc;
    const TopoD* __restrict__ topo;    // [nc]
    const LsqW* __restrict__ lsq;      // [nc] FP64 solvers
    const LsqWF* __restrict__ lsqf;    // [nc] FP32 solvers
    const double2* __restrict__ vxy;   // [vertices]
    const double* __restrict__ perim;  // [nc]
};

struct FaceTileMap {
    const int32_t* __restrict__ bstart;  // [ntiles + 1] halo faces of each tile
    const uint32_t* __restrict__ bitem;  // (cell << 2) | face of the halo cell
    const int32_t* __restrict__ fstart;  // [ntiles + 1] faces each tile evaluates
    const FaceItemD* __restrict__ items;
    const uint32_t* __restrict__ tinfo;  // [ntiles] tile words
    int bmax;                            // most halo faces of any tile
    int ntiles;
    int nseg;
    int xcd_order;
};

// LDS of the FP64 face-parallel kernel: five planes of 3 T + bmax face
// slots (the face state eta, h, H, u, v, then the face's terms for the
// cell) and the depth H and bed depth h of the T cells.
inline size_t faces_lds_bytes(int tile, int bmax) {
    return sizeof(double) * (5 * size_t(3 * tile + bmax) + 2 * size_t(tile));
}

// Same contract as stage_kernel (state buffers Wa, Wb by the step parity,
// w1 in W1, control and log), for tiles of T cells.
template <int T, int STAGE>
__global__ void faces_stage_kernel(FaceMesh m, FaceTileMap tm, Cell4* Wa, Cell4* Wb, Cell4* W1,
                                   StepParams p, Ctrl* c, Seg* sg, int slot, int step_arg,
                                   double* log);

// faces_stage_kernel with a tape (same arithmetic and results, the tape of
// stage_tape_kernel): reads w^n from W and writes w^{n+1} to Wout (control
// par and step index 0).
template <int T, int STAGE>
__global__ void faces_tape_kernel(FaceMesh m, FaceTileMap tm, Cell4* W, Cell4* Wout, Cell4* W1,
                                  StepParams p, Ctrl* c, Seg* sg, int slot, int step_arg,
                                  double* log, Tape tp);

// CFL minimum of the incoming state for tiles of T cells.
template <int T>
__global__ void faces_dt_init_kernel(FaceMesh m, FaceTileMap tm, const Cell4* W, const double* area,
                                     double g, double thr, Seg* sg);

}  // namespace vsw
