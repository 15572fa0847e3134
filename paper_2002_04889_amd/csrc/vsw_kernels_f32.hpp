// Declarations of the mixed-precision (FP32) stage kernels.
#pragma once
#include "vsw_kernels.hpp"

namespace vsw {

// FP32 state record: the prognostic free surface eta = H - h and momentum
// (Hu, Hv) in FP32; 12 bytes.  The still-water depth h (FP64, static) is a
// separate array, read once per cell and stage.
struct CellF {
    float eta, hu, hv;
};

// Face state of the FP32 kernel: eta, u, v in FP32, bed and total depth in
// FP64.
struct FaceF {
    float eta, u, v;
    double h, H;
};

// LDS of the FP32 stage kernel: 2 FP64 and 3 FP32 planes of
// (3 * kTile + bmax) face slots.
inline size_t stage_f32_lds_bytes(int bmax) {
    return (2 * sizeof(double) + 3 * sizeof(float)) * size_t(3 * kTile + bmax);
}

// Same buffer convention as stage_kernel (w^n in buffer (par + step) & 1).
// What the discrete adjoint records while an FP32 run replays a checkpoint
// segment: the stage's residual R (3 per cell, FP64), the mask of its
// post-stage fix (bit 0: depth not clamped, bit 1: momentum kept), the state
// the stage reconstructs converted to FP64 records (H = eta + h), and in
// stage 2 the bits of the CFL minimum of w^{n+1} into *rmin (pre-set to
// +inf) instead of the scenario's record.
struct TapeF {
    double* __restrict__ R;
    uint8_t* __restrict__ mask;
    unsigned long long* rmin;
    Cell4* __restrict__ win;
};

// The still-water depth is m.hcell[k].
template <int STAGE>
__global__ void stage_f32_kernel(DevMesh m, TileMap tm, CellF* Wa, CellF* Wb, CellF* W1,
                                 StepParams p, Ctrl* c, Seg* sg, int slot, int step_arg,
                                 double* log);
// stage_f32_kernel with a tape (same arithmetic and results): reads w^n
// from W and writes w^{n+1} to Wout (control par and step index 0).
template <int STAGE>
__global__ void stage_f32_tape_kernel(DevMesh m, TileMap tm, CellF* W, CellF* Wout, CellF* W1,
                                      StepParams p, Ctrl* c, Seg* sg, int slot, int step_arg,
                                      double* log, TapeF tp);
__global__ void dt_init_f32_kernel(DevMesh m, TileMap tm, const CellF* W, double g, double thr,
                                   Seg* sg);
__global__ void gauge_f32_kernel(const CellF* Wa, const CellF* Wb, const double* h,
                                 const int64_t* cells, int ng, const int32_t* gseg,
                                 const Seg* sg, const Ctrl* c, int step_arg, double* log);
__global__ void pack_state_f32_kernel(int64_t n, const int64_t* perm, const double* H,
                                      const double* HU, const double* HV, const double* h,
                                      CellF* W, CellF* W1);
__global__ void unpack_state_f32_kernel(int64_t n, const int64_t* perm, const CellF* W,
                                        const double* h, double* H, double* HU, double* HV);

// Face-parallel FP32 kernels (same arithmetic as stage_f32_kernel, the
// geometry from the vertices as in faces_stage_kernel); LDS as
// faces_lds_bytes.
struct FaceMesh;
struct FaceTileMap;
template <int T, int STAGE>
__global__ void faces_stage_f32_kernel(FaceMesh m, FaceTileMap tm, const double* h, CellF* Wa,
                                       CellF* Wb, CellF* W1, StepParams p, Ctrl* c, Seg* sg,
                                       int slot, int step_arg, double* log);
// faces_stage_f32_kernel recording the tape of stage_f32_tape_kernel.
template <int T, int STAGE>
__global__ void faces_tape_f32_kernel(FaceMesh m, FaceTileMap tm, const double* h, CellF* W,
                                      CellF* Wout, CellF* W1, StepParams p, Ctrl* c, Seg* sg,
                                      int slot, int step_arg, double* log, TapeF tp);
template <int T>
__global__ void faces_dt_init_f32_kernel(FaceMesh m, FaceTileMap tm, const CellF* W,
                                         const double* h, const double* area, double g,
                                         double thr, Seg* sg);

}  // namespace vsw
