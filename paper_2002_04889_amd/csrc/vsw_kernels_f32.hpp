// Declarations of the mixed-precision (FP32) stage kernels.
#pragma once
#include "vsw_kernels.hpp"

namespace vsw {

// FP32 state record: still-water depth h (FP64, static) and the prognostic
// free surface eta = H - h and momentum (Hu, Hv) in FP32; 24 bytes.
struct alignas(8) CellF {
    double h;
    float eta, hu, hv, pad;
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

template <int STAGE>
__global__ void stage_f32_kernel(DevMesh m, TileMap tm, CellF* W, CellF* W1, StepParams p, Ctrl* c,
                                 Seg* sg, int slot, int step_arg, double* log);
__global__ void dt_init_f32_kernel(DevMesh m, TileMap tm, const CellF* W, double g, double thr,
                                   Seg* sg);
__global__ void gauge_f32_kernel(const CellF* W, const int64_t* cells, int ng,
                                 const uint32_t* tinfo, const Seg* sg, const Ctrl* c, int step_arg,
                                 double* log);
__global__ void pack_state_f32_kernel(int64_t n, const int64_t* perm, const double* H,
                                      const double* HU, const double* HV, const double* h,
                                      CellF* W, CellF* W1);
__global__ void unpack_state_f32_kernel(int64_t n, const int64_t* perm, const CellF* W, double* H,
                                        double* HU, double* HV);

}  // namespace vsw
