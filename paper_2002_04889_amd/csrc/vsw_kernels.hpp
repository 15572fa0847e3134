// Shared declarations of the stage kernels and their launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "vsw_device.hpp"

namespace vsw {

constexpr int kBlock = 256;  // threads per block (four wave64)

// The CFL minimum of a step is reduced into kMinGroups partial minima, each
// on its own 128-byte line (block b uses group b % kMinGroups, which follows
// the round-robin dealing of workgroups to XCDs), so the blocks' atomics do
// not all queue on one address.  The step's minimum is the min of the groups.
constexpr int kMinGroups = 8;
constexpr int kMinStride = 16;  // 16 x 8 bytes = one 128-byte line per group

// Device control block: per-step time and CFL minimum in two slots (the
// step using slot s writes the next step's values into slot s ^ 1).
struct Ctrl {
    unsigned long long rmin[2][kMinGroups * kMinStride];  // bits of min_K |K| / (P_K (|u| + c))
    double t[2];                 // time at the start of the step
    double dt_last;
    unsigned long long clamps;   // negative depths set to zero in this call
    long long steps_done;
    int err;                     // 0 ok, 1 non-finite state, 2 no valid dt
    int err_step;                // first failing step of the call
};

struct StepParams {
    double g, hg, thr, cfl, dt_fixed, t_stop;
};

// Face buffer of one stage: per face j and cell k the face state
// (eta, h, H, u, v) at f[(5 j + c) nc + k]; the centred bed source at
// sc[k], sc[nc + k]; the reconstruction order (1 or 2) at order[k].
struct FaceBuf {
    double* __restrict__ f;
    double* __restrict__ sc;
    int32_t* __restrict__ order;
};

constexpr int kTile = 256;   // cells per tile of the fused stage kernel (= kBlock)
constexpr uint16_t kNlocWall16 = 0xFFFFu;

struct TileMap {
    const uint16_t* __restrict__ nloc;   // [3][nc] LDS slot per face, bit 15 = left
    const int32_t* __restrict__ bstart;  // [ntiles + 1]
    const uint32_t* __restrict__ bitem;  // halo faces: (cell << 2) | face
    int bmax;                            // most boundary faces of any tile
    int ntiles;
};

// Fused stage kernel.  STAGE 1: w1 = w + dt R(w).  STAGE 2:
// w^{n+1} = w/2 + (w1 + dt R(w1))/2 in place, plus the next CFL minimum and
// the time bookkeeping.  Dynamic LDS: 5 * (3 * kTile + bmax) doubles.
template <int STAGE>
__global__ void stage_kernel(DevMesh m, TileMap tm, Cell4* W, Cell4* W1, StepParams p, Ctrl* c,
                             int slot, int step, double* tlog, double* dtlog);

inline size_t stage_lds_bytes(int bmax) { return sizeof(double) * 5 * size_t(3 * kTile + bmax); }

__global__ void ctrl_init_kernel(Ctrl* c, double t0);
__global__ void dt_init_kernel(DevMesh m, const Cell4* W, double g, double thr, Ctrl* c);
__global__ void recon_kernel(DevMesh m, const Cell4* W, FaceBuf fb, StepParams p, const Ctrl* c,
                             int slot);
__global__ void update1_kernel(DevMesh m, const Cell4* W, Cell4* W1, FaceBuf fb, StepParams p,
                               Ctrl* c, int slot);
__global__ void update2_kernel(DevMesh m, Cell4* W, const Cell4* W1, FaceBuf fb, StepParams p,
                               Ctrl* c, int slot, int step, double* tlog, double* dtlog);
__global__ void gauge_kernel(const Cell4* W, const int64_t* cells, int ng, const Ctrl* c, int step,
                             double* log);
__global__ void pack_state_kernel(int64_t n, const int64_t* perm, const double* H,
                                  const double* HU, const double* HV, const double* h, Cell4* W,
                                  Cell4* W1);
__global__ void unpack_state_kernel(int64_t n, const int64_t* perm, const Cell4* W, double* H,
                                    double* HU, double* HV);

}  // namespace vsw
