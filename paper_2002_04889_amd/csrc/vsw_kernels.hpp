// Shared declarations of the stage kernels and their launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "vsw_device.hpp"

namespace vsw {

constexpr int kBlock = 256;  // threads per block (four wave64)

// The solver holds one or more independent scenarios (an ensemble), each a
// mesh of its own whose cells occupy a contiguous run of whole tiles.  Each
// scenario has its own control record (one 64-byte line): the step using
// slot s reads rmin[s] and t[s] and writes the next step's values into
// slot s ^ 1, so a scenario's dt never waits for the host.
struct Seg {
    unsigned long long rmin[2];  // bits of min_K |K| / (P_K (|u| + c)) of the scenario
    double t[2];                 // time at the start of the step
    double dt_last;
    long long steps_done;        // steps the scenario took in this call
    long long pad[2];
};

// Control word of one call, shared by all scenarios.
struct Ctrl {
    unsigned long long clamps;   // negative depths set to zero in this call
    int err;                     // bit 0: non-finite state, bit 1: no valid dt
    int err_step;                // first failing step of the call
    int kbase;                   // step index = kbase + the kernel's step argument
    int pad;
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

// Tile word: bits 0-7 the tile's cell count minus one, bit 8 set on the
// first tile of a scenario, bits 9-31 the scenario index.
struct TileMap {
    const uint16_t* __restrict__ nloc;   // [3][nc] LDS slot per face, bit 15 = left
    const int32_t* __restrict__ bstart;  // [ntiles + 1]
    const uint32_t* __restrict__ bitem;  // halo faces: (cell << 2) | face
    const uint32_t* __restrict__ tinfo;  // [ntiles] tile words
    int bmax;                            // most boundary faces of any tile
    int ntiles;
    int nseg;                            // scenarios
    int xcd_order;                       // 1: deal contiguous tile runs to the XCDs
};

// Fused stage kernel.  STAGE 1: w1 = w + dt R(w).  STAGE 2:
// w^{n+1} = w/2 + (w1 + dt R(w1))/2 in place, plus the next CFL minimum and
// the time bookkeeping.  Dynamic LDS: stage_lds_bytes(bmax).
// Step k of the call is kbase + step_arg (kbase advances on the device, so a
// captured pair of steps can be replayed).  Log: log[2 (k nseg + scenario)]
// = time after the step, log[2 (k nseg + scenario) + 1] = its dt.
template <int STAGE>
__global__ void stage_kernel(DevMesh m, TileMap tm, Cell4* W, Cell4* W1, StepParams p, Ctrl* c,
                             Seg* sg, int slot, int step_arg, double* log);

// LDS of the fused stage kernel: four doubles (eta, h, u, v) per face slot.
inline size_t stage_lds_bytes(int bmax) { return sizeof(double) * 4 * size_t(3 * kTile + bmax); }

// What the discrete adjoint records of a stage while it replays a checkpoint
// segment: the stage's residual R (3 per cell) and the mask of its
// post-stage fix (bit 0: depth not clamped, bit 1: momentum kept); stage 2
// writes w^{n+1} to wout (w^n is kept) and the bits of the CFL minimum of
// w^{n+1} to *rmin (pre-set to +inf) instead of the scenario's record.
struct Tape {
    double* __restrict__ R;
    uint8_t* __restrict__ mask;
    Cell4* __restrict__ wout;
    unsigned long long* rmin;
};

// The fused stage kernel with a tape: the same arithmetic and results.
template <int STAGE>
__global__ void stage_tape_kernel(DevMesh m, TileMap tm, Cell4* W, Cell4* W1, StepParams p,
                                  Ctrl* c, Seg* sg, int slot, int step_arg, double* log, Tape tp);

// Start of a call: every scenario's time from t0[s], minima cleared.
__global__ void ctrl_init_kernel(Ctrl* c, Seg* sg, int nseg, const double* t0);
// CFL minimum of the incoming state, one block per tile.
__global__ void dt_init_kernel(DevMesh m, TileMap tm, const Cell4* W, double g, double thr,
                               Seg* sg);
__global__ void recon_kernel(DevMesh m, TileMap tm, const Cell4* W, FaceBuf fb, StepParams p,
                             const Ctrl* c, const Seg* sg, int slot);
__global__ void update1_kernel(DevMesh m, TileMap tm, const Cell4* W, Cell4* W1, FaceBuf fb,
                               StepParams p, Ctrl* c, Seg* sg, int slot);
__global__ void update2_kernel(DevMesh m, TileMap tm, Cell4* W, const Cell4* W1, FaceBuf fb,
                               StepParams p, Ctrl* c, Seg* sg, int slot, int step_arg,
                               double* log);
__global__ void gauge_kernel(const Cell4* W, const int64_t* cells, int ng, const uint32_t* tinfo,
                             const Seg* sg, const Ctrl* c, int step_arg, double* log);
// Advance the step base by `by` steps (the last node of a captured pair).
__global__ void step_bump_kernel(Ctrl* c, int by);
// perm[i] = caller index of internal cell i, or -1 for the padding cells
// that round each scenario up to whole tiles (left untouched).
__global__ void pack_state_kernel(int64_t n, const int64_t* perm, const double* H,
                                  const double* HU, const double* HV, const double* h, Cell4* W,
                                  Cell4* W1);
__global__ void unpack_state_kernel(int64_t n, const int64_t* perm, const Cell4* W, double* H,
                                    double* HU, double* HV);

}  // namespace vsw
