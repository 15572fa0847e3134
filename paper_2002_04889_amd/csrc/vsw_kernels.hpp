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
    int par;                     // state buffer (0 or 1) that holds the call's first state
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

// Tile word: bits 0-8 the tile's cell count minus one, bit 9 set on the
// first tile of a scenario, bits 10-31 the scenario index.
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

// The state lives in two buffers Wa, Wb: step k of a call reads w^n from
// buffer (par + k) & 1 and writes w^{n+1} to the other one, so the input of
// a step is never overwritten by it.  A scenario that has reached t_stop
// copies its cells across instead; a step that fails leaves its input in
// place (the solver's state after VSW_EUNSTABLE).
//
// Fused stage kernel.  STAGE 1: w1 = w + dt R(w).  STAGE 2:
// w^{n+1} = w/2 + (w1 + dt R(w1))/2, plus the next CFL minimum and the time
// bookkeeping.  Dynamic LDS: stage_lds_bytes(bmax).
// Step k of the call is kbase + step_arg (kbase advances on the device, so a
// captured pair of steps can be replayed).  Log: log[2 (k nseg + scenario)]
// = time after the step, log[2 (k nseg + scenario) + 1] = its dt.
template <int STAGE>
__global__ void stage_kernel(DevMesh m, TileMap tm, Cell4* Wa, Cell4* Wb, Cell4* W1, StepParams p,
                             Ctrl* c, Seg* sg, int slot, int step_arg, double* log);

// LDS of the fused stage kernel: four doubles (eta, h, u, v) per face slot.
inline size_t stage_lds_bytes(int bmax) { return sizeof(double) * 4 * size_t(3 * kTile + bmax); }

// What the discrete adjoint records of a stage while it replays a checkpoint
// segment: the stage's residual R (3 per cell) and the mask of its
// post-stage fix (bit 0: depth not clamped, bit 1: momentum kept); stage 2
// writes the bits of the CFL minimum of w^{n+1} to *rmin (pre-set to +inf)
// instead of the scenario's record.
struct Tape {
    double* __restrict__ R;
    uint8_t* __restrict__ mask;
    unsigned long long* rmin;
};

// The fused stage kernel with a tape: the same arithmetic and results.  It
// reads w^n from W and writes w^{n+1} to Wout (the control block's par and
// step index are 0).
template <int STAGE>
__global__ void stage_tape_kernel(DevMesh m, TileMap tm, Cell4* W, Cell4* Wout, Cell4* W1,
                                  StepParams p, Ctrl* c, Seg* sg, int slot, int step_arg,
                                  double* log, Tape tp);

// Start of a call: every scenario's time from t0[s], minima cleared; par is
// the state buffer holding the call's first state.  keep >= 0: the CFL
// minimum of that state is already in slot `keep` of every scenario's record
// (the previous call's last step computed it) and moves to slot 0.
__global__ void ctrl_init_kernel(Ctrl* c, Seg* sg, int nseg, const double* t0, int par,
                                 int keep);
// CFL minimum of the incoming state, one block per tile.
__global__ void dt_init_kernel(DevMesh m, TileMap tm, const Cell4* W, double g, double thr,
                               Seg* sg);
// Two-pass organisation: recon_kernel reconstructs the state the stage reads
// (STAGE 1: w^n from Wa/Wb; STAGE 2: w1) into the face buffer.
template <int STAGE>
__global__ void recon_kernel(DevMesh m, TileMap tm, const Cell4* Wa, const Cell4* Wb,
                             const Cell4* W1, FaceBuf fb, StepParams p, const Ctrl* c,
                             const Seg* sg, int slot, int step_arg);
__global__ void update1_kernel(DevMesh m, TileMap tm, const Cell4* Wa, const Cell4* Wb,
                               Cell4* W1, FaceBuf fb, StepParams p, Ctrl* c, Seg* sg, int slot,
                               int step_arg);
__global__ void update2_kernel(DevMesh m, TileMap tm, Cell4* Wa, Cell4* Wb, const Cell4* W1,
                               FaceBuf fb, StepParams p, Ctrl* c, Seg* sg, int slot, int step_arg,
                               double* log);
// Free surface at the gauge cells after step kbase + step_arg (read from the
// buffer that step wrote); gseg[g] is the scenario of gauge g.
__global__ void gauge_kernel(const Cell4* Wa, const Cell4* Wb, const int64_t* cells, int ng,
                             const int32_t* gseg, const Seg* sg, const Ctrl* c, int step_arg,
                             double* log);
// Advance the step base by `by` steps (the last node of a captured pair).
__global__ void step_bump_kernel(Ctrl* c, int by);
// perm[i] = caller index of internal cell i, or -1 for the padding cells
// that round each scenario up to whole tiles (left untouched).
__global__ void pack_state_kernel(int64_t n, const int64_t* perm, const double* H,
                                  const double* HU, const double* HV, const double* h, Cell4* W,
                                  Cell4* W1);
// Checks a caller-order state (nc cells): bit 0 of *flag for a non-finite
// value, bit 1 for a negative depth (*flag is cleared by the caller).
__global__ void check_state_kernel(int64_t nc, const double* H, const double* HU,
                                   const double* HV, int* flag);
__global__ void unpack_state_kernel(int64_t n, const int64_t* perm, const Cell4* W, double* H,
                                    double* HU, double* HV);

}  // namespace vsw
