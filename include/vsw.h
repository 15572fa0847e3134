/*
 * vsw.h -- C ABI of the MI355X (gfx950) shallow-water finite-volume library.
 *
 * The library advances the 2D nonlinear shallow water equations (Section
 * 2.1 of Giles et al., "Performance analysis of Volna-OP2", 2020) on an
 * unstructured triangular mesh with the explicit scheme of Sections 2.2-2.5:
 * cell-centred finite volumes, MUSCL reconstruction by a least-squares
 * gradient and a Barth-Jespersen limiter (eq. (3)), HLL fluxes with the wave
 * speeds of Section 2.2, wall boundaries by ghost cells (Section 2.5), and
 * the SSP-RK(2,2) time stepper with a CFL time step (Section 2.3).  Every
 * step runs in HIP kernels on one GPU.
 *
 * Conventions
 *  - Return value 0 (VSW_OK) on success, a negative VSW_E* code on failure;
 *    vsw_last_error() then describes the failure.  No C++ exception crosses
 *    this interface.
 *  - Units are SI.  h is the still-water depth (positive below the datum,
 *    negative on land; the bed elevation is z = -h), H = h + eta the total
 *    depth, (HU, HV) = H (u, v) the momentum.  State arrays are FP64.
 *  - Pointers named host_* or without a suffix are host memory owned by the
 *    caller; the library copies from or into them during the call and keeps
 *    no reference.  Pointers named dev_* are device memory on the solver's
 *    device, owned by the caller, used only during the call (in stream order
 *    on the solver's stream).
 *  - Cell order at the interface is always the caller's order; the internal
 *    renumbering is invisible.
 *  - A solver is used by one host thread at a time.
 */
#ifndef VSW_H
#define VSW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    VSW_OK = 0,
    VSW_EINVAL = -1,    /* bad argument (NULL, size, non-finite, H < 0) */
    VSW_EMESH = -2,     /* invalid mesh (see vsw_upload_mesh) */
    VSW_ESTATE = -3,    /* call out of order (no mesh or no state yet) */
    VSW_ENOMEM = -4,    /* device or host allocation failed */
    VSW_EDEVICE = -5,   /* HIP runtime error */
    VSW_EUNSTABLE = -6  /* non-finite state or no valid time step */
};

/* Arithmetic of the solver.  VSW_FP64: every step in FP64.  VSW_FP32:
 * mixed precision -- the free surface eta = H - h and the momentum are
 * stored in FP32, and the reconstruction, face velocities, wave speeds and
 * the mass and tangential fluxes are FP32; depths, the hydrostatic
 * reconstruction, the normal-momentum flux, the bed-source terms, each
 * cell's residual accumulation, the stage update and the CFL reduction stay
 * FP64.  State transfer stays FP64 at the interface. */
enum { VSW_FP64 = 0, VSW_FP32 = 1 };
/* Internal cell order (results are bitwise the same under every order; it
 * sets the memory locality and the tiles of the fused stage kernels, which
 * are runs of 256 consecutive internal cells).  HILBERT: cell centroids
 * along a Hilbert curve.  NONE: the caller's order.  RANDOM: a seeded
 * permutation.  BISECTION: recursive coordinate bisection of the centroids
 * into 256-cell leaves (compact tiles with about a fifth fewer faces on
 * their boundary than Hilbert runs), Hilbert order inside each leaf. */
enum { VSW_ORDER_HILBERT = 0, VSW_ORDER_NONE = 1, VSW_ORDER_RANDOM = 2,
       VSW_ORDER_BISECTION = 3 };

typedef struct vsw_params {
    double g;            /* gravity (m/s^2), in (0, 2^100] */
    double cfl;          /* Courant number of the dt rule, > 0 (Section 2.3) */
    double h_threshold;  /* threshold depth H_thr (m), >= 0 (Section 2.4):
                            below it a cell is not reconstructed and its
                            velocity is taken as zero */
    double dt_fixed;     /* > 0: constant time step; 0: CFL rule
                            dt = cfl * min_K |K| / (P_K (|u_K| + sqrt(g H_K)))
                            over cells with H_K >= H_thr */
    int32_t precision;   /* VSW_FP64 or VSW_FP32 */
    int32_t ordering;    /* internal cell order: VSW_ORDER_* */
    uint64_t seed;       /* seed of VSW_ORDER_RANDOM */
} vsw_params;

typedef struct vsw_solver vsw_solver;

/* Create a solver on HIP device `device` (Section 2 parameters in p).
 * EINVAL if p is NULL, g outside (0, 2^100], cfl <= 0, h_threshold < 0,
 * dt_fixed < 0 or an unknown precision/ordering; EDEVICE if the device
 * cannot be used. */
int vsw_create(const vsw_params *p, int device, vsw_solver **out);

/* Free every device and host resource of the solver.  NULL is a no-op. */
void vsw_destroy(vsw_solver *s);

/* Upload the triangular mesh (Section 2.2): nv vertices (vx, vy), nc
 * triangles tri[3*nc] (vertex indices, either orientation) and the
 * still-water depth h[nc] sampled at each triangle's centroid.  Builds
 * edges, neighbours and wall faces (every face with one triangle is a wall,
 * Section 2.5), the geometry and the internal renumbering, and copies the
 * result to the device.  EMESH on an index out of range, a zero-area
 * triangle, a face shared by more than two triangles, two triangles on the
 * same side of a face, or duplicate vertex coordinates on a face; EINVAL
 * on a vertex coordinate that is neither 0 nor within [2^-300, 2^300] in
 * magnitude (the range in which the kernels' face geometry is exact),
 * or a non-finite depth.  Replaces any previous mesh and discards the
 * state. */
int vsw_upload_mesh(vsw_solver *s, int64_t nv, const double *vx,
                    const double *vy, int64_t nc, const int32_t *tri,
                    const double *h);

/* Ensembles: nscen independent scenarios (the many-run uncertainty and
 * sensitivity studies that Section 1 motivates) advanced together, each on
 * its own mesh, with its own CFL time step and time, in the same kernel
 * launches.  Scenario s has nv[s] vertices and nc[s] triangles; vx, vy hold
 * all scenarios' vertices one scenario after the other, tri and h all
 * triangles (tri indexes the scenario's own vertices, from 0).  Every other
 * call then uses the concatenated cell numbering: cell k of scenario s is
 * cell nc[0] + ... + nc[s-1] + k (state arrays, gauges, vsw_mesh_info's
 * cell count).  vsw_step advances every scenario by up to n steps of its
 * own dt, each stopping on its own at t_stop; *steps_done is the most steps
 * any scenario took and *t_out the earliest scenario time; vsw_dt_history,
 * vsw_last_dt and the gauge times refer to scenario 0.  Errors as
 * vsw_upload_mesh, for the failing scenario; EINVAL if nscen <= 0 or
 * nscen > 2^22.  vsw_upload_mesh is the case nscen = 1. */
int vsw_upload_ensemble(vsw_solver *s, int32_t nscen, const int64_t *nv,
                        const double *vx, const double *vy, const int64_t *nc,
                        const int32_t *tri, const double *h);

/* Number of scenarios of the uploaded mesh (1 after vsw_upload_mesh). */
int vsw_scenario_count(vsw_solver *s, int32_t *nscen);

/* Per scenario (up to max): its time, its last dt and the steps it took in
 * the last vsw_step call (any output may be NULL). */
int vsw_scenario_status(vsw_solver *s, int32_t max, double *t, double *dt_last,
                        int64_t *steps);

/* dt of each step scenario scen took in the last vsw_step call: up to max
 * values into dts (may be NULL); *count receives the number of steps.
 * EINVAL on a scenario index out of range. */
int vsw_scenario_dt_history(vsw_solver *s, int32_t scen, int64_t max,
                            double *dts, int64_t *count);

/* Discrete adjoint (one scenario, tiles of 256 cells).  From the current state,
 * run nsteps steps (the solver's dt rule, no t_stop) and evaluate the gauge
 * misfit loss = sum_{n=1..nsteps} sum_g (eta_g^n - eta_obs[(n-1) * ng + g])^2,
 * eta = H - h at gauge_cells[g] (caller's cell indices) after step n; then
 * run the hand-written reverse of every step (Section 2.3 stages, Section
 * 2.2 fluxes, Section 2.4 reconstruction with its branches as taken, the
 * post-stage fix and the CFL time step) backwards from checkpoints taken
 * every `checkpoint_every` steps, each segment replayed forward with the
 * recorded dts while the stage kernels record a tape (states, residuals,
 * fix masks, CFL minima) for the reverse.  Outputs
 * (caller's order, nc values each; any gradient pointer may be NULL): *loss,
 * and d loss / d H, HU, HV of the initial state and d loss / d h (the bed
 * depth, with the initial H, HU, HV held fixed).  The solver's state, time,
 * gauges and logs are unchanged on return.  Device memory: about
 * 32 * ceil(nsteps / checkpoint_every) + 114 * min(checkpoint_every, nsteps)
 * + 250 bytes per cell.  On an FP32 solver the forward run and the segment
 * replays are the FP32 kernels (its trajectory, its dts) and the reverse
 * sweep is the FP64 adjoint of the scheme evaluated on the FP32 states:
 * an approximation of the FP32 run's gradient, not its exact adjoint.
 * EINVAL on an ensemble solver, tiles other than 256 cells, ng < 1 or bad
 * counts; ENOMEM when that memory is not available; EUNSTABLE if the
 * forward run fails. */
int vsw_adjoint_gauge_loss(vsw_solver *s, int64_t nsteps,
                           int64_t checkpoint_every, int32_t ng,
                           const int32_t *gauge_cells, const double *eta_obs,
                           double *loss, double *grad_H, double *grad_HU,
                           double *grad_HV, double *grad_h);

/* Set the state w = (H, HU, HV) (Section 2.1) from host arrays of nc values
 * in the caller's cell order, at time t.  EINVAL on a non-finite value or
 * H < 0; ESTATE before vsw_upload_mesh. */
int vsw_set_state(vsw_solver *s, const double *H, const double *HU,
                  const double *HV, double t);

/* Same as vsw_set_state from device arrays (caller's cell order), which
 * the solver's stream must be able to read.  The values are checked on the
 * device before anything is written: EINVAL on a non-finite value or
 * H < 0, and the solver's state is then left as it was.  Synchronises the
 * solver's stream. */
int vsw_set_state_device(vsw_solver *s, const double *dev_H,
                         const double *dev_HU, const double *dev_HV, double t);

/* Advance up to n SSP-RK(2,2) steps (Section 2.3), stopping early when the
 * time reaches t_stop (the last step is shortened so that t lands exactly
 * on t_stop; pass INFINITY for no limit).  Kernels are queued on the
 * solver's stream without host synchronisation between steps; the call
 * synchronises once at the end.  *steps_done (may be NULL) receives the
 * number of completed steps and *t_out (may be NULL) the new time.
 * EUNSTABLE if a step made the state non-finite or found no valid time
 * step: steps_done then counts the good steps before it, and the solver's
 * state and time are those the good steps reached, i.e. the input of the
 * failing step (a further call fails at the same step again unless the
 * state or parameters change).  ESTATE without mesh and state. */
int vsw_step(vsw_solver *s, int64_t n, double t_stop, int64_t *steps_done,
             double *t_out);

/* vsw_step for callers that cannot allocate memory (code under HIP graph
 * capture, serving loops that forbid hipMalloc): the same steps with the
 * same results and error behaviour, but the per-call step log (time and dt
 * of every step and scenario) and the gauge records are kept in a fixed
 * device array of the library, VSW_NOALLOC_BYTES per device (set up by
 * vsw_create, held until the process ends), instead of buffers the solver
 * grows.  It allocates no device or host memory, captures no graph
 * (vsw_set_graph is ignored) and records no profiling events.  The call must
 * fit the array: n * (2 * scenarios + gauges) doubles <= VSW_NOALLOC_BYTES /
 * 8, else EINVAL; with VSW_KERNEL_TWO_PASS its face buffer must already
 * exist (after one vsw_step), else EINVAL.  Every call on a device uses
 * that device's one array and overwrites what the previous call left there
 * (nothing in it needs to start at zero): calls that overlap on one device,
 * from several host threads or solvers on different streams, race. */
#define VSW_NOALLOC_BYTES (1u << 20)
int vsw_step_noalloc(vsw_solver *s, int64_t n, double t_stop,
                     int64_t *steps_done, double *t_out);

/* Copy the state to host arrays (caller's order); *t (may be NULL) gets the
 * time. */
int vsw_get_state(vsw_solver *s, double *H, double *HU, double *HV, double *t);

/* Copy the state to device arrays (caller's order). */
int vsw_get_state_device(vsw_solver *s, double *dev_H, double *dev_HU,
                         double *dev_HV, double *t);

/* dt of the last completed step (0 before the first). */
int vsw_last_dt(vsw_solver *s, double *dt);

/* dt of each completed step of the last vsw_step call: up to max values
 * into dts (may be NULL); *count receives the number of steps. */
int vsw_dt_history(vsw_solver *s, int64_t max, double *dts, int64_t *count);

/* Virtual gauges (the time series of Sections 3 and 5): n cells in the
 * caller's order whose free surface eta = H - h is recorded on the device
 * after every step of each vsw_step call.  n = 0 removes them.  EINVAL on a
 * cell index out of range; ESTATE before vsw_upload_mesh (a new mesh clears
 * the gauges). */
int vsw_set_gauges(vsw_solver *s, int32_t n, const int32_t *cells);

/* Records of the last vsw_step call: *count = its steps; up to max_steps
 * rows into eta_out[step * n + gauge] and the time after each step into
 * t_out (either may be NULL). */
int vsw_get_gauges(vsw_solver *s, int64_t max_steps, double *eta_out,
                   double *t_out, int64_t *count);

/* Number of negative depths set to zero after a stage since the last
 * vsw_set_state (a post-stage positivity fix; 0 in a well-resolved run). */
int vsw_clamp_count(vsw_solver *s, int64_t *count);

/* Run on the caller's HIP stream (a hipStream_t passed as void*, on the
 * solver's device); NULL returns to the solver's own stream. */
int vsw_set_stream(vsw_solver *s, void *hip_stream);

/* Kernel organisation of a stage (same results, bitwise):
 * VSW_KERNEL_FACES (default): one kernel per stage; each workgroup
 *   reconstructs a tile of consecutive (Hilbert-ordered) cells and its halo
 *   faces into LDS, evaluates every face of the tile once (normal and
 *   length from the face's vertices) and updates its cells.
 * VSW_KERNEL_FUSED: one kernel per stage, tiles of 256 cells; each cell
 *   evaluates its three faces itself from LDS, with the face geometry read
 *   from device memory.
 * VSW_KERNEL_TWO_PASS (FP64 only): a reconstruction kernel writes every
 *   face state to device memory, a second kernel computes fluxes and the
 *   update.
 * FUSED and TWO_PASS need tiles of 256 cells (vsw_step: EINVAL otherwise).
 * EINVAL for an unknown variant, and for TWO_PASS on FP32. */
enum { VSW_KERNEL_FUSED = 0, VSW_KERNEL_TWO_PASS = 1, VSW_KERNEL_FACES = 2 };
int vsw_set_kernel_variant(vsw_solver *s, int variant);

/* Cells per tile (one workgroup, one thread per cell) of the layout of the
 * mesh on the device: 128, 256 (default) or 512.  With a mesh uploaded the
 * mesh is laid out again and its state records (unchanged, in either
 * precision), time and gauges carried over (results are bitwise the same
 * for every tile size); otherwise it applies to the next upload.  The solver keeps a copy of the uploaded mesh for this.  EINVAL
 * for other sizes; ENOMEM/EDEVICE as vsw_upload_mesh. */
int vsw_set_tile_size(vsw_solver *s, int cells);
int vsw_tile_size(vsw_solver *s, int *cells);

/* Graph mode: 0 (default) launches every kernel of a vsw_step call
 * directly; 1 captures one pair of steps (their kernel launches and a
 * one-thread kernel that advances the device-side step index) into a HIP
 * graph once and replays it n / 2 times, an odd last step launched
 * directly; 2 captures the whole call (n steps, up to 20000; longer calls
 * use mode 1) as one graph, captured again when n changes.  Results are
 * bitwise the same in every mode.  The graphs hold kernel nodes only and
 * are captured again when the mesh, the gauges, t_stop, the kernel
 * variant, the tile layout or the log buffers change.  Profiling
 * (vsw_set_profiling) and vsw_step_noalloc launch directly.  Setting a mode
 * frees the current graph.  EINVAL for other values. */
int vsw_set_graph(vsw_solver *s, int on);

/* Order in which the stage kernels' workgroups visit the tiles: 1
 * (default) deals each of the eight XCDs (each with its own L2) one
 * contiguous run of Hilbert-ordered tiles; 0 visits tiles in index order.
 * Results are bitwise the same.  EINVAL for other values. */
int vsw_set_tile_order(vsw_solver *s, int xcd_order);

/* Workgroups of the fused stage kernels resident per compute unit:
 * 0 (default) as many as registers and LDS allow (4 for FP64, 5 for FP32
 * on gfx950); 3 or 2 cap them (each workgroup then requests more than
 * 1/(cap + 1) of the CU's 160 KiB of LDS), which trades latency hiding for
 * less cache pressure.  Results are bitwise the same.  EINVAL for other
 * values. */
int vsw_set_occupancy(vsw_solver *s, int wg_per_cu);

/* Autotuner: runs `steps` steps (after a warm-up: two steps, or in graph
 * mode 2 one call of `steps` steps that captures its graph) of the current
 * state under every launch configuration
 *   c = (org * 2 + xcd) * 3 + graph,  c = 0 .. VSW_TUNE_CONFIGS - 1,
 * org: 0, 1, 2 the face-parallel kernels with tiles of 128, 256, 512
 * cells; 3, 4, 5 the fused cell-parallel kernel (tiles of 256) with as many
 * workgroups per CU as fit, at most 3, at most 2; 6 the two-pass
 * organisation (FP64 only); xcd: the tile order of vsw_set_tile_order;
 * graph: the mode of vsw_set_graph.  Each configuration is timed with HIP
 * events on the solver's stream, the state, time and logs are restored
 * after each, and the fastest configuration is kept for later vsw_step
 * calls (its tile size laid out as vsw_set_tile_size does).  Every
 * configuration gives bitwise the same results.  ms_per_step (may be NULL)
 * receives VSW_TUNE_CONFIGS values (INFINITY where a configuration does not
 * apply), *chosen (may be NULL) the winner.  EINVAL unless
 * 2 <= steps <= 100000; ESTATE without mesh and state. */
enum { VSW_TUNE_CONFIGS = 42 };
int vsw_autotune(vsw_solver *s, int64_t steps, int32_t *chosen,
                 double *ms_per_step);

/* Per-kernel timing with HIP events recorded around every launch of the
 * stage kernels on the solver's stream (off by default).  vsw_kernel_times
 * returns, for kernel kinds 0..nkinds-1 (see vsw_kernel_name), the summed
 * milliseconds and launch counts since profiling was switched on. */
int vsw_set_profiling(vsw_solver *s, int on);
int vsw_kernel_times(vsw_solver *s, int nkinds, double *ms, int64_t *launches);
const char *vsw_kernel_name(int kind);

/* Host-only mesh preparation (no device needed): runs the same validation,
 * face matching, canonical orientation and geometry as vsw_upload_mesh and
 * returns them in the caller's cell order.  Outputs (any may be NULL):
 * geom[7*3*nc] as [field][face j][cell] with fields nx, ny (outward unit
 * normal of face j, which joins local vertices j and j+1 of the
 * counter-clockwise triangle), len, dx, dy (face midpoint minus centroid),
 * wx, wy (least-squares weights of stencil member j); area[nc], perim[nc];
 * nbr[3*nc] as [face j][cell]: neighbour cell or -1 for a wall; is_left
 * [3*nc]: 1 if the cell is the canonical left side of the face (walls: 1).
 * Returns VSW_EMESH / VSW_EINVAL like vsw_upload_mesh. */
int vsw_prepare_mesh_host(int64_t nv, const double *vx, const double *vy,
                          int64_t nc, const int32_t *tri, const double *h,
                          double *geom, double *area, double *perim,
                          int32_t *nbr, int32_t *is_left, int64_t *ne,
                          int64_t *nw);

/* Internal cell order: perm[i] = caller's index of the i-th internal cell
 * (nc values; the padding that rounds each scenario of an ensemble up to
 * whole tiles is skipped). */
int vsw_get_permutation(vsw_solver *s, int64_t *perm);

/* Mesh sizes after upload: cells, edges, wall faces. */
int vsw_mesh_info(vsw_solver *s, int64_t *nc, int64_t *ne, int64_t *nw);

/* Message of the last failing call on this thread ("" if none). */
const char *vsw_last_error(void);

/* Library version string. */
const char *vsw_version(void);

#ifdef __cplusplus
}
#endif
#endif /* VSW_H */
