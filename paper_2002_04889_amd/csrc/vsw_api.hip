// C ABI of the solver (include/vsw.h): context, device buffers, stream,
// mesh upload, state transfer and the step loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/vsw.h"
#include "vsw_adjoint.hpp"
#include "vsw_faces.hpp"
#include "vsw_kernels.hpp"
#include "vsw_kernels_f32.hpp"
#include "vsw_mesh.hpp"

using namespace vsw;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(e_ == hipErrorOutOfMemory ? VSW_ENOMEM : VSW_EDEVICE,           \
                        std::string(#expr) + ": " + hipGetErrorString(e_));             \
    } while (0)

enum KernelKind { KK_RECON = 0, KK_UPDATE1, KK_UPDATE2, KK_DTINIT, KK_STAGE1, KK_STAGE2, KK_COUNT };
const char* kKernelNames[KK_COUNT] = {"recon_kernel",   "update1_kernel", "update2_kernel",
                                      "dt_init_kernel", "stage1_kernel",  "stage2_kernel"};

// Everything a captured step pair bakes into its launch arguments besides
// the mesh (a new mesh drops the graph).
struct GraphKey {
    const double* log;
    const double* gauge_log;
    const int64_t* gauge_cells;
    int ngauges;
    double t_stop;
    int variant;
    int64_t nsteps;  // steps of a whole-call graph, 0 for the step pair
    bool operator==(const GraphKey& o) const {
        return log == o.log && gauge_log == o.gauge_log && gauge_cells == o.gauge_cells &&
               ngauges == o.ngauges && (t_stop == o.t_stop || (t_stop != t_stop && o.t_stop != o.t_stop)) &&
               variant == o.variant && nsteps == o.nsteps;
    }
};

// Steps of room the per-call logs start with.
constexpr size_t kLogMinSteps = 4096;

// Longest call captured as one graph in graph mode 2 (longer calls replay
// the step pair).
constexpr int64_t kWholeGraphMaxSteps = 20000;

// Runs f when the scope ends, on every return path.
template <class F>
struct OnExit {
    F f;
    bool armed = true;
    ~OnExit() {
        if (armed) f();
    }
};
template <class F>
OnExit<F> on_exit(F f) {
    return OnExit<F>{f};
}

// Dynamic LDS of a fused stage launch: the kernel's own need, raised above
// 1/(cap + 1) of the CU's 160 KiB when the resident workgroups per CU are
// capped, so that at most `cap` fit.
size_t capped_lds(size_t need, int cap) {
    if (cap <= 0) return need;
    const size_t cu = size_t(160) * 1024;
    return std::max(need, cu / size_t(cap + 1) + 1024);
}

// Device array owned by one object: freed by release() or when it goes out
// of scope.
template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    hipError_t alloc(size_t count) {
        release();
        if (count == 0) return hipSuccess;
        hipError_t e = hipMalloc(&p, count * sizeof(T));
        if (e == hipSuccess) n = count;
        return e;
    }
};

// Pinned host array (hipHostMalloc): the per-call transfers of the step
// loop run as plain DMA, without staging.
template <class T>
struct PinBuf {
    T* p = nullptr;
    size_t n = 0;
    PinBuf() = default;
    PinBuf(const PinBuf&) = delete;
    PinBuf& operator=(const PinBuf&) = delete;
    ~PinBuf() { release(); }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        n = 0;
    }
    hipError_t alloc(size_t count) {
        release();
        if (count == 0) return hipSuccess;
        hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&p), count * sizeof(T),
                                     hipHostMallocDefault);
        if (e == hipSuccess) n = count;
        return e;
    }
};

// Device memory of vsw_step_noalloc: the step log (time and dt of each step
// and scenario) and the gauge records of a call, in one array per device
// that lives until the process ends.  Host code never passes the array's
// name to a kernel or a copy: it uses the device address resolved for each
// device by resolve_scratch (called from vsw_create with the device current).
constexpr size_t kScratchDoubles = VSW_NOALLOC_BYTES / sizeof(double);
static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mu;
std::vector<double*> g_scratch_ptr;  // per device; null until resolved

int resolve_scratch(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr.size() <= size_t(device)) g_scratch_ptr.resize(size_t(device) + 1, nullptr);
    if (g_scratch_ptr[size_t(device)]) return VSW_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(VSW_EDEVICE, std::string("no-allocation scratch array: ") + hipGetErrorString(e));
    g_scratch_ptr[size_t(device)] = static_cast<double*>(ptr);
    return VSW_OK;
}

double* scratch_ptr(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return (size_t(device) < g_scratch_ptr.size()) ? g_scratch_ptr[size_t(device)] : nullptr;
}

}  // namespace

struct vsw_solver {
    vsw_params prm{};
    int device = 0;
    hipStream_t own_stream = nullptr;
    hipStream_t stream = nullptr;
    bool has_mesh = false, has_state = false;
    int64_t nc = 0, ne = 0, nw = 0;   // caller cells (all scenarios), faces, walls
    int64_t nint = 0;                 // internal cells, padding included
    int nseg = 1;                     // scenarios
    std::vector<int64_t> seg_off;     // [nseg + 1] caller offsets of the scenarios
    std::vector<double> seg_t;        // time of each scenario
    std::vector<double> seg_dt;       // last dt of each scenario
    std::vector<int64_t> seg_steps;   // steps each scenario took in the last call
    std::vector<double> seg_log;      // last call's dt log, [step][scenario]
    std::vector<int64_t> perm;        // internal -> caller, -1 on padding
    DevBuf<int64_t> d_perm;
    DevBuf<Nbr4> d_nbr;            // neighbour slots per cell
    DevBuf<double> d_geom, d_area, d_perim, d_h;
    DevBuf<RGeom> d_rgeom;         // reconstruction geometry records
    DevBuf<RGeomF> d_rgeomf;       // the same in FP32 (FP32 solvers)
    // The state alternates between two buffers (a step reads one and writes
    // the other); cur is the one holding the current state.
    DevBuf<Cell4> d_w[2];          // w^n records (H, HU, HV, h), FP64 solver
    DevBuf<Cell4> d_w1;            // stage-1 records, FP64 solver
    DevBuf<CellF> d_wf[2];         // w^n records (h, eta, Hu, Hv), FP32 solver
    DevBuf<CellF> d_w1f;           // stage-1 records, FP32 solver
    int cur = 0;
    DevBuf<int> d_flag;            // state check of vsw_set_state_device
    DevBuf<double> d_face;         // 15 * nc face buffer
    DevBuf<double> d_sc;           // 2 * nc
    DevBuf<int32_t> d_order;       // nc
    DevBuf<double> d_tmp;          // 3 * nc staging of caller-order arrays
    DevBuf<double> d_log;          // 2 * cap: t and dt per step
    DevBuf<Ctrl> d_ctrl;
    DevBuf<Seg> d_seg;             // per-scenario control records
    DevBuf<double> d_t0;           // per-scenario start times of a call
    DevBuf<uint32_t> d_tinfo;      // tile words
    DevBuf<int64_t> d_gauge_cells; // internal indices of the gauge cells
    DevBuf<int32_t> d_gauge_seg;   // scenario of each gauge
    DevBuf<double> d_gauge_log;    // [step][gauge] free surface of the last call
    int ngauges = 0;
    std::vector<int32_t> gauge_user;  // the gauge cells in the caller's order
    std::vector<double> gauge_eta; // host copy of the last call's records
    std::vector<double> gauge_t;
    DevBuf<uint16_t> d_nloc;       // tile map of the fused kernel
    DevBuf<int32_t> d_bstart;
    DevBuf<uint32_t> d_bitem;
    int bmax = 0, ntiles = 0;
    // face-parallel kernels: tiles of `tile` cells
    int tile = kTile;           // tile size of the uploaded layout
    int tile_req = kTile;       // tile size of the next layout
    DevBuf<TopoD> d_topo;
    DevBuf<LsqW> d_lsq;
    DevBuf<LsqWF> d_lsqf;
    DevBuf<double2> d_vxy;
    DevBuf<int32_t> d_fbstart, d_fstart;
    DevBuf<uint32_t> d_fbitem;
    DevBuf<FaceItemD> d_fitems;
    int fbmax = 0;
    // the caller's mesh, kept to lay it out again for another tile size
    int raw_nseg = 0;
    std::vector<int64_t> raw_nv, raw_nc;
    std::vector<double> raw_vx, raw_vy, raw_h;
    std::vector<int32_t> raw_tri;
    int variant = VSW_KERNEL_FACES;
    int graph_mode = 0;  // 0 direct launches, 1 step-pair graph, 2 whole-call graph
    int xcd_order = 1;
    int occupancy = 0;  // fused stage kernels: workgroups per CU cap (0 = none)
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    GraphKey graph_key{};
    void release_graph() {
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        if (graph) (void)hipGraphDestroy(graph);
        graph_exec = nullptr;
        graph = nullptr;
    }
    double t = 0.0;
    double dt_last = 0.0;
    int64_t clamps = 0;
    // profiling
    bool profiling = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<int> ev_kind;      // kind of each event pair
    double prof_ms[KK_COUNT] = {};
    int64_t prof_n[KK_COUNT] = {};
    std::vector<double> last_dts;
    // host copies a step call reads back (kept between calls so that a call
    // within the sizes of vsw_step_noalloc allocates no host memory)
    std::vector<Seg> h_seg;
    std::vector<double> h_logs;
    PinBuf<double> pin_t0;       // [nseg] start times of a call
    PinBuf<Ctrl> pin_ctrl;
    PinBuf<Seg> pin_seg;         // [nseg]
    PinBuf<double> pin_logs;     // step log of a call (grows with vsw_step)
    // Slot of the scenarios' records that holds the CFL minimum of the
    // current state (set when every scenario took every step of the last
    // call), -1 when it must be computed.
    int rmin_slot = -1;

    void release_mesh() {
        release_graph();
        d_perm.release(); d_nbr.release(); d_geom.release(); d_area.release();
        d_rgeom.release();
        d_rgeomf.release();
        d_perim.release(); d_h.release(); d_w[0].release(); d_w[1].release(); d_w1.release();
        d_wf[0].release(); d_wf[1].release(); d_w1f.release();
        cur = 0;
        d_face.release(); d_sc.release(); d_order.release(); d_tmp.release();
        d_nloc.release(); d_bstart.release(); d_bitem.release(); d_tinfo.release();
        d_topo.release(); d_lsq.release(); d_lsqf.release(); d_vxy.release(); d_fbstart.release();
        d_fstart.release(); d_fbitem.release(); d_fitems.release();
        d_seg.release(); d_t0.release();
        rmin_slot = -1;
        d_gauge_cells.release();
        d_gauge_seg.release();
        ngauges = 0;
        gauge_user.clear();
        has_mesh = has_state = false;
    }
    // caller-order arrays (device) -> state records of both stage buffers
    void pack(const double* H, const double* HU, const double* HV) {
        const dim3 g(unsigned((nint + kBlock - 1) / kBlock));
        if (prm.precision == VSW_FP32)
            hipLaunchKernelGGL(pack_state_f32_kernel, g, dim3(kBlock), 0, stream, nint, d_perm.p,
                               H, HU, HV, d_h.p, d_wf[cur].p, d_w1f.p);
        else
            hipLaunchKernelGGL(pack_state_kernel, g, dim3(kBlock), 0, stream, nint, d_perm.p, H,
                               HU, HV, d_h.p, d_w[cur].p, d_w1.p);
    }
    // state records -> caller-order arrays (device; NULL skips a field)
    void unpack(double* H, double* HU, double* HV) {
        const dim3 g(unsigned((nint + kBlock - 1) / kBlock));
        if (prm.precision == VSW_FP32)
            hipLaunchKernelGGL(unpack_state_f32_kernel, g, dim3(kBlock), 0, stream, nint, d_perm.p,
                               d_wf[cur].p, d_h.p, H, HU, HV);
        else
            hipLaunchKernelGGL(unpack_state_kernel, g, dim3(kBlock), 0, stream, nint, d_perm.p,
                               d_w[cur].p, H, HU, HV);
    }
    void set_time(double t0) {
        t = t0;
        dt_last = 0.0;
        clamps = 0;
        seg_t.assign(size_t(nseg), t0);
        seg_dt.assign(size_t(nseg), 0.0);
        seg_steps.assign(size_t(nseg), 0);
        seg_log.clear();
        last_dts.clear();
        has_state = true;
        rmin_slot = -1;
    }
    FaceMesh face_mesh() const {
        FaceMesh m;
        m.nc = nint;
        m.topo = d_topo.p;
        m.lsq = d_lsq.p;
        m.lsqf = d_lsqf.p;
        m.vxy = d_vxy.p;
        m.perim = d_perim.p;
        return m;
    }
    FaceTileMap face_tiles(int nsg) const {
        return FaceTileMap{d_fbstart.p, d_fbitem.p, d_fstart.p, d_fitems.p, d_tinfo.p, fbmax,
                           ntiles, nsg, xcd_order};
    }
    DevMesh dev_mesh() const {
        DevMesh m;
        m.nc = nint;
        m.nbr = d_nbr.p;
        m.geom = d_geom.p;
        m.rgeom = d_rgeom.p;
        m.rgeomf = d_rgeomf.p;
        m.area = d_area.p;
        m.perim = d_perim.p;
        m.hcell = d_h.p;
        return m;
    }
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

unsigned grid_for(int64_t n) { return unsigned((n + kBlock - 1) / kBlock); }

// Face-parallel stage kernel of the tile size in use.
void launch_faces_stage(int tile, int stage, int ntiles, size_t lds, hipStream_t q,
                        const FaceMesh& m, const FaceTileMap& tm, Cell4* Wa, Cell4* Wb,
                        Cell4* W1, const StepParams& p, Ctrl* c, Seg* sg, int slot, int sa,
                        double* lg) {
    const dim3 grid{unsigned(ntiles), 1u, 1u};
#define VSW_LAUNCH_FACES(T)                                                                    \
    if (stage == 1)                                                                            \
        hipLaunchKernelGGL((faces_stage_kernel<T, 1>), grid, dim3(T), lds, q, m, tm, Wa, Wb,   \
                           W1, p, c, sg, slot, sa, lg);                                        \
    else                                                                                       \
        hipLaunchKernelGGL((faces_stage_kernel<T, 2>), grid, dim3(T), lds, q, m, tm, Wa, Wb,   \
                           W1, p, c, sg, slot, sa, lg);
    if (tile == 128) {
        VSW_LAUNCH_FACES(128)
    } else if (tile == 512) {
        VSW_LAUNCH_FACES(512)
    } else {
        VSW_LAUNCH_FACES(256)
    }
#undef VSW_LAUNCH_FACES
}

void launch_faces_stage_f32(int tile, int stage, int ntiles, size_t lds, hipStream_t q,
                            const FaceMesh& m, const FaceTileMap& tm, const double* h, CellF* Wa,
                            CellF* Wb, CellF* W1, const StepParams& p, Ctrl* c, Seg* sg, int slot,
                            int sa, double* lg) {
    const dim3 grid{unsigned(ntiles), 1u, 1u};
#define VSW_LAUNCH_FACES_F32(T)                                                                \
    if (stage == 1)                                                                            \
        hipLaunchKernelGGL((faces_stage_f32_kernel<T, 1>), grid, dim3(T), lds, q, m, tm, h,    \
                           Wa, Wb, W1, p, c, sg, slot, sa, lg);                                \
    else                                                                                       \
        hipLaunchKernelGGL((faces_stage_f32_kernel<T, 2>), grid, dim3(T), lds, q, m, tm, h,    \
                           Wa, Wb, W1, p, c, sg, slot, sa, lg);
    if (tile == 128) {
        VSW_LAUNCH_FACES_F32(128)
    } else if (tile == 512) {
        VSW_LAUNCH_FACES_F32(512)
    } else {
        VSW_LAUNCH_FACES_F32(256)
    }
#undef VSW_LAUNCH_FACES_F32
}

void launch_faces_dt_init_f32(int tile, int ntiles, hipStream_t q, const FaceMesh& m,
                              const FaceTileMap& tm, const CellF* W, const double* h,
                              const double* area, double g, double thr, Seg* sg) {
    const dim3 grid{unsigned(ntiles), 1u, 1u};
    if (tile == 128)
        hipLaunchKernelGGL(faces_dt_init_f32_kernel<128>, grid, dim3(128), 0, q, m, tm, W, h,
                           area, g, thr, sg);
    else if (tile == 512)
        hipLaunchKernelGGL(faces_dt_init_f32_kernel<512>, grid, dim3(512), 0, q, m, tm, W, h,
                           area, g, thr, sg);
    else
        hipLaunchKernelGGL(faces_dt_init_f32_kernel<256>, grid, dim3(256), 0, q, m, tm, W, h,
                           area, g, thr, sg);
}

void launch_faces_dt_init(int tile, int ntiles, hipStream_t q, const FaceMesh& m,
                          const FaceTileMap& tm, const Cell4* W, const double* area, double g,
                          double thr, Seg* sg) {
    const dim3 grid{unsigned(ntiles), 1u, 1u};
    if (tile == 128)
        hipLaunchKernelGGL(faces_dt_init_kernel<128>, grid, dim3(128), 0, q, m, tm, W, area, g,
                           thr, sg);
    else if (tile == 512)
        hipLaunchKernelGGL(faces_dt_init_kernel<512>, grid, dim3(512), 0, q, m, tm, W, area, g,
                           thr, sg);
    else
        hipLaunchKernelGGL(faces_dt_init_kernel<256>, grid, dim3(256), 0, q, m, tm, W, area, g,
                           thr, sg);
}

bool f32_solver(const vsw_solver* s) { return s->prm.precision == VSW_FP32; }

// State records into a new layout: cell i of the new layout takes record
// from[i] of the old one (its stage buffer too); padding cells (from < 0)
// keep what the layout gave them.
template <class R>
__global__ void move_records_kernel(int64_t n, const int64_t* __restrict__ from,
                                    const R* __restrict__ old, R* __restrict__ W,
                                    R* __restrict__ W1) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t j = from[i];
    if (j < 0) return;
    const R q = old[j];
    W[i] = q;
    W1[i] = q;
}

}  // namespace

extern "C" {

const char* vsw_last_error(void) { return g_last_error.c_str(); }

const char* vsw_version(void) { return "vsw 0.2 gfx950 fp64 fp32"; }

const char* vsw_kernel_name(int kind) {
    return (kind >= 0 && kind < KK_COUNT) ? kKernelNames[kind] : "";
}

int vsw_create(const vsw_params* p, int device, vsw_solver** out) {
    if (!p || !out) return fail(VSW_EINVAL, "NULL argument");
    *out = nullptr;
    if (!(p->g > 0.0) || !(p->g <= 0x1p100)) return fail(VSW_EINVAL, "g must be in (0, 2^100]");
    if (!(p->cfl > 0.0) || !std::isfinite(p->cfl)) return fail(VSW_EINVAL, "cfl must be > 0");
    if (!(p->h_threshold >= 0.0) || !std::isfinite(p->h_threshold))
        return fail(VSW_EINVAL, "h_threshold must be >= 0");
    if (!(p->dt_fixed >= 0.0) || !std::isfinite(p->dt_fixed))
        return fail(VSW_EINVAL, "dt_fixed must be >= 0");
    if (p->precision != VSW_FP64 && p->precision != VSW_FP32)
        return fail(VSW_EINVAL, "unsupported precision");
    if (p->ordering < VSW_ORDER_HILBERT || p->ordering > VSW_ORDER_BISECTION)
        return fail(VSW_EINVAL, "unknown ordering");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
        return fail(VSW_EDEVICE, "no HIP device");
    if (device < 0 || device >= ndev) return fail(VSW_EINVAL, "device index out of range");
    DeviceGuard dg(device);
    vsw_solver* s = new vsw_solver();
    s->prm = *p;
    s->device = device;
    // the face-parallel kernels for FP64, the cell-parallel kernel for FP32
    s->variant = VSW_KERNEL_FACES;
    hipError_t e = hipStreamCreateWithFlags(&s->own_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = s->d_ctrl.alloc(1);
    if (e != hipSuccess) {
        vsw_destroy(s);
        return fail(VSW_EDEVICE, std::string("device setup: ") + hipGetErrorString(e));
    }
    s->stream = s->own_stream;
    const int rs = resolve_scratch(device);
    if (rs != VSW_OK) {
        vsw_destroy(s);
        return rs;
    }
    // host side of the largest vsw_step_noalloc call
    s->h_logs.reserve(kScratchDoubles);
    s->seg_log.reserve(kScratchDoubles / 2);
    s->last_dts.reserve(kScratchDoubles / 2);
    s->gauge_t.reserve(kScratchDoubles / 2);
    s->gauge_eta.reserve(kScratchDoubles);
    *out = s;
    return VSW_OK;
}

void vsw_destroy(vsw_solver* s) {
    if (!s) return;
    DeviceGuard dg(s->device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    s->release_mesh();
    s->release_graph();
    s->d_log.release();
    s->d_ctrl.release();
    s->d_flag.release();
    s->d_gauge_log.release();
    for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
    if (s->own_stream) (void)hipStreamDestroy(s->own_stream);
    delete s;
}

int vsw_set_stream(vsw_solver* s, void* hip_stream) {
    if (!s) return fail(VSW_EINVAL, "NULL solver");
    s->stream = hip_stream ? (hipStream_t)hip_stream : s->own_stream;
    return VSW_OK;
}

namespace {

// Device copies of an assembled (single or ensemble) mesh.
int upload_assembled(vsw_solver* s, EnsembleMesh& em) {
    HostMesh& hm = em.hm;
    DeviceGuard dg(s->device);
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->release_mesh();
    s->nc = em.ncell;
    s->nint = hm.nc;
    s->ne = hm.ne;
    s->nw = hm.nw;
    s->nseg = em.nseg;
    s->h_seg.reserve(size_t(em.nseg));
    HIP_TRY(s->pin_t0.alloc(size_t(em.nseg)));
    HIP_TRY(s->pin_seg.alloc(size_t(em.nseg)));
    if (!s->pin_ctrl.p) HIP_TRY(s->pin_ctrl.alloc(1));
    s->seg_off = em.coff;
    s->seg_t.assign(size_t(em.nseg), 0.0);
    s->seg_dt.assign(size_t(em.nseg), 0.0);
    s->seg_steps.assign(size_t(em.nseg), 0);
    s->seg_log.clear();
    s->perm = hm.perm;
    const size_t n = size_t(hm.nc);
    const bool cellpar = (em.ftiles.tile == kTile);  // the cell-parallel kernels' layout
    HIP_TRY(s->d_perm.alloc(n));
    HIP_TRY(s->d_nbr.alloc(n));
    HIP_TRY(s->d_geom.alloc(size_t(G_NFACE) * 3 * n));
    HIP_TRY(s->d_area.alloc(n));
    HIP_TRY(s->d_perim.alloc(n));
    HIP_TRY(s->d_h.alloc(n));
    if (s->prm.precision == VSW_FP32) {
        HIP_TRY(s->d_wf[0].alloc(n));
        HIP_TRY(s->d_wf[1].alloc(n));
        HIP_TRY(s->d_w1f.alloc(n));
    } else {
        HIP_TRY(s->d_w[0].alloc(n));
        HIP_TRY(s->d_w[1].alloc(n));
        HIP_TRY(s->d_w1.alloc(n));
        // the two-pass variant's face buffer is allocated when it first runs
    }
    HIP_TRY(s->d_tmp.alloc(3 * size_t(em.ncell)));
    HIP_TRY(s->d_seg.alloc(size_t(em.nseg)));
    HIP_TRY(s->d_t0.alloc(size_t(em.nseg)));
    HIP_TRY(hipMemcpy(s->d_perm.p, hm.perm.data(), n * sizeof(int64_t), hipMemcpyHostToDevice));
    {
        std::vector<Nbr4> nb(n);
        for (size_t i = 0; i < n; ++i)
            nb[i] = Nbr4{hm.nbr[i], hm.nbr[n + i], hm.nbr[2 * n + i], 0u};
        HIP_TRY(hipMemcpy(s->d_nbr.p, nb.data(), n * sizeof(Nbr4), hipMemcpyHostToDevice));
    }
    HIP_TRY(hipMemcpy(s->d_geom.p, hm.face_geom.data(), hm.face_geom.size() * sizeof(double),
                      hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(s->d_area.p, hm.area.data(), n * sizeof(double), hipMemcpyHostToDevice));
    {
        std::vector<RGeom> rg(n);
        for (size_t i = 0; i < n; ++i)
            for (int j = 0; j < 3; ++j) {
                rg[i].w[2 * j] = hm.face_geom[(size_t(G_WX) * 3 + j) * n + i];
                rg[i].w[2 * j + 1] = hm.face_geom[(size_t(G_WY) * 3 + j) * n + i];
                rg[i].d[2 * j] = hm.face_geom[(size_t(G_DX) * 3 + j) * n + i];
                rg[i].d[2 * j + 1] = hm.face_geom[(size_t(G_DY) * 3 + j) * n + i];
            }
        HIP_TRY(s->d_rgeom.alloc(n));
        HIP_TRY(hipMemcpy(s->d_rgeom.p, rg.data(), n * sizeof(RGeom), hipMemcpyHostToDevice));
        if (s->prm.precision == VSW_FP32) {
            // rounded to nearest here, as the kernel would round each value
            std::vector<RGeomF> rf(n);
            for (size_t i = 0; i < n; ++i)
                for (int q = 0; q < 6; ++q) {
                    rf[i].w[q] = float(rg[i].w[q]);
                    rf[i].d[q] = float(rg[i].d[q]);
                }
            HIP_TRY(s->d_rgeomf.alloc(n));
            HIP_TRY(hipMemcpy(s->d_rgeomf.p, rf.data(), n * sizeof(RGeomF),
                              hipMemcpyHostToDevice));
        }
    }
    HIP_TRY(hipMemcpy(s->d_perim.p, hm.perim.data(), n * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(s->d_h.p, hm.h.data(), n * sizeof(double), hipMemcpyHostToDevice));
    // face-parallel kernels
    {
        FaceTilesHost& ft = em.ftiles;
        static_assert(sizeof(TopoRec) == sizeof(TopoD), "topology record layout");
        static_assert(sizeof(FaceItem) == sizeof(FaceItemD), "face item layout");
        std::vector<LsqW> lw(n);
        for (size_t i = 0; i < n; ++i)
            for (int j = 0; j < 3; ++j) {
                lw[i].w[2 * j] = hm.face_geom[(size_t(G_WX) * 3 + j) * n + i];
                lw[i].w[2 * j + 1] = hm.face_geom[(size_t(G_WY) * 3 + j) * n + i];
            }
        const size_t nvu = hm.vxy.size() / 2;
        HIP_TRY(s->d_topo.alloc(n));
        HIP_TRY(s->d_lsq.alloc(n));
        if (s->prm.precision == VSW_FP32) {
            // rounded to nearest here, as the FP32 kernels round each weight
            std::vector<LsqWF> lf(n);
            for (size_t i = 0; i < n; ++i)
                for (int q = 0; q < 6; ++q) lf[i].w[q] = float(lw[i].w[q]);
            HIP_TRY(s->d_lsqf.alloc(n));
            HIP_TRY(hipMemcpy(s->d_lsqf.p, lf.data(), n * sizeof(LsqWF), hipMemcpyHostToDevice));
        }
        HIP_TRY(s->d_vxy.alloc(std::max<size_t>(nvu, 1)));
        HIP_TRY(s->d_fbstart.alloc(ft.bstart.size()));
        HIP_TRY(s->d_fstart.alloc(ft.fstart.size()));
        HIP_TRY(s->d_fbitem.alloc(std::max<size_t>(ft.bitem.size(), 1)));
        HIP_TRY(s->d_fitems.alloc(std::max<size_t>(ft.items.size(), 1)));
        HIP_TRY(hipMemcpy(s->d_topo.p, ft.topo.data(), n * sizeof(TopoD), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(s->d_lsq.p, lw.data(), n * sizeof(LsqW), hipMemcpyHostToDevice));
        if (nvu)
            HIP_TRY(hipMemcpy(s->d_vxy.p, hm.vxy.data(), nvu * sizeof(double2),
                              hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(s->d_fbstart.p, ft.bstart.data(), ft.bstart.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(s->d_fstart.p, ft.fstart.data(), ft.fstart.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice));
        if (!ft.bitem.empty())
            HIP_TRY(hipMemcpy(s->d_fbitem.p, ft.bitem.data(), ft.bitem.size() * sizeof(uint32_t),
                              hipMemcpyHostToDevice));
        if (!ft.items.empty())
            HIP_TRY(hipMemcpy(s->d_fitems.p, ft.items.data(),
                              ft.items.size() * sizeof(FaceItemD), hipMemcpyHostToDevice));
        s->fbmax = ft.bmax;
        s->tile = ft.tile;
        s->ntiles = ft.ntiles;
    }
    TileMapHost& tmh = em.tiles;
    HIP_TRY(s->d_nloc.alloc(tmh.nloc.size()));
    HIP_TRY(s->d_bstart.alloc(tmh.bstart.size()));
    HIP_TRY(s->d_bitem.alloc(std::max<size_t>(tmh.bitem.size(), 1)));
    HIP_TRY(s->d_tinfo.alloc(em.tinfo.size()));
    HIP_TRY(hipMemcpy(s->d_nloc.p, tmh.nloc.data(), tmh.nloc.size() * sizeof(uint16_t),
                      hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(s->d_bstart.p, tmh.bstart.data(), tmh.bstart.size() * sizeof(int32_t),
                      hipMemcpyHostToDevice));
    if (!tmh.bitem.empty())
        HIP_TRY(hipMemcpy(s->d_bitem.p, tmh.bitem.data(), tmh.bitem.size() * sizeof(uint32_t),
                          hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(s->d_tinfo.p, em.tinfo.data(), em.tinfo.size() * sizeof(uint32_t),
                      hipMemcpyHostToDevice));
    s->bmax = tmh.bmax;
    (void)cellpar;
    s->has_mesh = true;
    s->has_state = false;
    return VSW_OK;
}

}  // namespace

namespace {

// Builds and uploads the layout of the solver's stored mesh for tiles of
// `tile` cells.
int layout_raw(vsw_solver* s, int tile) {
    EnsembleMesh em;
    std::string err;
    int rc = build_ensemble(s->raw_nseg, s->raw_nv.data(), s->raw_vx.data(), s->raw_vy.data(),
                            s->raw_nc.data(), s->raw_tri.data(), s->raw_h.data(),
                            s->prm.ordering, s->prm.seed, tile, em, err);
    if (rc != VSW_OK) return fail(rc, err);
    return upload_assembled(s, em);
}

int store_raw(vsw_solver* s, int nseg, const int64_t* nv, const double* vx, const double* vy,
              const int64_t* nc, const int32_t* tri, const double* h) {
    int64_t V = 0, C = 0;
    for (int q = 0; q < nseg; ++q) {
        if (nv[q] <= 0 || nc[q] <= 0 || nc[q] > kMaxCells || nv[q] > INT32_MAX)
            return fail(VSW_EINVAL, "scenario " + std::to_string(q) + ": empty or oversized mesh");
        V += nv[q];
        C += nc[q];
    }
    s->raw_nseg = nseg;
    s->raw_nv.assign(nv, nv + nseg);
    s->raw_nc.assign(nc, nc + nseg);
    s->raw_vx.assign(vx, vx + V);
    s->raw_vy.assign(vy, vy + V);
    s->raw_h.assign(h, h + C);
    s->raw_tri.assign(tri, tri + 3 * C);
    return VSW_OK;
}

}  // namespace

int vsw_upload_mesh(vsw_solver* s, int64_t nv, const double* vx, const double* vy, int64_t nc,
                    const int32_t* tri, const double* h) {
    if (!s) return fail(VSW_EINVAL, "NULL solver");
    if (!vx || !vy || !tri || !h) return fail(VSW_EINVAL, "NULL array");
    int rc = store_raw(s, 1, &nv, vx, vy, &nc, tri, h);
    if (rc != VSW_OK) return rc;
    return layout_raw(s, s->tile_req);
}

int vsw_upload_ensemble(vsw_solver* s, int32_t nscen, const int64_t* nv, const double* vx,
                        const double* vy, const int64_t* nc, const int32_t* tri,
                        const double* h) {
    if (!s) return fail(VSW_EINVAL, "NULL solver");
    if (nscen <= 0 || nscen > (1 << 22)) return fail(VSW_EINVAL, "bad scenario count");
    if (!vx || !vy || !tri || !h || !nv || !nc) return fail(VSW_EINVAL, "NULL array");
    int rc = store_raw(s, nscen, nv, vx, vy, nc, tri, h);
    if (rc != VSW_OK) return rc;
    return layout_raw(s, s->tile_req);
}

int vsw_set_tile_size(vsw_solver* s, int cells) {
    if (!s) return fail(VSW_EINVAL, "NULL solver");
    if (cells != 128 && cells != 256 && cells != 512)
        return fail(VSW_EINVAL, "tile size must be 128, 256 or 512");
    s->tile_req = cells;
    if (!s->has_mesh || s->tile == cells) return VSW_OK;
    // lay the mesh out again, moving the state records (as they are, in
    // either precision), the scenarios' times, the clamp count and the
    // gauges over
    DeviceGuard dg(s->device);
    const bool had_state = s->has_state;
    const bool f32 = f32_solver(s);
    const size_t rec = f32 ? sizeof(CellF) : sizeof(Cell4);
    DevBuf<unsigned char> keep;
    const std::vector<int64_t> old_perm = s->perm;
    if (had_state) {
        const size_t bytes = size_t(s->nint) * rec;
        HIP_TRY(keep.alloc(bytes));
        const void* w = f32 ? (const void*)s->d_wf[s->cur].p : (const void*)s->d_w[s->cur].p;
        HIP_TRY(hipMemcpyAsync(keep.p, w, bytes, hipMemcpyDeviceToDevice, s->stream));
        HIP_TRY(hipStreamSynchronize(s->stream));
    }
    const double t = s->t, dt_last = s->dt_last;
    const int64_t clamps = s->clamps;
    const std::vector<double> seg_t = s->seg_t, seg_dt = s->seg_dt;
    const std::vector<int32_t> gauges = s->gauge_user;
    int rc = layout_raw(s, cells);
    if (rc != VSW_OK) return rc;
    if (!gauges.empty()) {
        rc = vsw_set_gauges(s, int32_t(gauges.size()), gauges.data());
        if (rc != VSW_OK) return rc;
    }
    if (had_state) {
        // new internal index -> old internal index of the same cell
        std::vector<int64_t> inv(size_t(s->nc), -1), from(size_t(s->nint), -1);
        for (size_t i = 0; i < old_perm.size(); ++i)
            if (old_perm[i] >= 0) inv[size_t(old_perm[i])] = int64_t(i);
        for (int64_t i = 0; i < s->nint; ++i)
            if (s->perm[size_t(i)] >= 0) from[size_t(i)] = inv[size_t(s->perm[size_t(i)])];
        DevBuf<int64_t> d_from;
        HIP_TRY(d_from.alloc(from.size()));
        HIP_TRY(hipMemcpy(d_from.p, from.data(), from.size() * sizeof(int64_t),
                          hipMemcpyHostToDevice));
        const dim3 g(unsigned((s->nint + kBlock - 1) / kBlock));
        if (f32)
            hipLaunchKernelGGL(move_records_kernel<CellF>, g, dim3(kBlock), 0, s->stream, s->nint,
                               d_from.p, (const CellF*)keep.p, s->d_wf[s->cur].p, s->d_w1f.p);
        else
            hipLaunchKernelGGL(move_records_kernel<Cell4>, g, dim3(kBlock), 0, s->stream, s->nint,
                               d_from.p, (const Cell4*)keep.p, s->d_w[s->cur].p, s->d_w1.p);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(s->stream));
        s->set_time(t);
        s->dt_last = dt_last;
        s->clamps = clamps;
        s->seg_t = seg_t;
        s->seg_dt = seg_dt;
    }
    return VSW_OK;
}

int vsw_tile_size(vsw_solver* s, int* cells) {
    if (!s || !cells) return fail(VSW_EINVAL, "NULL argument");
    *cells = s->has_mesh ? s->tile : s->tile_req;
    return VSW_OK;
}

int vsw_set_state(vsw_solver* s, const double* H, const double* HU, const double* HV, double t) {
    if (!s) return fail(VSW_EINVAL, "NULL solver");
    if (!s->has_mesh) return fail(VSW_ESTATE, "no mesh uploaded");
    if (!H || !HU || !HV) return fail(VSW_EINVAL, "NULL state array");
    if (!std::isfinite(t)) return fail(VSW_EINVAL, "non-finite time");
    const int64_t nc = s->nc;
    for (int64_t k = 0; k < nc; ++k) {
        if (!std::isfinite(H[k]) || !std::isfinite(HU[k]) || !std::isfinite(HV[k]))
            return fail(VSW_EINVAL, "non-finite state value");
        if (H[k] < 0.0) return fail(VSW_EINVAL, "negative depth H");
    }
    DeviceGuard dg(s->device);
    double* tmp = s->d_tmp.p;
    HIP_TRY(hipMemcpyAsync(tmp, H, nc * sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(tmp + nc, HU, nc * sizeof(double), hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(tmp + 2 * nc, HV, nc * sizeof(double), hipMemcpyHostToDevice,
                           s->stream));
    s->pack(tmp, tmp + nc, tmp + 2 * nc);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->set_time(t);
    return VSW_OK;
}

int vsw_set_state_device(vsw_solver* s, const double* dH, const double* dHU, const double* dHV,
                         double t) {
    if (!s) return fail(VSW_EINVAL, "NULL solver");
    if (!s->has_mesh) return fail(VSW_ESTATE, "no mesh uploaded");
    if (!dH || !dHU || !dHV) return fail(VSW_EINVAL, "NULL state array");
    if (!std::isfinite(t)) return fail(VSW_EINVAL, "non-finite time");
    DeviceGuard dg(s->device);
    // checked on the device before anything is written
    if (!s->d_flag.p) HIP_TRY(s->d_flag.alloc(1));
    const int zero = 0;
    HIP_TRY(hipMemcpyAsync(s->d_flag.p, &zero, sizeof(int), hipMemcpyHostToDevice, s->stream));
    hipLaunchKernelGGL(check_state_kernel, dim3(grid_for(s->nc)), dim3(kBlock), 0, s->stream,
                       s->nc, dH, dHU, dHV, s->d_flag.p);
    HIP_TRY(hipGetLastError());
    int flag = 0;
    HIP_TRY(hipMemcpyAsync(&flag, s->d_flag.p, sizeof(int), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (flag & 1) return fail(VSW_EINVAL, "non-finite state value");
    if (flag & 2) return fail(VSW_EINVAL, "negative depth H");
    s->pack(dH, dHU, dHV);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s->stream));
    s->set_time(t);
    return VSW_OK;
}

int vsw_get_state(vsw_solver* s, double* H, double* HU, double* HV, double* t) {
    if (!s) return fail(VSW_EINVAL, "NULL solver");
    if (!s->has_state) return fail(VSW_ESTATE, "no state");
    DeviceGuard dg(s->device);
    const int64_t nc = s->nc;
    double* tmp = s->d_tmp.p;
    s->unpack(tmp, tmp + nc, tmp + 2 * nc);
    HIP_TRY(hipGetLastError());
    double* dst[3] = {H, HU, HV};
    for (int c = 0; c < 3; ++c)
        if (dst[c])
            HIP_TRY(hipMemcpyAsync(dst[c], tmp + c * nc, nc * sizeof(double),
                                   hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (t) *t = s->t;
    return VSW_OK;
}

int vsw_get_state_device(vsw_solver* s, double* dH, double* dHU, double* dHV, double* t) {
    if (!s) return fail(VSW_EINVAL, "NULL solver");
    if (!s->has_state) return fail(VSW_ESTATE, "no state");
    DeviceGuard dg(s->device);
    s->unpack(dH, dHU, dHV);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s->stream));
    if (t) *t = s->t;
    return VSW_OK;
}

}  // extern "C"

namespace {

// The step loop of vsw_step and vsw_step_noalloc: n steps with the step log
// in lg (2 n nseg doubles) and the gauge records in glog (n ngauges
// doubles).  noalloc: no device or host memory is allocated (the two-pass
// face buffer must exist), no graph is captured and no profiling events are
// recorded.
int step_impl(vsw_solver* s, int64_t n, double t_stop, int64_t* steps_done, double* t_out,
              double* lg, double* glog, bool noalloc) {
    const int nseg = s->nseg;
    const size_t nlog = size_t(n) * size_t(nseg);
    const int ng = s->ngauges;
    const DevMesh m = s->dev_mesh();
    StepParams p;
    p.g = s->prm.g;
    p.hg = 0.5 * s->prm.g;
    p.thr = s->prm.h_threshold;
    p.cfl = s->prm.cfl;
    p.dt_fixed = s->prm.dt_fixed;
    p.t_stop = t_stop;
    Cell4* Wa = s->d_w[0].p;
    Cell4* Wb = s->d_w[1].p;
    Cell4* W1 = s->d_w1.p;
    if (!f32_solver(s) && s->variant == VSW_KERNEL_TWO_PASS && !s->d_face.p) {
        if (noalloc)
            return fail(VSW_EINVAL, "the two-pass kernels' face buffer is not allocated yet");
        const size_t nn = size_t(s->nint);
        HIP_TRY(s->d_face.alloc(15 * nn));
        HIP_TRY(s->d_sc.alloc(2 * nn));
        HIP_TRY(s->d_order.alloc(nn));
    }
    FaceBuf fb{s->d_face.p, s->d_sc.p, s->d_order.p};
    Ctrl* c = s->d_ctrl.p;
    Seg* sg = s->d_seg.p;
    const dim3 grid(unsigned(s->ntiles)), block(kBlock);
    hipStream_t st = s->stream;
    TileMap tm{s->d_nloc.p, s->d_bstart.p, s->d_bitem.p, s->d_tinfo.p, s->bmax, s->ntiles, nseg,
               s->xcd_order};
    const bool f32 = (s->prm.precision == VSW_FP32);
    const bool faces = s->variant == VSW_KERNEL_FACES;
    if (!faces && s->tile != kTile)
        return fail(VSW_EINVAL, "this kernel variant needs tiles of 256 cells");
    const size_t lds = capped_lds(stage_lds_bytes(s->bmax), s->occupancy);
    const size_t lds32 = capped_lds(stage_f32_lds_bytes(s->bmax), s->occupancy);
    const size_t ldsf = capped_lds(faces_lds_bytes(s->tile, s->fbmax), s->occupancy);
    if (faces) {
        int maxlds = 0;
        HIP_TRY(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock,
                                      s->device));
        if (ldsf > size_t(maxlds))
            return fail(VSW_EINVAL, "tile too large for the LDS of a workgroup (" +
                                        std::to_string(ldsf) + " > " + std::to_string(maxlds) +
                                        " bytes)");
    }
    const FaceMesh fm = s->face_mesh();
    const FaceTileMap ftm = s->face_tiles(nseg);

    // profiling events: one pair per timed launch
    size_t ev_used = 0;
    bool prof = s->profiling && !noalloc;
    auto ev_begin = [&](int kind, hipStream_t q) {
        if (!prof) return;
        if (ev_used + 2 > s->ev_pool.size()) {
            for (int i = 0; i < 64; ++i) {
                hipEvent_t e;
                if (hipEventCreate(&e) != hipSuccess) break;
                s->ev_pool.push_back(e);
            }
        }
        if (ev_used + 2 > s->ev_pool.size()) return;
        (void)hipEventRecord(s->ev_pool[ev_used], q);
        if (s->ev_kind.size() < s->ev_pool.size() / 2 + 1) s->ev_kind.resize(s->ev_pool.size() / 2 + 1);
        s->ev_kind[ev_used / 2] = kind;
    };
    auto ev_end = [&](hipStream_t q) {
        if (!prof || ev_used + 2 > s->ev_pool.size()) return;
        (void)hipEventRecord(s->ev_pool[ev_used + 1], q);
        ev_used += 2;
    };
    // One step on stream q with control slot `slot`; its index is the
    // device step base plus sa (which also picks the state buffers).
    auto launch_step = [&](hipStream_t q, int slot, int sa) {
        const dim3 gg(unsigned((ng + 63) / 64));
        if (f32) {
            CellF* Fa = s->d_wf[0].p;
            CellF* Fb = s->d_wf[1].p;
            for (int stage = 1; stage <= 2; ++stage) {
                ev_begin(stage == 1 ? KK_STAGE1 : KK_STAGE2, q);
                if (faces)
                    launch_faces_stage_f32(s->tile, stage, s->ntiles, ldsf, q, fm, ftm, s->d_h.p,
                                           Fa, Fb, s->d_w1f.p, p, c, sg, slot, sa, lg);
                else if (stage == 1)
                    hipLaunchKernelGGL(stage_f32_kernel<1>, grid, block, lds32, q, m, tm, Fa, Fb,
                                       s->d_w1f.p, p, c, sg, slot, sa, lg);
                else
                    hipLaunchKernelGGL(stage_f32_kernel<2>, grid, block, lds32, q, m, tm, Fa, Fb,
                                       s->d_w1f.p, p, c, sg, slot, sa, lg);
                ev_end(q);
            }
            if (ng > 0)
                hipLaunchKernelGGL(gauge_f32_kernel, gg, dim3(64), 0, q, Fa, Fb, s->d_h.p,
                                   s->d_gauge_cells.p, ng, s->d_gauge_seg.p, sg, c, sa, glog);
            return;
        }
        if (faces) {
            ev_begin(KK_STAGE1, q);
            launch_faces_stage(s->tile, 1, s->ntiles, ldsf, q, fm, ftm, Wa, Wb, W1, p, c, sg,
                               slot, sa, lg);
            ev_end(q);
            ev_begin(KK_STAGE2, q);
            launch_faces_stage(s->tile, 2, s->ntiles, ldsf, q, fm, ftm, Wa, Wb, W1, p, c, sg,
                               slot, sa, lg);
            ev_end(q);
        } else if (s->variant == VSW_KERNEL_FUSED) {
            ev_begin(KK_STAGE1, q);
            hipLaunchKernelGGL(stage_kernel<1>, grid, block, lds, q, m, tm, Wa, Wb, W1, p, c, sg,
                               slot, sa, lg);
            ev_end(q);
            ev_begin(KK_STAGE2, q);
            hipLaunchKernelGGL(stage_kernel<2>, grid, block, lds, q, m, tm, Wa, Wb, W1, p, c, sg,
                               slot, sa, lg);
            ev_end(q);
        } else {
            ev_begin(KK_RECON, q);
            hipLaunchKernelGGL(recon_kernel<1>, grid, block, 0, q, m, tm, Wa, Wb, W1, fb, p, c,
                               sg, slot, sa);
            ev_end(q);
            ev_begin(KK_UPDATE1, q);
            hipLaunchKernelGGL(update1_kernel, grid, block, 0, q, m, tm, Wa, Wb, W1, fb, p, c, sg,
                               slot, sa);
            ev_end(q);
            ev_begin(KK_RECON, q);
            hipLaunchKernelGGL(recon_kernel<2>, grid, block, 0, q, m, tm, Wa, Wb, W1, fb, p, c,
                               sg, slot, sa);
            ev_end(q);
            ev_begin(KK_UPDATE2, q);
            hipLaunchKernelGGL(update2_kernel, grid, block, 0, q, m, tm, Wa, Wb, W1, fb, p, c, sg,
                               slot, sa, lg);
            ev_end(q);
        }
        if (ng > 0)
            hipLaunchKernelGGL(gauge_kernel, gg, dim3(64), 0, q, Wa, Wb, s->d_gauge_cells.p, ng,
                               s->d_gauge_seg.p, sg, c, sa, glog);
    };

    // Graph mode: a captured pair of steps followed by a step-base bump,
    // replayed n / 2 times (kernel nodes only).  Rebuilt when anything baked
    // into its launch arguments changes.  The state buffers a step uses follow
    // from the device step index and the call's parity, so one capture
    // serves every call.
    // Graph mode 2: the whole call (n steps, direct step indices) captured
    // as one graph, launched once.
    const int gmode = (prof || noalloc) ? 0 : s->graph_mode;
    const bool whole = gmode == 2 && n <= kWholeGraphMaxSteps;
    const bool use_graph = (gmode == 1 || (gmode == 2 && !whole)) && n >= 2;
    if (use_graph || whole) {
        const GraphKey key{lg, glog, s->d_gauge_cells.p, ng, t_stop,
                           ((s->variant * 2 + s->xcd_order) * 8 + s->occupancy) * 1024 + s->tile,
                           whole ? n : 0};
        if (!s->graph_exec || !(key == s->graph_key)) {
            s->release_graph();
            prof = false;
            hipStream_t cs = s->own_stream;
            HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            if (whole) {
                for (int64_t k = 0; k < n; ++k) launch_step(cs, int(k & 1), int(k));
            } else {
                launch_step(cs, 0, 0);
                launch_step(cs, 1, 1);
                hipLaunchKernelGGL(step_bump_kernel, dim3(1), dim3(64), 0, cs, c, 2);
            }
            hipGraph_t g = nullptr;
            const hipError_t ec = hipStreamEndCapture(cs, &g);
            if (ec != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return fail(VSW_EDEVICE, std::string("graph capture: ") + hipGetErrorString(ec));
            }
            s->graph = g;
            HIP_TRY(hipGraphInstantiate(&s->graph_exec, g, nullptr, nullptr, 0));
            s->graph_key = key;
        }
    }

    std::copy(s->seg_t.begin(), s->seg_t.end(), s->pin_t0.p);
    HIP_TRY(hipMemcpyAsync(s->d_t0.p, s->pin_t0.p, size_t(nseg) * sizeof(double),
                           hipMemcpyHostToDevice, st));
    // the previous call's last step left the CFL minimum of this state
    const int keep = s->rmin_slot;
    hipLaunchKernelGGL(ctrl_init_kernel, dim3(1), dim3(256), 0, st, c, sg, nseg, s->d_t0.p,
                       s->cur, keep);
    if (keep < 0) ev_begin(KK_DTINIT, st);
    if (keep >= 0) {
    } else if (f32 && faces)
        launch_faces_dt_init_f32(s->tile, s->ntiles, st, fm, ftm, s->d_wf[s->cur].p, s->d_h.p,
                                 s->d_area.p, p.g, p.thr, sg);
    else if (f32)
        hipLaunchKernelGGL(dt_init_f32_kernel, grid, block, 0, st, m, tm, s->d_wf[s->cur].p, p.g,
                           p.thr, sg);
    else if (faces)
        launch_faces_dt_init(s->tile, s->ntiles, st, fm, ftm, s->d_w[s->cur].p, s->d_area.p, p.g,
                             p.thr, sg);
    else
        hipLaunchKernelGGL(dt_init_kernel, grid, block, 0, st, m, tm, s->d_w[s->cur].p, p.g,
                           p.thr, sg);
    if (keep < 0) ev_end(st);
    if (whole) {
        HIP_TRY(hipGraphLaunch(s->graph_exec, st));
    } else if (use_graph) {
        for (int64_t k = 0; k + 1 < n; k += 2) HIP_TRY(hipGraphLaunch(s->graph_exec, st));
        if (n & 1) launch_step(st, 0, 0);  // the base is n - 1 here
    } else {
        for (int64_t k = 0; k < n; ++k) launch_step(st, int(k & 1), int(k));
    }
    HIP_TRY(hipGetLastError());
    // read back into pinned buffers (the step log into the pageable copy
    // when the pinned one is too small and may not grow here)
    if (!noalloc && s->pin_logs.n < 2 * nlog)
        HIP_TRY(s->pin_logs.alloc(std::max({2 * nlog, 2 * s->pin_logs.n, kLogMinSteps * 2 *
                                                                         size_t(nseg)})));
    const bool pinned_log = s->pin_logs.n >= 2 * nlog;
    HIP_TRY(hipMemcpyAsync(s->pin_ctrl.p, c, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(s->pin_seg.p, sg, size_t(nseg) * sizeof(Seg), hipMemcpyDeviceToHost,
                           st));
    std::vector<double>& logs = s->h_logs;
    logs.resize(2 * nlog);
    HIP_TRY(hipMemcpyAsync(pinned_log ? s->pin_logs.p : logs.data(), lg,
                           2 * nlog * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    const Ctrl hc = *s->pin_ctrl.p;
    std::vector<Seg>& hs = s->h_seg;
    hs.assign(s->pin_seg.p, s->pin_seg.p + nseg);
    if (pinned_log) std::copy(s->pin_logs.p, s->pin_logs.p + 2 * nlog, logs.begin());
    if (s->profiling) {
        for (size_t i = 0; i + 1 < ev_used; i += 2) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, s->ev_pool[i], s->ev_pool[i + 1]) == hipSuccess) {
                const int kind = s->ev_kind[i / 2];
                s->prof_ms[kind] += ms;
                s->prof_n[kind] += 1;
            }
        }
    }
    // A scenario's steps are a prefix of the call (once it stops it takes no
    // later step); on an error, only the steps before the failing one count.
    int rc = VSW_OK;
    int64_t cap = n;
    if (hc.err) {
        cap = hc.err_step;
        rc = fail(VSW_EUNSTABLE, (hc.err & 1) ? "non-finite state" : "no valid time step");
    }
    // every step before the failing one (all n without an error) moved the
    // state to the other buffer; the failing step's input stays where it is
    s->cur ^= int(cap & 1);
    int64_t done = 0;
    double tmin = INFINITY;
    s->seg_log.resize(nlog);
    for (size_t e = 0; e < nlog; ++e) s->seg_log[e] = logs[2 * e + 1];
    for (int q = 0; q < nseg; ++q) {
        const int64_t d = std::min<int64_t>(hs[q].steps_done, cap);
        s->seg_steps[q] = d;
        if (d > 0) {
            s->seg_t[q] = logs[2 * (size_t(d - 1) * nseg + q)];
            s->seg_dt[q] = logs[2 * (size_t(d - 1) * nseg + q) + 1];
        }
        done = std::max(done, d);
        tmin = std::min(tmin, s->seg_t[q]);
    }
    s->clamps += int64_t(hc.clamps);
    s->last_dts.resize(size_t(s->seg_steps[0]));
    for (int64_t k = 0; k < s->seg_steps[0]; ++k) s->last_dts[k] = s->seg_log[size_t(k) * nseg];
    s->gauge_t.assign(size_t(done), s->seg_t[0]);
    for (int64_t k = 0; k < std::min(done, s->seg_steps[0]); ++k)
        s->gauge_t[k] = logs[2 * size_t(k) * nseg];
    s->gauge_eta.assign(size_t(done) * size_t(ng), 0.0);
    if (ng > 0 && done > 0)
        HIP_TRY(hipMemcpy(s->gauge_eta.data(), glog, size_t(done) * size_t(ng) * sizeof(double),
                          hipMemcpyDeviceToHost));
    s->t = tmin;
    s->dt_last = s->seg_dt[0];
    // every scenario took every step: the last one left the CFL minimum of
    // the state the next call starts from in slot n & 1
    bool all = !hc.err;
    for (int q = 0; q < nseg; ++q) all = all && (s->seg_steps[q] == n);
    s->rmin_slot = all ? int(n & 1) : -1;
    if (steps_done) *steps_done = done;
    if (t_out) *t_out = s->t;
    return rc;
}

// Argument checks shared by vsw_step and vsw_step_noalloc; 1 when there is
// nothing to do (n = 0).
int step_args(vsw_solver* s, int64_t n, double t_stop, int64_t* steps_done, double* t_out) {
    if (!s) return fail(VSW_EINVAL, "NULL solver");
    if (!s->has_mesh || !s->has_state) return fail(VSW_ESTATE, "mesh and state required");
    if (n < 0) return fail(VSW_EINVAL, "negative step count");
    if (std::isnan(t_stop)) return fail(VSW_EINVAL, "t_stop is NaN");
    if (n > INT32_MAX) return fail(VSW_EINVAL, "too many steps in one call");
    if (steps_done) *steps_done = 0;
    if (t_out) *t_out = s->t;
    return (n == 0) ? 1 : VSW_OK;
}

}  // namespace

extern "C" {

int vsw_step(vsw_solver* s, int64_t n, double t_stop, int64_t* steps_done, double* t_out) {
    const int a = step_args(s, n, t_stop, steps_done, t_out);
    if (a != VSW_OK) return (a == 1) ? VSW_OK : a;
    DeviceGuard dg(s->device);
    const size_t nlog = size_t(n) * size_t(s->nseg);
    // logs grow by doubling from room for kLogMinSteps steps, so that short
    // calls (a benchmark's timed call after a shorter warm-up) allocate
    // nothing
    if (s->d_log.n < 2 * nlog)
        HIP_TRY(s->d_log.alloc(std::max({2 * nlog, 2 * s->d_log.n,
                                         kLogMinSteps * 2 * size_t(s->nseg)})));
    const int ng = s->ngauges;
    if (ng > 0 && s->d_gauge_log.n < size_t(n) * size_t(ng))
        HIP_TRY(s->d_gauge_log.alloc(std::max({size_t(n) * size_t(ng), 2 * s->d_gauge_log.n,
                                               kLogMinSteps * size_t(ng)})));
    return step_impl(s, n, t_stop, steps_done, t_out, s->d_log.p, s->d_gauge_log.p, false);
}

int vsw_step_noalloc(vsw_solver* s, int64_t n, double t_stop, int64_t* steps_done,
                     double* t_out) {
    const int a = step_args(s, n, t_stop, steps_done, t_out);
    if (a != VSW_OK) return (a == 1) ? VSW_OK : a;
    const size_t need = size_t(n) * (2 * size_t(s->nseg) + size_t(s->ngauges));
    if (need > kScratchDoubles)
        return fail(VSW_EINVAL, "vsw_step_noalloc: n * (2 scenarios + gauges) = " +
                                    std::to_string(need) + " doubles exceeds its " +
                                    std::to_string(kScratchDoubles) + "-double array");
    DeviceGuard dg(s->device);
    double* sp = scratch_ptr(s->device);
    if (!sp) return fail(VSW_EDEVICE, "no-allocation scratch array not resolved");
    // the step log first, the gauge records after it
    return step_impl(s, n, t_stop, steps_done, t_out, sp, sp + 2 * size_t(n) * size_t(s->nseg),
                     true);
}

int vsw_scenario_count(vsw_solver* s, int32_t* nscen) {
    if (!s || !nscen) return fail(VSW_EINVAL, "NULL argument");
    if (!s->has_mesh) return fail(VSW_ESTATE, "no mesh uploaded");
    *nscen = s->nseg;
    return VSW_OK;
}

int vsw_scenario_status(vsw_solver* s, int32_t max, double* t, double* dt_last,
                        int64_t* steps) {
    if (!s) return fail(VSW_EINVAL, "NULL solver");
    if (!s->has_mesh) return fail(VSW_ESTATE, "no mesh uploaded");
    const int m = std::min<int>(max, s->nseg);
    for (int q = 0; q < m; ++q) {
        if (t) t[q] = s->seg_t[q];
        if (dt_last) dt_last[q] = s->seg_dt[q];
        if (steps) steps[q] = s->seg_steps[q];
    }
    return VSW_OK;
}

int vsw_scenario_dt_history(vsw_solver* s, int32_t scen, int64_t max, double* dts,
                            int64_t* count) {
    if (!s || !count) return fail(VSW_EINVAL, "NULL argument");
    if (!s->has_mesh) return fail(VSW_ESTATE, "no mesh uploaded");
    if (scen < 0 || scen >= s->nseg) return fail(VSW_EINVAL, "scenario index out of range");
    const int64_t n = s->seg_log.empty() ? 0 : s->seg_steps[scen];
    *count = n;
    if (dts)
        for (int64_t k = 0; k < n && k < max; ++k)
            dts[k] = s->seg_log[size_t(k) * s->nseg + scen];
    return VSW_OK;
}

int vsw_adjoint_gauge_loss(vsw_solver* s, int64_t nsteps, int64_t ckpt, int32_t ng,
                           const int32_t* gauge_cells, const double* eta_obs, double* loss,
                           double* gH, double* gHU, double* gHV, double* gh) {
    if (!s) return fail(VSW_EINVAL, "NULL solver");
    if (!s->has_mesh || !s->has_state) return fail(VSW_ESTATE, "mesh and state required");
    if (s->nseg != 1) return fail(VSW_EINVAL, "the adjoint takes a single scenario");
    if (s->tile != kTile) return fail(VSW_EINVAL, "the adjoint needs tiles of 256 cells");
    // FP32 solvers: FP32 forward and replay, FP64 adjoint on their trajectory
    const bool f32 = (s->prm.precision == VSW_FP32);
    if (nsteps < 1 || nsteps > INT32_MAX || ckpt < 1)
        return fail(VSW_EINVAL, "bad step or checkpoint count");
    if (ng < 1 || !gauge_cells || !eta_obs || !loss) return fail(VSW_EINVAL, "NULL argument");
    DeviceGuard dg(s->device);
    hipStream_t st = s->stream;
    HIP_TRY(hipStreamSynchronize(st));
    const int64_t n = s->nint;
    const int64_t nck = (nsteps + ckpt - 1) / ckpt;
    const int64_t segl = std::min(ckpt, nsteps);
    // the caller's solver state, restored on return
    const std::vector<int32_t> user_gauge_cells = s->gauge_user;
    std::vector<int64_t> user_gauges(size_t(s->ngauges));
    if (s->ngauges > 0)
        HIP_TRY(hipMemcpy(user_gauges.data(), s->d_gauge_cells.p,
                          user_gauges.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
    const double t_save = s->t, dt_save = s->dt_last;
    const int64_t clamps_save = s->clamps;
    const std::vector<double> seg_t_save = s->seg_t, seg_dt_save = s->seg_dt;
    const std::vector<int64_t> seg_steps_save = s->seg_steps;
    const std::vector<double> seg_log_save = s->seg_log, last_dts_save = s->last_dts;
    // state records of the solver's precision: the current one and stage 1
    const size_t rec = f32 ? sizeof(CellF) : sizeof(Cell4);
    auto wcur = [&]() { return f32 ? (void*)s->d_wf[s->cur].p : (void*)s->d_w[s->cur].p; };
    void* const w1buf = f32 ? (void*)s->d_w1f.p : (void*)s->d_w1.p;
    DevBuf<unsigned char> W0, ck;
    DevBuf<Cell4> seg;
    HIP_TRY(W0.alloc(size_t(n) * rec));
    HIP_TRY(hipMemcpyAsync(W0.p, wcur(), size_t(n) * rec, hipMemcpyDeviceToDevice, st));
    auto restore = [&]() {
        (void)hipMemcpyAsync(wcur(), W0.p, size_t(n) * rec, hipMemcpyDeviceToDevice, st);
        (void)hipMemcpyAsync(w1buf, W0.p, size_t(n) * rec, hipMemcpyDeviceToDevice, st);
        (void)hipStreamSynchronize(st);
        s->t = t_save;
        s->dt_last = dt_save;
        s->clamps = clamps_save;
        s->seg_t = seg_t_save;
        s->seg_dt = seg_dt_save;
        s->seg_steps = seg_steps_save;
        s->seg_log = seg_log_save;
        s->last_dts = last_dts_save;
        s->rmin_slot = -1;
        // the adjoint takes a single scenario: every gauge is in scenario 0
        const std::vector<int32_t> zeros(user_gauges.size(), 0);
        const bool ok = s->d_gauge_cells.alloc(user_gauges.size()) == hipSuccess &&
                        s->d_gauge_seg.alloc(user_gauges.size()) == hipSuccess;
        if (ok && !user_gauges.empty()) {
            (void)hipMemcpy(s->d_gauge_cells.p, user_gauges.data(),
                            user_gauges.size() * sizeof(int64_t), hipMemcpyHostToDevice);
            (void)hipMemcpy(s->d_gauge_seg.p, zeros.data(), zeros.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice);
        }
        s->ngauges = ok ? int(user_gauges.size()) : 0;
        s->gauge_user = ok ? user_gauge_cells : std::vector<int32_t>();
        s->gauge_eta.clear();
        s->gauge_t.clear();
        s->release_graph();
    };
    // the caller's state, time, gauges and logs come back on every return path
    const auto restore_on_exit = on_exit(restore);
    int rc = vsw_set_gauges(s, ng, gauge_cells);
    if (rc != VSW_OK) return rc;
    // ---- forward with checkpoints and gauge records
    if (ck.alloc(size_t(nck) * size_t(n) * rec) != hipSuccess)
        return fail(VSW_ENOMEM, "checkpoint memory");
    std::vector<double> dts, eta;
    for (int64_t c = 0; c < nck; ++c) {
        HIP_TRY(hipMemcpyAsync(ck.p + size_t(c) * size_t(n) * rec, wcur(), size_t(n) * rec,
                               hipMemcpyDeviceToDevice, st));
        const int64_t m = std::min(ckpt, nsteps - c * ckpt);
        int64_t done = 0;
        rc = vsw_step(s, m, INFINITY, &done, nullptr);
        if (rc != VSW_OK || done != m)
            return fail(rc != VSW_OK ? rc : VSW_EUNSTABLE, "forward run: " + g_last_error);
        dts.insert(dts.end(), s->last_dts.begin(), s->last_dts.end());
        eta.insert(eta.end(), s->gauge_eta.begin(), s->gauge_eta.end());
    }
    const double thr = s->prm.h_threshold, g = s->prm.g, hg = 0.5 * g, cfl = s->prm.cfl;
    const bool cfl_dt = !(s->prm.dt_fixed > 0.0);
    std::vector<double> r(size_t(nsteps) * size_t(ng));
    double L = 0.0;
    for (size_t i = 0; i < r.size(); ++i) {
        r[i] = eta[i] - eta_obs[i];
        L += r[i] * r[i];
    }
    *loss = L;
    // ---- reverse sweep
    // Per segment of L steps the stage kernels replay the steps from the
    // checkpoint with the forward's dts (bitwise the forward's states) and
    // record the tape: the states w and w1 of every step, both stages' residuals and
    // fix masks, and the CFL minimum of each state.
    const size_t N = size_t(n), SL = size_t(segl);
    DevBuf<Cell4> segW1, wend;
    DevBuf<double> d_r, tR0, tR1, mua, partA, partB, gout;
    DevBuf<uint8_t> tm1, tm2;
    DevBuf<Adj4> lam, lamn, cown, cx;
    DevBuf<int32_t> xin;
    DevBuf<unsigned long long> rmin_hist, argmin;
    hipError_t e = hipSuccess;
    DevBuf<CellF> fA, fB, f1;  // FP32 replay buffers
    if (f32) {
        for (hipError_t x : {fA.alloc(N), fB.alloc(N), f1.alloc(N)})
            if (x != hipSuccess) return fail(VSW_ENOMEM, "adjoint work memory");
    }
    for (hipError_t x : {d_r.alloc(r.size()), seg.alloc(SL * N), segW1.alloc(SL * N),
                         wend.alloc(f32 ? 1 : N), tR0.alloc(3 * SL * N), tR1.alloc(3 * SL * N),
                         tm1.alloc(SL * N), tm2.alloc(SL * N), rmin_hist.alloc(SL + 1), argmin.alloc(1),
                         lam.alloc(N), lamn.alloc(N), mua.alloc(3 * N), cown.alloc(N),
                         cx.alloc(s->d_bitem.n), xin.alloc(3 * N),
                         partA.alloc(size_t(s->ntiles)), partB.alloc(size_t(s->ntiles)),
                         gout.alloc(4 * size_t(s->nc))})
        if (x != hipSuccess) e = x;
    if (e != hipSuccess) return fail(VSW_ENOMEM, "adjoint work memory");
    HIP_TRY(hipMemcpy(d_r.p, r.data(), r.size() * sizeof(double), hipMemcpyHostToDevice));
    HIP_TRY(hipMemsetAsync(lam.p, 0, N * sizeof(Adj4), st));
    const DevMesh m = s->dev_mesh();
    TileMap tm{s->d_nloc.p, s->d_bstart.p, s->d_bitem.p, s->d_tinfo.p, s->bmax, s->ntiles, 1,
               s->xcd_order};
    const dim3 grid(unsigned(s->ntiles)), block(kBlock);
    HIP_TRY(hipMemsetAsync(xin.p, 0xFF, 3 * N * sizeof(int32_t), st));
    hipLaunchKernelGGL(adj_xin_kernel, grid, block, 0, st, tm, int64_t(N), xin.p);
    const AdjC cc{cown.p, cx.p, xin.p};
    int64_t* cells = s->d_gauge_cells.p;
    const size_t lds = stage_lds_bytes(s->bmax), lds32 = stage_f32_lds_bytes(s->bmax);
    // the replay of an FP64 run uses the face-parallel kernels unless the
    // solver runs the cell-parallel ones (both record the same tape)
    const bool faces = (s->variant == VSW_KERNEL_FACES);
    const FaceMesh fm = s->face_mesh();
    const FaceTileMap ftm = s->face_tiles(1);
    const size_t ldsf = faces_lds_bytes(kTile, s->fbmax);
    const double zero_t = 0.0;
    HIP_TRY(hipMemcpy(s->d_t0.p, &zero_t, sizeof(double), hipMemcpyHostToDevice));
    if (s->d_log.n < 2) HIP_TRY(s->d_log.alloc(2));
    const std::vector<unsigned long long> inf_bits(SL + 1, 0x7FF0000000000000ull);
    // the misfit of the last state
    hipLaunchKernelGGL(adj_gauge_kernel, dim3(1), dim3(64), 0, st, cells, ng,
                       d_r.p + (nsteps - 1) * ng, lam.p);
    for (int64_t c = nck - 1; c >= 0; --c) {
        const int64_t n0 = c * ckpt, n1 = std::min(nsteps, n0 + ckpt);
        const int64_t len = n1 - n0;
        if (cfl_dt)
            HIP_TRY(hipMemcpyAsync(rmin_hist.p, inf_bits.data(), (SL + 1) * sizeof(inf_bits[0]),
                                   hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(ctrl_init_kernel, dim3(1), dim3(256), 0, st, s->d_ctrl.p, s->d_seg.p,
                           1, s->d_t0.p, 0, -1);
        const unsigned char* ckc = ck.p + size_t(c) * N * rec;
        if (!f32) {
            HIP_TRY(hipMemcpyAsync(seg.p, ckc, N * sizeof(Cell4), hipMemcpyDeviceToDevice, st));
            if (cfl_dt)
                hipLaunchKernelGGL(adj_rmin_kernel, grid, block, 0, st, m, tm, seg.p, g, thr,
                                   rmin_hist.p);
            for (int64_t i = 0; i < len; ++i) {
                Cell4* Wi = seg.p + i * n;
                Cell4* W1i = segW1.p + i * n;
                const StepParams p{g, hg, thr, cfl, dts[size_t(n0 + i)], INFINITY};
                Cell4* Wo = (i + 1 < len) ? Wi + n : wend.p;
                const Tape t1{tR0.p + 3 * i * n, tm1.p + i * n, nullptr};
                const Tape t2{tR1.p + 3 * i * n, tm2.p + i * n, rmin_hist.p + i + 1};
                if (faces) {
                    hipLaunchKernelGGL((faces_tape_kernel<256, 1>), grid, block, ldsf, st, fm, ftm,
                                       Wi, Wo, W1i, p, s->d_ctrl.p, s->d_seg.p, 0, 0, s->d_log.p,
                                       t1);
                    hipLaunchKernelGGL((faces_tape_kernel<256, 2>), grid, block, ldsf, st, fm, ftm,
                                       Wi, Wo, W1i, p, s->d_ctrl.p, s->d_seg.p, 0, 0, s->d_log.p,
                                       t2);
                } else {
                    hipLaunchKernelGGL(stage_tape_kernel<1>, grid, block, lds, st, m, tm, Wi, Wo,
                                       W1i, p, s->d_ctrl.p, s->d_seg.p, 0, 0, s->d_log.p, t1);
                    hipLaunchKernelGGL(stage_tape_kernel<2>, grid, block, lds, st, m, tm, Wi, Wo,
                                       W1i, p, s->d_ctrl.p, s->d_seg.p, 0, 0, s->d_log.p, t2);
                }
            }
        } else {
            // the FP32 steps again from the FP32 checkpoint; the tape holds
            // the states they reconstruct as FP64 records
            HIP_TRY(hipMemcpyAsync(fA.p, ckc, N * sizeof(CellF), hipMemcpyDeviceToDevice, st));
            for (int64_t i = 0; i < len; ++i) {
                CellF* Fi = (i & 1) ? fB.p : fA.p;
                CellF* Fo = (i & 1) ? fA.p : fB.p;
                const StepParams p{g, hg, thr, cfl, dts[size_t(n0 + i)], INFINITY};
                const TapeF t1{tR0.p + 3 * i * n, tm1.p + i * n, nullptr, seg.p + i * n};
                const TapeF t2{tR1.p + 3 * i * n, tm2.p + i * n, rmin_hist.p + i + 1,
                               segW1.p + i * n};
                if (faces) {
                    hipLaunchKernelGGL((faces_tape_f32_kernel<256, 1>), grid, block, ldsf, st, fm,
                                       ftm, s->d_h.p, Fi, Fo, f1.p, p, s->d_ctrl.p, s->d_seg.p, 0,
                                       0, s->d_log.p, t1);
                    hipLaunchKernelGGL((faces_tape_f32_kernel<256, 2>), grid, block, ldsf, st, fm,
                                       ftm, s->d_h.p, Fi, Fo, f1.p, p, s->d_ctrl.p, s->d_seg.p, 0,
                                       0, s->d_log.p, t2);
                } else {
                    hipLaunchKernelGGL(stage_f32_tape_kernel<1>, grid, block, lds32, st, m, tm, Fi,
                                       Fo, f1.p, p, s->d_ctrl.p, s->d_seg.p, 0, 0, s->d_log.p, t1);
                    hipLaunchKernelGGL(stage_f32_tape_kernel<2>, grid, block, lds32, st, m, tm, Fi,
                                       Fo, f1.p, p, s->d_ctrl.p, s->d_seg.p, 0, 0, s->d_log.p, t2);
                }
            }
            if (cfl_dt)
                hipLaunchKernelGGL(adj_rmin_kernel, grid, block, 0, st, m, tm, seg.p, g, thr,
                                   rmin_hist.p);
        }
        bool started = false;  // the start of step k was done by the previous turn
        // per-tile dt adjoint terms of step k (part) and of step k-1 (partn)
        double *part = partA.p, *partn = partB.p;
        for (int64_t k = n1 - 1; k >= n0; --k) {
            const int64_t i = k - n0;
            const Cell4* Wn = seg.p + i * n;
            const Cell4* W1 = segW1.p + i * n;
            const double* R0 = tR0.p + 3 * i * n;
            const double* R1 = tR1.p + 3 * i * n;
            const uint8_t* m1 = tm1.p + i * n;
            const uint8_t* m2 = tm2.p + i * n;
            const double dt = dts[size_t(k)];
            if (!started)
                hipLaunchKernelGGL(adj_start_kernel, grid, block, 0, st, m, tm, lam.p, m2, R1, dt,
                                   mua.p, lamn.p, part);
            // the first product also clears the minimising-cell word, which
            // the gather fills from w^k and the turn kernel reads
            unsigned long long* const am = cfl_dt ? argmin.p : nullptr;
            hipLaunchKernelGGL(adj_vjp_kernel, grid, block, lds, st, m, tm, W1, mua.p, g, hg, thr,
                               cc, am);
            hipLaunchKernelGGL(adj_gather_rk2_kernel, grid, block, 0, st, m, tm, cc, lam.p, m2,
                               m1, R0, dt, mua.p, lamn.p, part, Wn, g, thr, rmin_hist.p + i, am);
            hipLaunchKernelGGL(adj_vjp_kernel, grid, block, lds, st, m, tm, Wn, mua.p, g, hg, thr,
                               cc, (unsigned long long*)nullptr);
            // step k-1's tape is in this segment: start its reverse in the same pass
            const bool next = (k - 1 >= n0);
            hipLaunchKernelGGL(adj_turn_kernel, grid, block, 0, st, m, tm, cc, Wn, g, thr, cfl,
                               am, part, cells, ng, k >= 1 ? d_r.p + (k - 1) * ng : nullptr,
                               lamn.p, next ? m2 - n : nullptr, next ? R1 - 3 * n : nullptr,
                               next ? dts[size_t(k - 1)] : 0.0, mua.p, lam.p, partn);
            std::swap(lam.p, lamn.p);
            std::swap(part, partn);
            started = next;
        }
        HIP_TRY(hipGetLastError());
    }
    const int64_t nc = s->nc;
    hipLaunchKernelGGL(adj_unpack_kernel, dim3(unsigned((n + kBlock - 1) / kBlock)), block, 0, st,
                       n, s->d_perm.p, lam.p, gout.p, gout.p + nc, gout.p + 2 * nc,
                       gout.p + 3 * nc);
    HIP_TRY(hipGetLastError());
    double* outs[4] = {gH, gHU, gHV, gh};
    for (int q = 0; q < 4; ++q)
        if (outs[q])
            HIP_TRY(hipMemcpyAsync(outs[q], gout.p + q * nc, size_t(nc) * sizeof(double),
                                   hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return VSW_OK;
}

int vsw_last_dt(vsw_solver* s, double* dt) {
    if (!s || !dt) return fail(VSW_EINVAL, "NULL argument");
    *dt = s->dt_last;
    return VSW_OK;
}

int vsw_clamp_count(vsw_solver* s, int64_t* count) {
    if (!s || !count) return fail(VSW_EINVAL, "NULL argument");
    *count = s->clamps;
    return VSW_OK;
}

int vsw_dt_history(vsw_solver* s, int64_t max, double* dts, int64_t* count) {
    if (!s || !count) return fail(VSW_EINVAL, "NULL argument");
    const int64_t n = int64_t(s->last_dts.size());
    *count = n;
    if (dts)
        for (int64_t i = 0; i < n && i < max; ++i) dts[i] = s->last_dts[i];
    return VSW_OK;
}

int vsw_set_gauges(vsw_solver* s, int32_t n, const int32_t* cells) {
    if (!s) return fail(VSW_EINVAL, "NULL solver");
    if (!s->has_mesh) return fail(VSW_ESTATE, "no mesh uploaded");
    if (n < 0 || (n > 0 && !cells)) return fail(VSW_EINVAL, "bad gauge list");
    std::vector<int64_t> inv(s->nc);
    for (int64_t i = 0; i < s->nint; ++i)
        if (s->perm[i] >= 0) inv[s->perm[i]] = i;
    std::vector<int64_t> idx(n);
    std::vector<int32_t> seg(n);
    for (int32_t g = 0; g < n; ++g) {
        if (cells[g] < 0 || cells[g] >= s->nc) return fail(VSW_EINVAL, "gauge cell out of range");
        idx[g] = inv[cells[g]];
        seg[g] = int32_t(std::upper_bound(s->seg_off.begin(), s->seg_off.end(),
                                          int64_t(cells[g])) - s->seg_off.begin()) - 1;
    }
    DeviceGuard dg(s->device);
    HIP_TRY(s->d_gauge_cells.alloc(size_t(n)));
    HIP_TRY(s->d_gauge_seg.alloc(size_t(n)));
    if (n > 0) {
        HIP_TRY(hipMemcpy(s->d_gauge_cells.p, idx.data(), size_t(n) * sizeof(int64_t),
                          hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(s->d_gauge_seg.p, seg.data(), size_t(n) * sizeof(int32_t),
                          hipMemcpyHostToDevice));
    }
    s->ngauges = n;
    s->gauge_user.assign(cells, cells + n);
    s->gauge_eta.clear();
    s->gauge_t.clear();
    return VSW_OK;
}

int vsw_get_gauges(vsw_solver* s, int64_t max_steps, double* eta_out, double* t_out,
                   int64_t* count) {
    if (!s || !count) return fail(VSW_EINVAL, "NULL argument");
    const int64_t steps = int64_t(s->gauge_t.size());
    *count = steps;
    const int64_t m = std::min(steps, max_steps);
    if (eta_out && s->ngauges > 0)
        std::memcpy(eta_out, s->gauge_eta.data(), size_t(m) * s->ngauges * sizeof(double));
    if (t_out) std::memcpy(t_out, s->gauge_t.data(), size_t(m) * sizeof(double));
    return VSW_OK;
}

int vsw_set_kernel_variant(vsw_solver* s, int variant) {
    if (!s) return fail(VSW_EINVAL, "NULL solver");
    if (variant != VSW_KERNEL_FUSED && variant != VSW_KERNEL_TWO_PASS &&
        variant != VSW_KERNEL_FACES)
        return fail(VSW_EINVAL, "unknown kernel variant");
    if (variant == VSW_KERNEL_TWO_PASS && s->prm.precision == VSW_FP32)
        return fail(VSW_EINVAL, "the two-pass variant is FP64 only");
    s->variant = variant;
    return VSW_OK;
}

int vsw_set_tile_order(vsw_solver* s, int xcd_order) {
    if (!s) return fail(VSW_EINVAL, "NULL solver");
    if (xcd_order != 0 && xcd_order != 1) return fail(VSW_EINVAL, "tile order is 0 or 1");
    s->xcd_order = xcd_order;
    return VSW_OK;
}

int vsw_set_occupancy(vsw_solver* s, int wg_per_cu) {
    if (!s) return fail(VSW_EINVAL, "NULL solver");
    if (wg_per_cu != 0 && wg_per_cu != 2 && wg_per_cu != 3)
        return fail(VSW_EINVAL, "workgroups per CU is 0, 2 or 3");
    s->occupancy = wg_per_cu;
    return VSW_OK;
}

int vsw_autotune(vsw_solver* s, int64_t steps, int32_t* chosen, double* ms_per_step) {
    if (!s) return fail(VSW_EINVAL, "NULL solver");
    if (!s->has_mesh || !s->has_state) return fail(VSW_ESTATE, "mesh and state required");
    if (steps < 2 || steps > 100000) return fail(VSW_EINVAL, "steps must be in [2, 100000]");
    DeviceGuard dg(s->device);
    HIP_TRY(hipStreamSynchronize(s->stream));
    const bool f32 = s->prm.precision == VSW_FP32;
    const size_t rec = f32 ? sizeof(CellF) : sizeof(Cell4);
    // the buffer holding the current state (it alternates as steps run)
    auto wp = [&]() { return f32 ? (void*)s->d_wf[s->cur].p : (void*)s->d_w[s->cur].p; };
    const double t_save = s->t, dt_save = s->dt_last;
    const int64_t clamps_save = s->clamps;
    const std::vector<double> seg_t_save = s->seg_t, seg_dt_save = s->seg_dt;
    const std::vector<int64_t> seg_steps_save = s->seg_steps;
    const int variant_save = s->variant, xcd_save = s->xcd_order, occ_save = s->occupancy;
    const int graph_save = s->graph_mode, tile_save = s->tile;
    const bool prof_save = s->profiling;
    // kernel organisation of each configuration group
    static const int kTileOf[7] = {128, 256, 512, kTile, kTile, kTile, kTile};
    static const int kVariantOf[7] = {VSW_KERNEL_FACES, VSW_KERNEL_FACES, VSW_KERNEL_FACES,
                                      VSW_KERNEL_FUSED, VSW_KERNEL_FUSED, VSW_KERNEL_FUSED,
                                      VSW_KERNEL_TWO_PASS};
    static const int kOccOf[7] = {0, 0, 0, 0, 3, 2, 0};
    // The state records of the current layout, copied back after every
    // configuration (a layout for another tile size is made from them).
    DevBuf<unsigned char> save;
    auto snapshot = [&]() -> hipError_t {
        const size_t bytes = size_t(s->nint) * rec;
        if (save.n < bytes) {
            const hipError_t e = save.alloc(bytes);
            if (e != hipSuccess) return e;
        }
        const hipError_t e = hipMemcpyAsync(save.p, wp(), bytes, hipMemcpyDeviceToDevice, s->stream);
        return (e != hipSuccess) ? e : hipStreamSynchronize(s->stream);
    };
    auto restore = [&]() {
        (void)hipMemcpyAsync(wp(), save.p, size_t(s->nint) * rec, hipMemcpyDeviceToDevice,
                             s->stream);
        (void)hipStreamSynchronize(s->stream);
        s->t = t_save;
        s->dt_last = dt_save;
        s->clamps = clamps_save;
        s->seg_t = seg_t_save;
        s->seg_dt = seg_dt_save;
        s->seg_steps = seg_steps_save;
        s->seg_log.clear();
        s->last_dts.clear();
        s->gauge_eta.clear();
        s->gauge_t.clear();
        s->rmin_slot = -1;
    };
    // On every return path: the state, time and logs as they were; the
    // caller's launch configuration unless a winner was applied.
    bool applied = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const auto restore_on_exit = on_exit([&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        restore();
        s->profiling = prof_save;
        s->release_graph();
        if (!applied) {
            s->variant = variant_save;
            s->xcd_order = xcd_save;
            s->graph_mode = graph_save;
            s->occupancy = occ_save;
            if (s->tile != tile_save) (void)vsw_set_tile_size(s, tile_save);
        }
    });
    HIP_TRY(snapshot());
    s->profiling = false;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    double best = INFINITY;
    int best_c = -1;
    for (int c = 0; c < VSW_TUNE_CONFIGS; ++c)
        if (ms_per_step) ms_per_step[c] = INFINITY;
    // the caller's tile size first, so that the others are laid out from
    // the caller's own records
    int tiles[3] = {tile_save, 0, 0};
    for (int i = 0, j = 1; i < 3; ++i)
        if (kTileOf[i] != tile_save) tiles[j++] = kTileOf[i];
    for (int ti = 0; ti < 3; ++ti) {
        const int tile = tiles[ti];
        if (tile != s->tile) {
            restore();
            const int rc = vsw_set_tile_size(s, tile);
            if (rc != VSW_OK) return rc;
            HIP_TRY(snapshot());
        }
        for (int org = 0; org < 7; ++org) {
            if (kTileOf[org] != tile) continue;
            if (kVariantOf[org] == VSW_KERNEL_TWO_PASS && f32) continue;
            for (int xcd = 0; xcd < 2; ++xcd)
                for (int graph = 0; graph < 3; ++graph) {
                    const int c = (org * 2 + xcd) * 3 + graph;
                    s->variant = kVariantOf[org];
                    s->xcd_order = xcd;
                    s->occupancy = kOccOf[org];
                    s->graph_mode = graph;
                    s->release_graph();
                    restore();
                    // warm-up (and graph capture: a whole-call graph is
                    // captured for the step count it runs)
                    int rc = vsw_step(s, graph == 2 ? steps : 2, INFINITY, nullptr, nullptr);
                    if (rc != VSW_OK) return rc;
                    HIP_TRY(hipEventRecord(e0, s->stream));
                    rc = vsw_step(s, steps, INFINITY, nullptr, nullptr);
                    if (rc != VSW_OK) return rc;
                    HIP_TRY(hipEventRecord(e1, s->stream));
                    HIP_TRY(hipEventSynchronize(e1));
                    float f = 0.f;
                    HIP_TRY(hipEventElapsedTime(&f, e0, e1));
                    const double ms = double(f) / double(steps);
                    if (ms_per_step) ms_per_step[c] = ms;
                    if (ms < best) {
                        best = ms;
                        best_c = c;
                    }
                }
        }
    }
    const int org = (best_c / 3) / 2;
    if (kTileOf[org] != s->tile) {
        restore();
        const int rc = vsw_set_tile_size(s, kTileOf[org]);
        if (rc != VSW_OK) return rc;
        HIP_TRY(snapshot());
    }
    s->variant = kVariantOf[org];
    s->xcd_order = (best_c / 3) % 2;
    s->graph_mode = best_c % 3;
    s->occupancy = kOccOf[org];
    applied = true;
    if (chosen) *chosen = best_c;
    return VSW_OK;
}

int vsw_set_graph(vsw_solver* s, int on) {
    if (!s) return fail(VSW_EINVAL, "NULL solver");
    if (on < 0 || on > 2) return fail(VSW_EINVAL, "graph mode must be 0, 1 or 2");
    s->graph_mode = on;
    {
        DeviceGuard dg(s->device);
        (void)hipStreamSynchronize(s->stream);
        s->release_graph();
    }
    return VSW_OK;
}

int vsw_set_profiling(vsw_solver* s, int on) {
    if (!s) return fail(VSW_EINVAL, "NULL solver");
    s->profiling = on != 0;
    for (int i = 0; i < KK_COUNT; ++i) {
        s->prof_ms[i] = 0;
        s->prof_n[i] = 0;
    }
    return VSW_OK;
}

int vsw_kernel_times(vsw_solver* s, int nkinds, double* ms, int64_t* launches) {
    if (!s) return fail(VSW_EINVAL, "NULL solver");
    for (int i = 0; i < nkinds; ++i) {
        if (ms) ms[i] = i < KK_COUNT ? s->prof_ms[i] : 0.0;
        if (launches) launches[i] = i < KK_COUNT ? s->prof_n[i] : 0;
    }
    return VSW_OK;
}

int vsw_prepare_mesh_host(int64_t nv, const double* vx, const double* vy, int64_t nc,
                          const int32_t* tri, const double* h, double* geom, double* area,
                          double* perim, int32_t* nbr, int32_t* is_left, int64_t* ne,
                          int64_t* nw) {
    HostMesh hm;
    std::string err;
    int rc = build_host_mesh(nv, vx, vy, nc, tri, h, VSW_ORDER_NONE, 0, kTile, hm, err);
    if (rc != VSW_OK) return fail(rc, err);
    for (int64_t i = 0; i < nc; ++i) {
        const int64_t k = hm.perm[i];
        for (int j = 0; j < 3; ++j) {
            for (int f = 0; f < G_NFACE; ++f)
                if (geom)
                    geom[(size_t(f) * 3 + j) * nc + k] = hm.face_geom[(size_t(f) * 3 + j) * nc + i];
            const uint32_t sl = hm.nbr[size_t(j) * nc + i];
            if (nbr) nbr[size_t(j) * nc + k] = sl == kWall ? -1 : int32_t(hm.perm[sl >> 3]);
            if (is_left) is_left[size_t(j) * nc + k] = (sl == kWall || (sl & 4u)) ? 1 : 0;
        }
        if (area) area[k] = hm.area[i];
        if (perim) perim[k] = hm.perim[i];
    }
    if (ne) *ne = hm.ne;
    if (nw) *nw = hm.nw;
    return VSW_OK;
}

int vsw_get_permutation(vsw_solver* s, int64_t* perm) {
    if (!s || !perm) return fail(VSW_EINVAL, "NULL argument");
    if (!s->has_mesh) return fail(VSW_ESTATE, "no mesh uploaded");
    int64_t o = 0;
    for (int64_t v : s->perm)
        if (v >= 0) perm[o++] = v;
    return VSW_OK;
}

int vsw_mesh_info(vsw_solver* s, int64_t* nc, int64_t* ne, int64_t* nw) {
    if (!s) return fail(VSW_EINVAL, "NULL solver");
    if (!s->has_mesh) return fail(VSW_ESTATE, "no mesh uploaded");
    if (nc) *nc = s->nc;
    if (ne) *ne = s->ne;
    if (nw) *nw = s->nw;
    return VSW_OK;
}

}  // extern "C"
