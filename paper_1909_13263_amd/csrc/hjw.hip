// hjw.hip - the single-grid C ABI declared in include/hjw.h (kernels in hjw_kernels.h).
//
// One TVD-RK3 step (Rathan & Biswas, arXiv:1909.13263, Step 5) is three launches:
//   k_stage<Pre>   WENO-L derivatives of phi^n (Steps 1-4), writes Hbar = H(ubar,vbar),
//                  Dx = (u+ - u-)/2, Dy = (v+ - v-)/2 and folds the workgroup's min/max
//                  of u+-, v+- into range slots;
//   k_stage<Mid>   every workgroup reduces the slots -> alpha_x, alpha_y (eq. LF, maximum
//                  of |H_p| over the box) -> dt (CFL rule); rebuilds
//                  phi_1 = phi^n - dt (Hbar - ax Dx - ay Dy) on the tile and its halo,
//                  derivatives of phi_1, phi_2 = 3/4 phi^n + 1/4 (phi_1 + dt L);
//   k_stage<Last>  derivatives of phi_2, phi^{n+1} = 1/3 phi^n + 2/3 (phi_2 + dt L),
//                  written in place over phi^n.
// The step state lives on the device, so whole steps are captured once in a HIP
// graph and replayed; kernels of a step past t_final exit at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "hjw.h"
#include "hjw_common.h"
#include "hjw_kernels.h"

using namespace hjw;

namespace hjw {
std::string& last_error() {
    thread_local std::string text;
    return text;
}
}  // namespace hjw

namespace {

constexpr int kGraphSteps = 16;
constexpr int kMaxBatch = 512;  // steps enqueued between two reads of the step state

}  // namespace

// ------------------------------------------------------------------ the grid object
struct hjw_grid {
    int dim = 0;
    int64_t nx = 0, ny = 1;
    double dx = 0.0, dy = 1.0;
    double x0 = 0.0, y0 = 0.0;   // coordinates of node (0, 0)
    int bcx = 0, bcy = 0;
    int prec = 0;
    int ham = kHBurgers;
    double hp[4] = {1.0, 1.0, 1.0, 0.0};
    bool ham_set = false;

    // binding
    char* ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool bound = false;
    void* phi = nullptr;
    void* phi2 = nullptr;
    void* flux = nullptr;  // Hbar, Dx, Dy back to back
    DevState* state = nullptr;   // two step records, st[par] is the current one
    void* slots = nullptr;       // range accumulators
    int par = 0;
    int nbx = 0, nby = 0;
    int tile_rows = 16;  // 2-D tile height (16 or 32)
    int seg_opt = 0;     // nodes per thread in the 2-D sweeps: 0 automatic, 4 or 8
    int plan_opt = 0;    // step plan: 0 automatic, 1 in every workgroup, 2 own launch
    int llf = 0;         // dissipation: 0 the step's global alpha, 1 per node (local LF)
    int scheme = HJW_WENO_L;

    // host mirror
    DevState* pinned = nullptr;  // pinned host copy of the device state
    bool phi_set = false;
    bool failed = false;
    DevState last{};

    // graphs
    bool use_graph = true;
    hipGraphExec_t graph[2] = {nullptr, nullptr};   // by the parity the replay starts at

    // per-kernel event timing (eager launches only)
    bool timing = false;
    std::vector<hipEvent_t> ev;       // start/end pairs
    std::vector<int> ev_kind;
    int ev_used = 0;
    double kernel_ms[4] = {0, 0, 0, 0};
    int64_t kernel_count[4] = {0, 0, 0, 0};

    size_t elem_phi() const { return prec == HJW_FP32 ? 4 : 8; }
    size_t elem_flux() const { return prec == HJW_FP64 ? 8 : 4; }
    int64_t cells() const { return nx * ny; }
};

namespace {

void layout(const hjw_grid* g, size_t* off_phi2, size_t* off_flux, size_t* off_part,
            size_t* off_state, size_t* total, int* nbx, int* nby) {
    const size_t n = size_t(g->cells());
    if (g->dim == 2) {
        *nbx = int((g->nx + kTX - 1) / kTX);
        *nby = int((g->ny + 15) / 16);
    } else {
        *nbx = int((g->nx + kTX1 - 1) / kTX1);
        *nby = 1;
    }
    const size_t nb = size_t(*nbx) * size_t(*nby);
    size_t o = 0;
    o += align256(n * g->elem_phi());
    *off_phi2 = o;
    o += align256(n * g->elem_phi());
    *off_flux = o;
    // three flux arrays, and at least 8n bytes (an FP64 staging area in FP32 mode)
    o += align256(std::max(size_t(3) * n * g->elem_flux(), n * 8));
    (void)nb;
    *off_part = o;                       // range slots
    o += align256(sizeof(RangeSlots));
    *off_state = o;                      // two step records
    o += align256(2 * sizeof(DevState));
    *total = o;
}

// The step plan gets a launch of its own (one wave between the first and second stage
// kernels) on grids of more than kPlanLaunchTiles tiles; on smaller grids the extra
// launch costs more than every workgroup planning for itself.
constexpr int kPlanLaunchTiles = 2048;
bool plan_launch(const hjw_grid* g) {
    if (g->dim != 2) return false;
    if (g->plan_opt) return g->plan_opt == 2;
    return g->nbx * g->nby > kPlanLaunchTiles;
}

template <typename T, typename P>
StageArgs<T, P> make_args(const hjw_grid* g) {
    StageArgs<T, P> a{};
    a.phi_n = static_cast<const P*>(g->phi);
    a.phi_s = static_cast<const P*>(g->phi2);
    a.flux = static_cast<T*>(g->flux);
    a.st = g->state;
    a.par = g->par;
    a.slots = g->slots;
    a.nx = g->nx;
    a.ny = g->ny;
    a.bcx = g->bcx;
    a.bcy = g->bcy;
    a.ihx = P(1.0 / g->dx);
    a.ihy = P(1.0 / g->dy);
    a.ihxT = T(1.0 / g->dx);
    a.ihyT = T(1.0 / g->dy);
    a.epsx = T(weight_eps(g->scheme, g->dx));
    a.epsy = T(weight_eps(g->scheme, g->dy));
    a.scheme = g->scheme;
    a.ham = g->ham;
    for (int k = 0; k < 4; ++k) {
        a.hpT[k] = T(g->hp[k]);
        a.hpD[k] = g->hp[k];
    }
    a.ihxD = 1.0 / g->dx;
    a.ihyD = g->dim == 2 ? 1.0 / g->dy : 0.0;
    a.nbx = g->nbx;
    a.nby = g->nby;
    a.remap = (g->dim == 2 && (g->nbx * g->nby) % 8 == 0) ? 1 : 0;
    a.dim = g->dim;
    a.plan_ready = plan_launch(g) ? 1 : 0;
    a.x0 = g->x0;
    a.y0 = g->y0;
    a.dxD = g->dx;
    a.dyD = g->dy;
    a.llf = g->llf;
    return a;
}

// Segment length of the 2-D sweeps: 4 nodes per thread (twice the waves) for the
// FP32 stencil on 16-row tiles when the grid has at most 2.5 tiles per compute unit, so
// that small grids still keep every SIMD busy; 8 otherwise (fewer instructions per
// node).  FP64 keeps 8: its registers leave no room for the extra waves.
constexpr int kSmallGridTiles = 640;
int segment(const hjw_grid* g) {
    if (g->seg_opt) return g->seg_opt;
    return (g->prec != HJW_FP64 && g->tile_rows == 16 && g->nbx * g->nby <= kSmallGridTiles) ? 4
                                                                                          : 8;
}

template <typename T, typename P, int STAGE>
hipError_t launch_stage(const hjw_grid* g, StageArgs<T, P> a) {
    const dim3 grid(unsigned(g->nbx * g->nby));
    constexpr bool kNarrow = !std::is_same<T, double>::value;   // the S = 4 kernels
    // the time- and phi-dependent family and the local dissipation have kernels of their
    // own (16-row tiles, 8-node segments), so that the other kernels carry none of their code
    constexpr bool kH = STAGE != kStageDeriv;   // the derivatives do not evaluate H
    const bool own = g->ham == HJW_H_TIMED || g->llf;
    if (kH && own && g->dim == 2)
        hipLaunchKernelGGL((k_stage2d<T, P, STAGE, 16, 8, true>), grid, dim3(threads2d(16, 8)),
                           0, g->stream, a);
    else if (kH && own)
        hipLaunchKernelGGL((k_stage1d<T, P, STAGE, true>), grid, dim3(256), 0, g->stream, a);
    else if (g->dim == 2 && g->tile_rows == 32)
        hipLaunchKernelGGL((k_stage2d<T, P, STAGE, 32, 8, false>), grid, dim3(threads2d(32, 8)),
                           0, g->stream, a);
    else if (g->dim == 2 && kNarrow && segment(g) == 4)
        hipLaunchKernelGGL((k_stage2d<T, P, STAGE, 16, kNarrow ? 4 : 8, false>), grid,
                           dim3(threads2d(16, 4)), 0, g->stream, a);
    else if (g->dim == 2)
        hipLaunchKernelGGL((k_stage2d<T, P, STAGE, 16, 8, false>), grid, dim3(threads2d(16, 8)),
                           0, g->stream, a);
    else
        hipLaunchKernelGGL((k_stage1d<T, P, STAGE, false>), grid, dim3(256), 0, g->stream, a);
    return hipGetLastError();
}

// Launch one kernel through fn(); with timing on, bracket it by a pair of events.
template <class Fn>
hipError_t timed(hjw_grid* g, int kind, Fn fn) {
    if (!g->timing) return fn();
    if (size_t(2 * g->ev_used + 2) > g->ev.size()) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(g->ev[2 * g->ev_used], g->stream);
    if (e != hipSuccess) return e;
    e = fn();
    if (e != hipSuccess) return e;
    e = hipEventRecord(g->ev[2 * g->ev_used + 1], g->stream);
    if (e != hipSuccess) return e;
    g->ev_kind[g->ev_used++] = kind;
    return hipSuccess;
}

template <typename T, typename P>
hipError_t enqueue_step_typed(hjw_grid* g) {
    StageArgs<T, P> a = make_args<T, P>(g);
    g->par ^= 1;   // every enqueued step moves the current record to the other slot
    hipError_t e = timed(g, 0, [&] { return launch_stage<T, P, kStagePre>(g, a); });
    if (e != hipSuccess) return e;
    if (a.plan_ready) {
        e = timed(g, 1, [&] {
            hipLaunchKernelGGL((k_plan<T, P>), dim3(1), dim3(64), 0, g->stream, a);
            return hipGetLastError();
        });
        if (e != hipSuccess) return e;
    }
    a.out = static_cast<P*>(g->phi2);
    e = timed(g, 2, [&] { return launch_stage<T, P, kStageMid>(g, a); });
    if (e != hipSuccess) return e;
    a.out = static_cast<P*>(g->phi);
    return timed(g, 3, [&] { return launch_stage<T, P, kStageLast>(g, a); });
}

hipError_t enqueue_step(hjw_grid* g) {
    switch (g->prec) {
    case HJW_FP64:
        return enqueue_step_typed<double, double>(g);
    case HJW_FP32_MIXED:
        return enqueue_step_typed<float, double>(g);
    default:
        return enqueue_step_typed<float, float>(g);
    }
}

// Kernel k of a step (0 first stage, 1 plan, 2 second, 3 third stage) against the
// records of the current parity.
template <typename T, typename P>
hipError_t launch_kind(const hjw_grid* g, int k) {
    StageArgs<T, P> a = make_args<T, P>(g);
    if (k == 0) return launch_stage<T, P, kStagePre>(g, a);
    if (k == 1) {
        hipLaunchKernelGGL((k_plan<T, P>), dim3(1), dim3(64), 0, g->stream, a);
        return hipGetLastError();
    }
    if (k == 2) {
        a.out = static_cast<P*>(g->phi2);
        return launch_stage<T, P, kStageMid>(g, a);
    }
    a.out = static_cast<P*>(g->phi);
    return launch_stage<T, P, kStageLast>(g, a);
}

template <typename T, typename P>
hipError_t enqueue_deriv_typed(const hjw_grid* g, double* um, double* up, double* vm,
                               double* vp) {
    StageArgs<T, P> a = make_args<T, P>(g);
    a.dout0 = um;
    a.dout1 = up;
    a.dout2 = vm;
    a.dout3 = vp;
    return launch_stage<T, P, kStageDeriv>(g, a);
}

void drop_graph(hjw_grid* g) {
    for (auto& gr : g->graph) {
        if (gr) (void)hipGraphExecDestroy(gr);
        gr = nullptr;
    }
}

// Capture kGraphSteps whole steps starting at the current parity.  kGraphSteps is
// even, so a replay leaves the parity where it found it.
hjw_status build_graph(hjw_grid* g) {
    static_assert(kGraphSteps % 2 == 0, "replays must preserve the record parity");
    const int par0 = g->par;
    hipGraph_t graph = nullptr;
    HIP_TRY(hipStreamBeginCapture(g->stream, hipStreamCaptureModeRelaxed));
    hipError_t e = hipSuccess;
    for (int s = 0; s < kGraphSteps && e == hipSuccess; ++s) e = enqueue_step(g);
    hipError_t e2 = hipStreamEndCapture(g->stream, &graph);
    g->par = par0;
    if (e != hipSuccess || e2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(HJW_EHIP, "graph capture failed: %s / %s", hipGetErrorString(e),
                    hipGetErrorString(e2));
    }
    hipError_t e3 = hipGraphInstantiate(&g->graph[par0], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e3 != hipSuccess) {
        g->graph[par0] = nullptr;
        return fail(HJW_EHIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e3));
    }
    return HJW_OK;
}

hjw_status enqueue_steps(hjw_grid* g, int64_t n) {
    if (g->use_graph && !g->timing && n >= kGraphSteps) {
        if (!g->graph[g->par]) {
            hjw_status s = build_graph(g);
            if (s != HJW_OK) return s;
        }
        while (n >= kGraphSteps) {
            HIP_TRY(hipGraphLaunch(g->graph[g->par], g->stream));
            n -= kGraphSteps;
        }
    }
    for (int64_t k = 0; k < n; ++k) HIP_TRY(enqueue_step(g));
    return HJW_OK;
}

hjw_status read_state(hjw_grid* g) {
    // the pinned mirror of a bound grid; the no-allocation solve has none and copies into
    // ordinary host memory
    DevState plain{};
    DevState* dst = g->pinned ? g->pinned : &plain;
    HIP_TRY(hipMemcpyAsync(dst, g->state + g->par, sizeof(DevState), hipMemcpyDeviceToHost,
                           g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    g->last = *dst;
    for (int k = 0; k < g->ev_used; ++k) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, g->ev[2 * k], g->ev[2 * k + 1]));
        g->kernel_ms[g->ev_kind[k]] += ms;
        g->kernel_count[g->ev_kind[k]] += 1;
    }
    g->ev_used = 0;
    return HJW_OK;
}

void fill_info(const hjw_grid* g, hjw_info* info) {
    if (!info) return;
    info->steps = g->last.steps;
    info->t = g->last.t;
    info->last_dt = g->last.dt;
    info->alpha_x = g->last.alpha_x;
    info->alpha_y = g->last.alpha_y;
    for (int k = 0; k < 4; ++k) info->range[k] = g->last.range[k];
}

hjw_status check_ready(const hjw_grid* g) {
    if (!g) return fail(HJW_EINVAL, "grid is NULL");
    if (!g->bound) return fail(HJW_ESTATE, "grid has no workspace bound");
    if (g->failed) return fail(HJW_ESTATE, "grid failed (non-finite values); set phi again");
    return HJW_OK;
}

// Check a grid description and write it into g (hjw_grid_create and the no-allocation
// solve).
hjw_status describe_grid(hjw_grid* g, int dim, const int64_t* n, const double* lo,
                         const double* hi, const int* bc, int prec) {
    if (dim != 1 && dim != 2) return fail(HJW_EINVAL, "dim must be 1 or 2 (got %d)", dim);
    if (!n || !lo || !hi || !bc) return fail(HJW_EINVAL, "NULL array argument");
    if (prec < HJW_FP64 || prec > HJW_FP32) return fail(HJW_EINVAL, "unknown precision %d", prec);
    for (int d = 0; d < dim; ++d) {
        if (n[d] < 8) return fail(HJW_EINVAL, "n[%d] = %lld < 8", d, (long long)n[d]);
        if (!(hi[d] > lo[d]) || !std::isfinite(lo[d]) || !std::isfinite(hi[d]))
            return fail(HJW_EINVAL, "axis %d: need finite lo < hi", d);
        if (bc[d] != HJW_BC_PERIODIC && bc[d] != HJW_BC_EXTRAP &&
            bc[d] != HJW_BC_DIRICHLET)
            return fail(HJW_EINVAL, "axis %d: unknown boundary %d", d, bc[d]);
    }
    if (n[0] > (int64_t(1) << 30) || (dim == 2 && n[1] > (int64_t(1) << 30)) ||
        (dim == 2 && n[0] * n[1] > (int64_t(1) << 34)))
        return fail(HJW_EINVAL, "grid too large");
    if (dim == 2 && (n[0] + kTX - 1) / kTX * ((n[1] + 15) / 16) > INT32_MAX)
        return fail(HJW_EINVAL, "too many tiles");
    g->dim = dim;
    g->nx = n[0];
    g->ny = dim == 2 ? n[1] : 1;
    g->dx = (hi[0] - lo[0]) / double(n[0]);
    g->dy = dim == 2 ? (hi[1] - lo[1]) / double(n[1]) : 1.0;
    // node 0: the low end of a periodic axis, the first cell centre of an extrapolated one
    g->x0 = lo[0] + (bc[0] == HJW_BC_EXTRAP ? 0.5 * g->dx : 0.0);
    g->y0 = dim == 2 ? lo[1] + (bc[1] == HJW_BC_EXTRAP ? 0.5 * g->dy : 0.0) : 0.0;
    g->bcx = bc[0];
    g->bcy = dim == 2 ? bc[1] : HJW_BC_PERIODIC;
    g->prec = prec;
    return HJW_OK;
}

}  // namespace

// ------------------------------------------------------------------ C ABI
extern "C" {

const char* hjw_last_error(void) { return hjw::last_error().c_str(); }

const char* hjw_version(void) { return "hjw 0.1 (WENO-L, gfx950)"; }

hjw_status hjw_grid_create(int dim, const int64_t* n, const double* lo, const double* hi,
                           const int* bc, int prec, hjw_grid** out) {
    hjw::last_error().clear();
    if (!out) return fail(HJW_EINVAL, "out is NULL");
    *out = nullptr;
    hjw_grid* g = new (std::nothrow) hjw_grid();
    if (!g) return fail(HJW_ENOMEM, "host allocation failed");
    const hjw_status st = describe_grid(g, dim, n, lo, hi, bc, prec);
    if (st != HJW_OK) {
        delete g;
        return st;
    }
    *out = g;
    return HJW_OK;
}

hjw_status hjw_workspace_bytes(const hjw_grid* g, size_t* bytes) {
    if (!g || !bytes) return fail(HJW_EINVAL, "NULL argument");
    size_t a, b, c, d, total;
    int nbx, nby;
    layout(g, &a, &b, &c, &d, &total, &nbx, &nby);
    *bytes = total;
    return HJW_OK;
}

hjw_status hjw_bind(hjw_grid* g, void* ws, size_t bytes, void* stream) {
    if (!g || !ws) return fail(HJW_EINVAL, "NULL argument");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0)
        return fail(HJW_EINVAL, "workspace must be 256-byte aligned");
    size_t o_phi2, o_flux, o_part, o_state, total;
    int nbx, nby;
    layout(g, &o_phi2, &o_flux, &o_part, &o_state, &total, &nbx, &nby);
    if (bytes < total)
        return fail(HJW_ENOMEM, "workspace has %zu bytes, grid needs %zu", bytes, total);
    drop_graph(g);
    if (g->own_stream && g->stream) (void)hipStreamDestroy(g->stream);
    g->own_stream = false;
    g->stream = static_cast<hipStream_t>(stream);
    if (!g->stream) {
        HIP_TRY(hipStreamCreate(&g->stream));
        g->own_stream = true;
    }
    if (!g->pinned) HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&g->pinned), sizeof(DevState),
                                          hipHostMallocDefault));
    g->ws = static_cast<char*>(ws);
    g->ws_bytes = bytes;
    g->phi = g->ws;
    g->phi2 = g->ws + o_phi2;
    g->flux = g->ws + o_flux;
    g->slots = g->ws + o_part;
    g->state = reinterpret_cast<DevState*>(g->ws + o_state);
    g->par = 0;
    g->nbx = nbx;
    g->nby = g->dim == 2 ? int((g->ny + g->tile_rows - 1) / g->tile_rows) : nby;
    g->bound = true;
    g->phi_set = false;
    g->failed = false;
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, g->stream, g->state,
                       static_cast<RangeSlots*>(g->slots));
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(g->stream));
    g->last = DevState{};
    return HJW_OK;
}

hjw_status hjw_set_scheme(hjw_grid* g, int scheme) {
    if (!g) return fail(HJW_EINVAL, "grid is NULL");
    if (scheme != HJW_WENO_L && scheme != HJW_WENO_JP)
        return fail(HJW_EINVAL, "unknown scheme %d", scheme);
    if (scheme != g->scheme) {
        g->scheme = scheme;
        drop_graph(g);   // graphs hold the stage arguments
    }
    return HJW_OK;
}

hjw_status hjw_set_hamiltonian(hjw_grid* g, int kind, const double* params, int nparams) {
    if (!g) return fail(HJW_EINVAL, "grid is NULL");
    if (kind < HJW_H_LINEAR || kind > HJW_H_TIMED)
        return fail(HJW_EINVAL, "unknown Hamiltonian %d", kind);
    if (nparams < 0 || nparams > 4 || (nparams > 0 && !params))
        return fail(HJW_EINVAL, "bad parameter list");
    double p[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < nparams; ++k) {
        if (!std::isfinite(params[k])) return fail(HJW_EINVAL, "non-finite parameter");
        p[k] = params[k];
    }
    if ((kind == HJW_H_NORM || kind == HJW_H_CURVATURE) && p[1] < 0.0)
        return fail(HJW_EINVAL, "NORM needs p[1] >= 0");
    if (kind == HJW_H_TIMED && g->dim == 2 && g->tile_rows == 32)
        return fail(HJW_EINVAL, "the TIMED family runs 16-row tiles");
    if (kind == HJW_H_CURVATURE) {
        if (g->dim != 2 || g->bcx == HJW_BC_EXTRAP || g->bcy == HJW_BC_EXTRAP)
            return fail(HJW_EINVAL, "CURVATURE needs a 2-D grid with periodic or Dirichlet axes");
        if (p[2] < 0.0) return fail(HJW_EINVAL, "CURVATURE needs eps = p[2] >= 0");
    }
    g->ham = kind;
    for (int k = 0; k < 4; ++k) g->hp[k] = p[k];
    g->ham_set = true;
    drop_graph(g);
    return HJW_OK;
}

hjw_status hjw_set_phi(hjw_grid* g, const double* phi0, int on_device) {
    if (!g || !phi0) return fail(HJW_EINVAL, "NULL argument");
    if (!g->bound) return fail(HJW_ESTATE, "grid has no workspace bound");
    const size_t n = size_t(g->cells());
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    // FP64 input lands in phi itself, or in the flux area when phi is FP32
    double* src = g->prec == HJW_FP32 ? static_cast<double*>(g->flux) : static_cast<double*>(g->phi);
    HIP_TRY(hipMemcpyAsync(src, phi0, n * sizeof(double), kind, g->stream));
    g->par = 0;
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, g->stream, g->state,
                       static_cast<RangeSlots*>(g->slots));
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_check_finite, dim3(1024), dim3(256), 0, g->stream, src, int64_t(n),
                       g->state);
    HIP_TRY(hipGetLastError());
    if (g->prec == HJW_FP32) {
        hipLaunchKernelGGL(k_d2f, dim3(1024), dim3(256), 0, g->stream, src,
                           static_cast<float*>(g->phi), int64_t(n));
        HIP_TRY(hipGetLastError());
    }
    hjw_status s = read_state(g);
    if (s != HJW_OK) return s;
    g->phi_set = true;
    g->failed = false;
    if (g->last.bad) {
        g->failed = true;
        return fail(HJW_ENONFINITE, "phi0 holds non-finite values");
    }
    return HJW_OK;
}

hjw_status hjw_step_to(hjw_grid* g, double t_final, double cfl, int64_t max_steps,
                       hjw_info* info) {
    hjw_status s = check_ready(g);
    if (s != HJW_OK) return s;
    if (!g->phi_set) return fail(HJW_ESTATE, "phi was not set");
    if (!g->ham_set) return fail(HJW_ESTATE, "Hamiltonian was not set");
    if (!std::isfinite(t_final) || !(cfl > 0.0) || !std::isfinite(cfl))
        return fail(HJW_EINVAL, "need finite t_final and cfl > 0");
    const int64_t limit = max_steps > 0 ? max_steps : std::numeric_limits<int64_t>::max();
    hipLaunchKernelGGL(k_set_target, dim3(1), dim3(64), 0, g->stream, g->state + g->par, t_final, cfl,
                       limit);
    HIP_TRY(hipGetLastError());
    s = read_state(g);
    if (s != HJW_OK) return s;
    int64_t taken = 0;
    while (g->last.t < t_final && taken < limit && !g->last.bad) {
        // Steps enqueued before the next read of the step state: one graph's worth
        // while dt is unknown, else the estimate from the last dt plus a margin (dt
        // shrinks as the dissipation grows).  Surplus steps find t_final reached and
        // exit at once; a short count costs a round trip to the host.
        int64_t n = kGraphSteps;
        if (g->last.dt > 0.0) {
            const double est = std::ceil((t_final - g->last.t) / g->last.dt);
            const double want = est + std::max(2.0, std::ceil(est / 32.0));
            n = int64_t(std::min(std::max(want, 1.0), double(kMaxBatch)));
        }
        n = std::min(n, limit - taken);
        s = enqueue_steps(g, n);
        if (s != HJW_OK) return s;
        const int64_t before = g->last.steps;
        s = read_state(g);
        if (s != HJW_OK) return s;
        taken += g->last.steps - before;
        if (g->last.steps == before && !g->last.bad) break;  // nothing advanced
    }
    fill_info(g, info);
    if (g->last.bad) {
        g->failed = true;
        return fail(HJW_ENONFINITE, "non-finite value at step %lld (t = %g)",
                    (long long)g->last.steps, g->last.t);
    }
    return HJW_OK;
}

hjw_status hjw_get_phi(const hjw_grid* g, double* out, int on_device) {
    if (!g || !out) return fail(HJW_EINVAL, "NULL argument");
    if (!g->bound || !g->phi_set) return fail(HJW_ESTATE, "phi was not set");
    const size_t n = size_t(g->cells());
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    const void* src = g->phi;
    if (g->prec == HJW_FP32) {
        double* stage = static_cast<double*>(g->flux);
        hipLaunchKernelGGL(k_f2d, dim3(1024), dim3(256), 0, g->stream,
                           static_cast<const float*>(g->phi), stage, int64_t(n));
        HIP_TRY(hipGetLastError());
        src = stage;
    }
    HIP_TRY(hipMemcpyAsync(out, src, n * sizeof(double), kind, g->stream));
    HIP_TRY(hipStreamSynchronize(g->stream));
    return HJW_OK;
}

hjw_status hjw_derivatives(hjw_grid* g, double* um, double* up, double* vm, double* vp) {
    hjw_status s = check_ready(g);
    if (s != HJW_OK) return s;
    if (!g->phi_set) return fail(HJW_ESTATE, "phi was not set");
    if (!um || !up || (g->dim == 2 && (!vm || !vp))) return fail(HJW_EINVAL, "NULL output");
    hipError_t e;
    switch (g->prec) {
    case HJW_FP64:
        e = enqueue_deriv_typed<double, double>(g, um, up, vm, vp);
        break;
    case HJW_FP32_MIXED:
        e = enqueue_deriv_typed<float, double>(g, um, up, vm, vp);
        break;
    default:
        e = enqueue_deriv_typed<float, float>(g, um, up, vm, vp);
    }
    if (e != hipSuccess) return fail(HJW_EHIP, "derivative launch failed: %s", hipGetErrorString(e));
    HIP_TRY(hipStreamSynchronize(g->stream));
    return HJW_OK;
}

hjw_status hjw_get_info(const hjw_grid* g, hjw_info* info) {
    if (!g || !info) return fail(HJW_EINVAL, "NULL argument");
    fill_info(g, info);
    return HJW_OK;
}

hjw_status hjw_set_option(hjw_grid* g, int option, int64_t value) {
    if (!g) return fail(HJW_EINVAL, "grid is NULL");
    if (option == HJW_OPT_USE_GRAPH) {
        g->use_graph = value != 0;
        if (!g->use_graph) drop_graph(g);
        return HJW_OK;
    }
    if (option == HJW_OPT_DISSIPATION) {
        if (value != 0 && value != 1) return fail(HJW_EINVAL, "dissipation must be 0 or 1");
        if (value == 1 && g->dim == 2 && g->tile_rows == 32)
            return fail(HJW_EINVAL, "the local dissipation runs 16-row tiles");
        g->llf = int(value);
        drop_graph(g);
        return HJW_OK;
    }
    if (option == HJW_OPT_PLAN) {
        if (value < 0 || value > 2) return fail(HJW_EINVAL, "plan option must be 0, 1 or 2");
        g->plan_opt = int(value);
        drop_graph(g);
        return HJW_OK;
    }
    if (option == HJW_OPT_SEGMENT) {
        if (value != 0 && value != 4 && value != 8)
            return fail(HJW_EINVAL, "segment must be 0 (automatic), 4 or 8");
        if (value == 4 && (g->prec == HJW_FP64 || g->tile_rows != 16))
            return fail(HJW_EINVAL, "4-node segments need 16-row tiles and an FP32 stencil");
        g->seg_opt = int(value);
        drop_graph(g);
        return HJW_OK;
    }
    if (option == HJW_OPT_TILE_ROWS) {
        if (value != 16 && value != 32) return fail(HJW_EINVAL, "tile rows must be 16 or 32");
        if (value == 32 && g->seg_opt == 4)
            return fail(HJW_EINVAL, "32-row tiles take 8-node segments");
        if (value == 32 && g->ham_set && g->ham == HJW_H_TIMED)
            return fail(HJW_EINVAL, "the TIMED family runs 16-row tiles");
        if (value == 32 && g->llf)
            return fail(HJW_EINVAL, "the local dissipation runs 16-row tiles");
        g->tile_rows = int(value);
        if (g->dim == 2) g->nby = int((g->ny + g->tile_rows - 1) / g->tile_rows);
        drop_graph(g);
        return HJW_OK;
    }
    if (option == HJW_OPT_KERNEL_EVENTS) {
        if (value != 0 && g->ev.empty()) {
            g->ev.resize(size_t(8) * kMaxBatch, nullptr);
            g->ev_kind.resize(size_t(4) * kMaxBatch, 0);
            for (auto& e : g->ev) HIP_TRY(hipEventCreate(&e));
        }
        g->timing = value != 0;
        g->ev_used = 0;
        for (int k = 0; k < 4; ++k) {
            g->kernel_ms[k] = 0.0;
            g->kernel_count[k] = 0;
        }
        return HJW_OK;
    }
    return fail(HJW_EINVAL, "unknown option %d", option);
}

hjw_status hjw_time_kernels(hjw_grid* g, int reps, double* ms) {
    hjw_status s = check_ready(g);
    if (s != HJW_OK) return s;
    if (!g->phi_set || !g->ham_set) return fail(HJW_ESTATE, "phi or Hamiltonian not set");
    if (reps < 1 || !ms) return fail(HJW_EINVAL, "need reps >= 1 and an output array");
    // one real step towards a far target, so that every stage kernel finds an open
    // step (first stage) or a planned one (second and third stages)
    const int64_t limit = std::numeric_limits<int64_t>::max();
    hipLaunchKernelGGL(k_set_target, dim3(1), dim3(64), 0, g->stream, g->state + g->par,
                       std::numeric_limits<double>::max(), 0.5, limit);
    HIP_TRY(hipGetLastError());
    const bool timing = g->timing;
    g->timing = false;   // restored on every path below
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t err = enqueue_step(g);
    if (err == hipSuccess) err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    g->par ^= 1;   // launch against the records of the step just taken
    const bool plan = plan_launch(g);
    auto launch = [&](int k) {
        switch (g->prec) {
        case HJW_FP64:
            return launch_kind<double, double>(g, k);
        case HJW_FP32_MIXED:
            return launch_kind<float, double>(g, k);
        default:
            return launch_kind<float, float>(g, k);
        }
    };
    // about 2 ms of the wall clock: longer than the host takes to submit the launches
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
        khz = 100000;
    const int64_t hold_ticks = int64_t(khz) * 2;
    for (int k = 0; k < 4 && err == hipSuccess; ++k) {
        ms[k] = 0.0;
        if (k == 1 && !plan) continue;   // the plan runs inside the second stage
        // the GPU waits in a hold kernel while the host submits every launch, so the timed
        // ones start back to back however slowly the host submits (under a profiler, say);
        // two untimed launches after the hold bring the clocks and caches up
        hipLaunchKernelGGL(k_hold, dim3(1), dim3(64), 0, g->stream, hold_ticks);
        err = hipGetLastError();
        for (int r = 0; r < 2 && err == hipSuccess; ++r) err = launch(k);
        if (err == hipSuccess) err = hipEventRecord(e0, g->stream);
        for (int r = 0; r < reps && err == hipSuccess; ++r) err = launch(k);
        if (err == hipSuccess) err = hipEventRecord(e1, g->stream);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float t = 0.0f;
        if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
        ms[k] = double(t) / reps;
    }
    g->par ^= 1;
    g->timing = timing;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    g->phi_set = false;   // phi was overwritten by the repeated third stage
    if (err != hipSuccess) return fail(HJW_EHIP, "kernel timing failed: %s", hipGetErrorString(err));
    HIP_TRY(hipStreamSynchronize(g->stream));
    return HJW_OK;
}

hjw_status hjw_kernel_times(const hjw_grid* g, double* ms, int64_t* count) {
    if (!g || !ms || !count) return fail(HJW_EINVAL, "NULL argument");
    for (int k = 0; k < 4; ++k) {
        ms[k] = g->kernel_ms[k];
        count[k] = g->kernel_count[k];
    }
    return HJW_OK;
}

void hjw_grid_destroy(hjw_grid* g) {
    if (!g) return;
    drop_graph(g);
    for (auto& e : g->ev)
        if (e) (void)hipEventDestroy(e);
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    if (g->own_stream && g->stream) (void)hipStreamDestroy(g->stream);
    if (g->pinned) (void)hipHostFree(g->pinned);
    delete g;
}

}  // extern "C"

// ------------------------------------------------------------------ no-allocation solve
// For callers that cannot allocate device memory.  The stage buffer, the flux records, the
// range slots and the step records of one grid (and phi itself in FP32 storage) live in a
// file-scope device array instead of a bound workspace.  Each device holds its own copy of
// the array; its device address is taken once per device, with that device current, on the
// first call there.  Every call on a device reuses that device's copy: calls that overlap in
// time on one device race.
namespace {

constexpr int64_t kNoAllocNodes = int64_t(1) << 20;   // e.g. a 1024 x 1024 grid
constexpr size_t kNoAllocControl = 4096;               // range slots and step records
// FP64 is the largest case: stage buffer 8 B and flux records 24 B per node.
constexpr size_t kNoAllocBytes = size_t(kNoAllocNodes) * 32 + kNoAllocControl;
static_assert(align256(sizeof(RangeSlots)) + align256(2 * sizeof(DevState)) <= kNoAllocControl,
              "control records fit");

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex scratch_mutex;
char* scratch_ptr[kMaxDevices] = {};

// The current device's copy of `scratch` (in host code the array's own name is only a
// host-side stand-in, so its device address is looked up and kept per device).
hjw_status scratch_base(char** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(HJW_EINVAL, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(HJW_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        scratch_ptr[dev] = static_cast<char*>(p);
    }
    *out = scratch_ptr[dev];
    return HJW_OK;
}

}  // namespace

extern "C" {

hjw_status hjw_solve_noalloc(int dim, const int64_t* n, const double* lo, const double* hi,
                             const int* bc, int prec, int ham, const double* params, int nparams,
                             double* phi, double t_final, double cfl, int64_t max_steps,
                             hjw_info* info, void* stream) {
    hjw::last_error().clear();
    if (!phi) return fail(HJW_EINVAL, "phi is NULL");
    hjw_grid g;
    hjw_status st = describe_grid(&g, dim, n, lo, hi, bc, prec);
    if (st != HJW_OK) return st;
    if (g.cells() > kNoAllocNodes)
        return fail(HJW_ENOMEM, "the no-allocation solve takes at most %lld nodes (got %lld)",
                    (long long)kNoAllocNodes, (long long)g.cells());
    st = hjw_set_hamiltonian(&g, ham, params, nparams);
    if (st != HJW_OK) return st;
    char* base = nullptr;
    st = scratch_base(&base);
    if (st != HJW_OK) return st;

    // the workspace layout of a bound grid, inside the scratch array; phi is the caller's
    // array except in FP32 storage
    const size_t cells = size_t(g.cells());
    size_t o = 0;
    if (prec == HJW_FP32) {
        g.phi = base + o;
        o += align256(cells * 4);
    } else {
        g.phi = phi;
    }
    g.phi2 = base + o;
    o += align256(cells * g.elem_phi());
    g.flux = base + o;
    o += align256(3 * cells * g.elem_flux());
    g.slots = base + o;
    o += align256(sizeof(RangeSlots));
    g.state = reinterpret_cast<DevState*>(base + o);
    o += align256(2 * sizeof(DevState));
    if (o > kNoAllocBytes) return fail(HJW_ENOMEM, "scratch layout exceeds the array");
    size_t a_, b_, c_, d_, total_;
    int nbx = 0, nby = 0;
    layout(&g, &a_, &b_, &c_, &d_, &total_, &nbx, &nby);
    g.nbx = nbx;
    g.nby = g.dim == 2 ? int((g.ny + g.tile_rows - 1) / g.tile_rows) : nby;
    g.stream = static_cast<hipStream_t>(stream);
    g.use_graph = false;   // instantiating a graph allocates
    g.bound = true;

    // phi0: reset the step records and range slots (the array keeps the last call's
    // contents), check it, and convert it to FP32 storage where phi is stored so
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, g.stream, g.state,
                       static_cast<RangeSlots*>(g.slots));
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_check_finite, dim3(1024), dim3(256), 0, g.stream, phi, int64_t(cells),
                       g.state);
    HIP_TRY(hipGetLastError());
    if (prec == HJW_FP32) {
        hipLaunchKernelGGL(k_d2f, dim3(1024), dim3(256), 0, g.stream, phi,
                           static_cast<float*>(g.phi), int64_t(cells));
        HIP_TRY(hipGetLastError());
    }
    st = read_state(&g);
    if (st != HJW_OK) return st;
    if (g.last.bad) return fail(HJW_ENONFINITE, "phi0 holds non-finite values");
    g.phi_set = true;

    st = hjw_step_to(&g, t_final, cfl, max_steps, info);
    if (st != HJW_OK) return st;
    if (prec == HJW_FP32) {
        hipLaunchKernelGGL(k_f2d, dim3(1024), dim3(256), 0, g.stream,
                           static_cast<const float*>(g.phi), phi, int64_t(cells));
        HIP_TRY(hipGetLastError());
    }
    HIP_TRY(hipStreamSynchronize(g.stream));
    return HJW_OK;
}

}  // extern "C"
