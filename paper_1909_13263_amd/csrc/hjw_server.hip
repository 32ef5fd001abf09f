// hjw_server.hip - continuous batching of many WENO-L solves on one GPU.
//
// Every admitted solve keeps phi, its stage buffer, its flux records, two step
// records and its range slots resident in HBM.  A batched step is the three stage
// kernels of one RK3 step (hjw_kernels.h) launched once over the tiles of all
// admitted solves: a device-resident table gives each solve's arguments and first
// tile, and each workgroup finds its solve by binary search.  Each solve keeps its own
// dissipation and time step; solves past their t_final exit at once.  Chunks of
// batched steps are replayed from HIP graphs cached by launch size, so admission and
// retirement only rewrite the table.  The host keeps two chunks queued: while the GPU
// runs one, the host reads the step records of the one before (copied out at its end),
// retires the solves it finished (phi copied out behind the running chunk, pool space
// released at once: every later use of that space is queued after the copy) and
// admits waiting requests first-in first-out (phi0 copied in through pinned staging),
// so the GPU does not wait for the host between chunks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <limits>
#include <map>
#include <new>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "hjw.h"
#include "hjw_common.h"
#include "hjw_kernels.h"

namespace hjw {

// One batched launch of a stage over all admitted solves.  table[g] holds solve g's
// arguments with the parity it has when flip is 0; tile_start[g] is its first tile
// (tile_start[ngrids] = total tiles).  Workgroups past the last tile exit.  The launch
// size is a multiple of 8: workgroup w goes to tile (w % 8) * (size / 8) + w / 8, so that
// each XCD (dealt workgroups round-robin) works through one contiguous run of tiles and
// their shared halos stay in its L2.
template <typename T, typename P, int STAGE, int S>
__global__ __launch_bounds__(threads2d(16, S), fp64_waves(sizeof(T), 16)) void k_stage2d_batch(const StageArgs<T, P>* table,
                                                                   const int* tile_start,
                                                                   const int* ngrids, int flip,
                                                                   int plan_ready) {
    const int ng = *ngrids;
    const int b = int(blockIdx.x % 8u * (gridDim.x / 8u) + blockIdx.x / 8u);
    if (ng <= 0 || b >= tile_start[ng]) return;
    int lo = 0, hi = ng;  // tile_start[lo] <= b < tile_start[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tile_start[mid] <= b)
            lo = mid;
        else
            hi = mid;
    }
    StageArgs<T, P> a = table[lo];
    a.par ^= flip;
    a.plan_ready = plan_ready;
    // the second stage writes phi_2, the third phi^{n+1} over phi^n
    if (STAGE == kStageMid) a.out = const_cast<P*>(a.phi_s);
    if (STAGE == kStageLast) a.out = const_cast<P*>(a.phi_n);
    // one launch serves solves of every family, the time- and phi-dependent one included
    stage_tile2d<T, P, STAGE, 16, S, true>(a, b - tile_start[lo]);
}

// The step plans of all admitted solves, one wave each (workgroup g plans solve g).
template <typename T, typename P>
__global__ __launch_bounds__(64) void k_plan_batch(const StageArgs<T, P>* table,
                                                   const int* ngrids, int flip) {
    if (int(blockIdx.x) >= *ngrids) return;
    StageArgs<T, P> a = table[blockIdx.x];
    a.par ^= flip;
    a.plan_ready = 0;   // this launch is the one that publishes the plan
    double dt, ax, ay;
    (void)plan_in_block(a, 0, dt, ax, ay);
}

// A newly admitted solve: record 0 is current (t = 0, target t_final), slots empty.
__global__ void k_admit(DevState* st, RangeSlots* sl, double t_final, double cfl) {
    if (threadIdx.x < 2) {
        DevState s;
        s.t = 0.0;
        s.t_final = t_final;
        s.cfl = cfl;
        s.dt = 0.0;
        s.alpha_x = 0.0;
        s.alpha_y = 0.0;
        for (int k = 0; k < 4; ++k) s.range[k] = 0.0;
        s.steps = 0;
        s.steps_left = INT64_MAX;
        s.active = 0;
        s.bad = 0;
        s.pad[0] = s.pad[1] = 0;
        st[threadIdx.x] = s;
    }
    if (threadIdx.x < kSlots) {
        const int k = threadIdx.x;
        sl->key[0][k] = ~0ull;
        sl->key[1][k] = 0ull;
        sl->key[2][k] = ~0ull;
        sl->key[3][k] = 0ull;
        sl->bad[k] = 0u;
    }
}

}  // namespace hjw

using namespace hjw;

namespace {

constexpr int kChunkSteps = 8;    // batched steps per chunk (even: replays keep the parity)
constexpr int kTileBucket = 128;  // smallest launch, in tiles
constexpr size_t kGraphCache = 12;
constexpr int kTY = 16;
constexpr int kInFlight = 2;      // chunks queued on the stream at most
// Bytes of phi0 (or of results) moved through one pinned staging buffer per processing
// step; more waits for the next step (one solve larger than this always moves alone).
constexpr size_t kStageCap = size_t(256) << 20;
// Pinned host memory that queued phi0 arrays are copied into at submission, so that
// admission copies them to the pool directly: a quarter of the pool, at most 1 GiB.
constexpr size_t kInboxMax = size_t(1) << 30;

// Copies n values and reports whether all are finite (exponent field not all ones): one
// pass over the caller's array instead of a test and then a copy.
bool copy_finite(double* dst, const double* src, int64_t n) {
    constexpr uint64_t kExp = 0x7ff0000000000000ull;
    uint64_t bad = 0;
    for (int64_t k = 0; k < n; ++k) {
        uint64_t u;
        std::memcpy(&u, src + k, sizeof u);
        bad |= uint64_t((u & kExp) == kExp);
        std::memcpy(dst + k, &u, sizeof u);
    }
    return bad == 0;
}

double seconds_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// First-fit allocator over [0, size) in 256-byte units, coalescing on release.
class PoolMap {
public:
    void reset(size_t size) {
        free_.clear();
        if (size) free_[0] = size;
    }
    size_t alloc(size_t bytes) {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const size_t off = it->first, rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                return off;
            }
        }
        return SIZE_MAX;
    }
    void release(size_t off, size_t bytes) {
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }

private:
    std::map<size_t, size_t> free_;
};

struct Req {
    int64_t id = 0;
    hjw_request r{};
    std::vector<double> phi0;
    double t_submit = 0.0, t_finish = 0.0;
    int state = 0;  // 0 queued, 1 admitted, 2 finished, 3 result being copied out
    hjw_status status = HJW_OK;
    std::vector<double> result;
    hjw_info info{};
    size_t off = 0, bytes = 0;
    int slot = -1, tiles = 0, par0 = 0;
    int64_t cells = 0, steps_seen = 0;
    int64_t first_chunk = 0;   // the first chunk whose table holds this solve
    int res_buf = -1;          // pinned staging buffer holding its result (state 3)
    size_t res_off = 0;
    size_t in_off = SIZE_MAX;  // its phi0 in the pinned inbox (else in phi0)
    size_t in_bytes = 0;
};

// A pinned host buffer for copies between the pool and host memory that must not wait:
// reused only after the copies issued from it (marked by its event) have completed.
struct Staging {
    char* p = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
    std::vector<int64_t> ids;   // results held (download buffers)
    std::vector<std::pair<size_t, size_t>> inbox;   // inbox blocks read by its copies
};

struct GraphEntry {
    int tiles;
    int flip;
    hipGraphExec_t exec;
    uint64_t used;
};

size_t elem_phi(int prec) { return prec == HJW_FP32 ? 4 : 8; }
size_t elem_flux(int prec) { return prec == HJW_FP64 ? 8 : 4; }

size_t footprint(int prec, const hjw_request& r) {
    const size_t n = size_t(r.n[0]) * size_t(r.n[1]);
    return 2 * align256(n * elem_phi(prec)) + align256(std::max(3 * n * elem_flux(prec), 8 * n));
}

size_t entry_bytes(int prec) {
    switch (prec) {
    case HJW_FP64:
        return sizeof(StageArgs<double, double>);
    case HJW_FP32_MIXED:
        return sizeof(StageArgs<float, double>);
    default:
        return sizeof(StageArgs<float, float>);
    }
}

hjw_status validate(const hjw_request& r) {
    for (int d = 0; d < 2; ++d) {
        if (r.n[d] < 8 || r.n[d] > (int64_t(1) << 20))
            return fail(HJW_EINVAL, "request axis %d: n = %lld out of range", d,
                        (long long)r.n[d]);
        if (!(r.hi[d] > r.lo[d]) || !std::isfinite(r.lo[d]) || !std::isfinite(r.hi[d]))
            return fail(HJW_EINVAL, "request axis %d: need finite lo < hi", d);
        if (r.bc[d] != HJW_BC_PERIODIC && r.bc[d] != HJW_BC_EXTRAP &&
            r.bc[d] != HJW_BC_DIRICHLET)
            return fail(HJW_EINVAL, "request axis %d: unknown boundary %d", d, r.bc[d]);
    }
    if (r.ham < HJW_H_LINEAR || r.ham > HJW_H_TIMED)
        return fail(HJW_EINVAL, "unknown Hamiltonian %d", r.ham);
    if (r.scheme != HJW_WENO_L && r.scheme != HJW_WENO_JP)
        return fail(HJW_EINVAL, "unknown scheme %d", r.scheme);
    for (int k = 0; k < 4; ++k)
        if (!std::isfinite(r.params[k])) return fail(HJW_EINVAL, "non-finite parameter");
    if ((r.ham == HJW_H_NORM || r.ham == HJW_H_CURVATURE) && r.params[1] < 0.0)
        return fail(HJW_EINVAL, "NORM needs p[1] >= 0");
    if (r.ham == HJW_H_CURVATURE &&
        (r.bc[0] == HJW_BC_EXTRAP || r.bc[1] == HJW_BC_EXTRAP || r.params[2] < 0.0))
        return fail(HJW_EINVAL, "CURVATURE needs periodic or Dirichlet axes and eps >= 0");
    if (!std::isfinite(r.t_final) || r.t_final < 0.0 || !(r.cfl > 0.0) || !std::isfinite(r.cfl))
        return fail(HJW_EINVAL, "need finite t_final >= 0 and cfl > 0");
    return HJW_OK;
}

}  // namespace

struct hjw_server {
    int prec = HJW_FP32_MIXED;
    char* base = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int max_active = 0;

    // control area at the head of the pool
    void* d_table = nullptr;
    int* d_tile_start = nullptr;
    int* d_ngrids = nullptr;
    DevState* d_states = nullptr;   // 2 records per slot
    RangeSlots* d_slots = nullptr;
    // pinned mirrors of the table, two sets: the host fills one while an upload from the
    // other may still be in flight
    char* h_table[2] = {nullptr, nullptr};
    int* h_tile_start[2] = {nullptr, nullptr};
    int* h_ngrids[2] = {nullptr, nullptr};
    hipEvent_t tab_ev[2] = {nullptr, nullptr};
    bool tab_pending[2] = {false, false};
    int tab_buf = 0;
    // step records of every slot, copied out at the end of each chunk (buffer chunk % 2)
    DevState* h_rec[kInFlight] = {};
    hipEvent_t rec_ev[kInFlight] = {};
    std::deque<int64_t> inflight;   // chunks queued on the stream, oldest first
    int64_t next_chunk = 0;
    // pinned staging of phi0 uploads and result downloads, alternating by processing step
    Staging up[2], down[2];
    int64_t step_no = 0;
    hipStream_t capture = nullptr;  // graphs are captured here (nothing runs on it)

    size_t heap_off = 0, heap_bytes = 0, in_use = 0, peak = 0;
    PoolMap heap;
    char* inbox = nullptr;   // pinned; blocks return once the copies reading them are done
    PoolMap inbox_map;
    std::vector<int> free_slots;
    std::deque<int64_t> queue;
    std::vector<int64_t> active;  // table order
    std::unordered_map<int64_t, Req> reqs;
    std::vector<int64_t> completed;
    int64_t next_id = 1;
    int flip = 0;
    bool table_dirty = true;
    int launch_tiles = 0;
    std::vector<GraphEntry> graphs;
    uint64_t use_clock = 0;
    hjw_server_stats stats{};
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
};

namespace {

// Launch sizes: the total tile count rounded up to one of eight steps per octave (at
// least kTileBucket), so that few graphs cover every mix and at most 1/8 of the
// workgroups of a launch find no tile.
int launch_size(int tiles) {
    if (tiles <= kTileBucket) return kTileBucket;
    int step = kTileBucket;
    while (step * 16 <= tiles) step *= 2;   // step = 2^floor(log2 tiles) / 8, >= kTileBucket
    return (tiles + step - 1) / step * step;
}

template <typename T, typename P>
StageArgs<T, P> request_args(const hjw_server* s, const Req& q) {
    const hjw_request& r = q.r;
    const size_t n = size_t(q.cells);
    char* w = s->base + s->heap_off + q.off;
    StageArgs<T, P> a{};
    a.phi_n = reinterpret_cast<const P*>(w);
    a.phi_s = reinterpret_cast<const P*>(w + align256(n * sizeof(P)));
    a.out = nullptr;  // chosen per stage by the batched kernel
    a.flux = reinterpret_cast<T*>(w + 2 * align256(n * sizeof(P)));
    a.st = s->d_states + 2 * q.slot;
    a.par = q.par0;
    a.slots = s->d_slots + q.slot;
    a.nx = r.n[0];
    a.ny = r.n[1];
    a.bcx = r.bc[0];
    a.bcy = r.bc[1];
    const double dx = (r.hi[0] - r.lo[0]) / double(r.n[0]);
    const double dy = (r.hi[1] - r.lo[1]) / double(r.n[1]);
    a.ihx = P(1.0 / dx);
    a.ihy = P(1.0 / dy);
    a.ihxT = T(1.0 / dx);
    a.ihyT = T(1.0 / dy);
    a.epsx = T(weight_eps(r.scheme, dx));
    a.epsy = T(weight_eps(r.scheme, dy));
    a.scheme = r.scheme;
    a.ham = r.ham;
    for (int k = 0; k < 4; ++k) {
        a.hpT[k] = T(r.params[k]);
        a.hpD[k] = r.params[k];
    }
    a.ihxD = 1.0 / dx;
    a.ihyD = 1.0 / dy;
    a.x0 = r.lo[0] + (r.bc[0] == HJW_BC_EXTRAP ? 0.5 * dx : 0.0);
    a.y0 = r.lo[1] + (r.bc[1] == HJW_BC_EXTRAP ? 0.5 * dy : 0.0);
    a.dxD = dx;
    a.dyD = dy;
    a.nbx = int((r.n[0] + kTX - 1) / kTX);
    a.nby = int((r.n[1] + kTY - 1) / kTY);
    a.remap = 0;
    a.dim = 2;
    return a;
}

template <typename T, typename P>
void write_table(hjw_server* s, int b) {
    StageArgs<T, P>* tab = reinterpret_cast<StageArgs<T, P>*>(s->h_table[b]);
    int tiles = 0;
    for (size_t g = 0; g < s->active.size(); ++g) {
        const Req& q = s->reqs.at(s->active[g]);
        tab[g] = request_args<T, P>(s, q);
        s->h_tile_start[b][g] = tiles;
        tiles += q.tiles;
    }
    s->h_tile_start[b][s->active.size()] = tiles;
    *s->h_ngrids[b] = int(s->active.size());
    s->launch_tiles = launch_size(tiles);
}

// Launches of more than kPlanLaunchTiles tiles plan every solve's step in a launch of its
// own (one wave per solve) instead of in every workgroup of the second stage.
constexpr int kPlanLaunchTiles = 2048;

template <typename T, typename P, int S>
hipError_t launch_batched_step_s(hjw_server* s, int flip, hipStream_t stream) {
    const StageArgs<T, P>* tab = static_cast<const StageArgs<T, P>*>(s->d_table);
    const dim3 grid(unsigned(s->launch_tiles)), block(threads2d(kTY, S));
    const int plan = s->launch_tiles > kPlanLaunchTiles ? 1 : 0;
    hipLaunchKernelGGL((k_stage2d_batch<T, P, kStagePre, S>), grid, block, 0, stream, tab,
                       s->d_tile_start, s->d_ngrids, flip, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (plan) {
        hipLaunchKernelGGL((k_plan_batch<T, P>), dim3(unsigned(s->max_active)), dim3(64), 0,
                           stream, tab, s->d_ngrids, flip);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_stage2d_batch<T, P, kStageMid, S>), grid, block, 0, stream, tab,
                       s->d_tile_start, s->d_ngrids, flip, plan);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_stage2d_batch<T, P, kStageLast, S>), grid, block, 0, stream, tab,
                       s->d_tile_start, s->d_ngrids, flip, 0);
    return hipGetLastError();
}

// Launches of at most kSmallLaunch tiles use 4-node segments with the FP32 stencil (twice
// the waves), as a single grid of that size would; both give the same bits.
constexpr int kSmallLaunch = 640;

template <typename T, typename P>
hipError_t launch_batched_step(hjw_server* s, int flip, hipStream_t stream) {
    if (!std::is_same<T, double>::value && s->launch_tiles <= kSmallLaunch)
        return launch_batched_step_s<T, P, std::is_same<T, double>::value ? 8 : 4>(s, flip,
                                                                                   stream);
    return launch_batched_step_s<T, P, 8>(s, flip, stream);
}

hipError_t batched_step(hjw_server* s, int flip, hipStream_t stream) {
    switch (s->prec) {
    case HJW_FP64:
        return launch_batched_step<double, double>(s, flip, stream);
    case HJW_FP32_MIXED:
        return launch_batched_step<float, double>(s, flip, stream);
    default:
        return launch_batched_step<float, float>(s, flip, stream);
    }
}

void rebuild_table(hjw_server* s, int b) {
    switch (s->prec) {
    case HJW_FP64:
        write_table<double, double>(s, b);
        break;
    case HJW_FP32_MIXED:
        write_table<float, double>(s, b);
        break;
    default:
        write_table<float, float>(s, b);
    }
}

// The table of the solves admitted now, from the pinned mirror not used last time (its
// previous upload is waited for), queued behind the chunks already on the stream.
hjw_status upload_table(hjw_server* s) {
    const int b = s->tab_buf ^= 1;
    if (s->tab_pending[b]) {
        HIP_TRY(hipEventSynchronize(s->tab_ev[b]));
        s->tab_pending[b] = false;
    }
    rebuild_table(s, b);
    const size_t ng = s->active.size();
    if (ng)
        HIP_TRY(hipMemcpyAsync(s->d_table, s->h_table[b], ng * entry_bytes(s->prec),
                               hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(s->d_tile_start, s->h_tile_start[b], (ng + 1) * sizeof(int),
                           hipMemcpyHostToDevice, s->stream));
    HIP_TRY(hipMemcpyAsync(s->d_ngrids, s->h_ngrids[b], sizeof(int), hipMemcpyHostToDevice,
                           s->stream));
    HIP_TRY(hipEventRecord(s->tab_ev[b], s->stream));
    s->tab_pending[b] = true;
    s->table_dirty = false;
    return HJW_OK;
}

// Room for `need` bytes in a staging buffer whose copies have completed.
hjw_status reserve(Staging& b, size_t need) {
    if (need <= b.cap) return HJW_OK;
    const size_t cap = std::max(need, std::max(size_t(16) << 20, 2 * b.cap));
    if (b.p) HIP_TRY(hipHostFree(b.p));
    b.p = nullptr;
    b.cap = 0;
    if (hipHostMalloc(reinterpret_cast<void**>(&b.p), cap, hipHostMallocDefault) != hipSuccess) {
        b.p = nullptr;
        return fail(HJW_ENOMEM, "hipHostMalloc of %zu staging bytes failed", cap);
    }
    b.cap = cap;
    return HJW_OK;
}

// Results whose copies out have completed move to host memory and are reported
// finished; with wait, the copies of buffer `only` (or of both, -1) are waited for.
hjw_status finish_downloads(hjw_server* s, bool wait, int only = -1) {
    for (int b = 0; b < 2; ++b) {
        Staging& d = s->down[b];
        if (!d.pending || (only >= 0 && b != only)) continue;
        if (wait) {
            HIP_TRY(hipEventSynchronize(d.ev));
        } else {
            const hipError_t e = hipEventQuery(d.ev);
            if (e == hipErrorNotReady) continue;
            if (e != hipSuccess) return fail(HJW_EHIP, "hipEventQuery: %s", hipGetErrorString(e));
        }
        const double now = seconds_since(s->t0);
        for (int64_t id : d.ids) {
            Req& q = s->reqs.at(id);
            q.result.resize(size_t(q.cells));
            std::memcpy(q.result.data(), d.p + q.res_off, size_t(q.cells) * sizeof(double));
            q.res_buf = -1;
            q.state = 2;
            q.t_finish = now;
            s->completed.push_back(id);
        }
        d.ids.clear();
        d.pending = false;
    }
    return HJW_OK;
}

// Inbox blocks read by the copies of an upload buffer whose event has completed.
void reclaim_inbox(hjw_server* s, Staging& up) {
    for (const auto& blk : up.inbox) s->inbox_map.release(blk.first, blk.second);
    up.inbox.clear();
}

// Admit waiting requests first-in first-out while a slot and pool space are free, and
// for phi0 not held in the inbox, room in this step's upload staging (kStageCap, or one
// larger request alone); phi0 is copied in behind the queued chunks.
hjw_status admit(hjw_server* s, Staging& up) {
    if (up.pending) {
        HIP_TRY(hipEventSynchronize(up.ev));
        up.pending = false;
    }
    reclaim_inbox(s, up);
    std::vector<int64_t> take;
    size_t total = 0;
    for (int64_t id : s->queue) {
        Req& q = s->reqs.at(id);
        const bool staged = q.in_off == SIZE_MAX;
        const size_t nb = staged ? align256(size_t(q.cells) * sizeof(double)) : 0;
        if (take.size() >= s->free_slots.size()) break;
        if (staged && total > 0 && total + nb > kStageCap) break;   // the next step takes it
        const size_t off = s->heap.alloc(q.bytes);
        if (off == SIZE_MAX) break;  // first in, first out: wait for space
        q.off = off;
        q.res_off = total;           // its place in the upload staging
        take.push_back(id);
        total += nb;
    }
    if (take.empty()) return s->table_dirty ? upload_table(s) : HJW_OK;
    hjw_status st = reserve(up, total);
    if (st != HJW_OK) {
        for (int64_t id : take) s->heap.release(s->reqs.at(id).off, s->reqs.at(id).bytes);
        return st;
    }
    for (int64_t id : take) {
        Req& q = s->reqs.at(id);
        const size_t n = size_t(q.cells);
        char* src = q.in_off == SIZE_MAX ? up.p + q.res_off : s->inbox + q.in_off;
        q.res_off = 0;
        q.slot = s->free_slots.back();
        s->free_slots.pop_back();
        q.par0 = s->flip;  // its record 0 is current at the next launch
        q.state = 1;
        q.steps_seen = 0;
        q.first_chunk = s->next_chunk;
        s->in_use += q.bytes;
        s->peak = std::max(s->peak, s->in_use);
        if (q.in_off == SIZE_MAX) {
            std::memcpy(src, q.phi0.data(), n * sizeof(double));
            std::vector<double>().swap(q.phi0);
        } else {
            up.inbox.emplace_back(q.in_off, q.in_bytes);   // returned after up.ev
            q.in_off = SIZE_MAX;
        }
        char* w = s->base + s->heap_off + q.off;
        if (s->prec == HJW_FP32) {
            double* stage = reinterpret_cast<double*>(w + 2 * align256(n * 4));
            HIP_TRY(hipMemcpyAsync(stage, src, n * sizeof(double), hipMemcpyHostToDevice,
                                   s->stream));
            hipLaunchKernelGGL(k_d2f, dim3(256), dim3(256), 0, s->stream, stage,
                               reinterpret_cast<float*>(w), int64_t(n));
            HIP_TRY(hipGetLastError());
        } else {
            HIP_TRY(hipMemcpyAsync(w, src, n * sizeof(double), hipMemcpyHostToDevice, s->stream));
        }
        hipLaunchKernelGGL(k_admit, dim3(1), dim3(64), 0, s->stream, s->d_states + 2 * q.slot,
                           s->d_slots + q.slot, q.r.t_final, q.r.cfl);
        HIP_TRY(hipGetLastError());
        s->active.push_back(q.id);
        s->queue.pop_front();
    }
    HIP_TRY(hipEventRecord(up.ev, s->stream));
    up.pending = true;
    return upload_table(s);
}

void drop_graphs(hjw_server* s) {
    for (auto& g : s->graphs) (void)hipGraphExecDestroy(g.exec);
    s->graphs.clear();
}

// Queue one chunk (a cached graph of kChunkSteps batched steps for this launch size and
// parity) and the copy of every slot's step records behind it.
hjw_status launch_chunk(hjw_server* s) {
    GraphEntry* ge = nullptr;
    for (auto& g : s->graphs)
        if (g.tiles == s->launch_tiles && g.flip == s->flip) ge = &g;
    if (!ge) {
        if (s->graphs.size() >= kGraphCache) {
            auto lru = std::min_element(s->graphs.begin(), s->graphs.end(),
                                        [](const GraphEntry& a, const GraphEntry& b) {
                                            return a.used < b.used;
                                        });
            (void)hipGraphExecDestroy(lru->exec);
            s->graphs.erase(lru);
        }
        hipGraph_t graph = nullptr;
        HIP_TRY(hipStreamBeginCapture(s->capture, hipStreamCaptureModeRelaxed));
        hipError_t e = hipSuccess;
        int f = s->flip;
        for (int k = 0; k < kChunkSteps && e == hipSuccess; ++k, f ^= 1)
            e = batched_step(s, f, s->capture);
        const hipError_t e2 = hipStreamEndCapture(s->capture, &graph);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return fail(HJW_EHIP, "batched graph capture failed: %s / %s", hipGetErrorString(e),
                        hipGetErrorString(e2));
        }
        hipGraphExec_t exec = nullptr;
        const hipError_t e3 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e3 != hipSuccess)
            return fail(HJW_EHIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e3));
        s->graphs.push_back(GraphEntry{s->launch_tiles, s->flip, exec, 0});
        ge = &s->graphs.back();
    }
    ge->used = ++s->use_clock;
    const int64_t c = s->next_chunk++;
    const int b = int(c % kInFlight);
    HIP_TRY(hipGraphLaunch(ge->exec, s->stream));
    HIP_TRY(hipMemcpyAsync(s->h_rec[b], s->d_states, 2 * size_t(s->max_active) * sizeof(DevState),
                           hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipEventRecord(s->rec_ev[b], s->stream));
    s->inflight.push_back(c);
    s->stats.batched_steps += kChunkSteps;  // kChunkSteps is even: the parity is unchanged
    return HJW_OK;
}

// The oldest queued chunk has ended: read its step records, retire the solves it
// finished (their phi copied out behind the chunks still queued, their pool space and
// slot free at once: whatever reuses them is queued after that copy) and admit.
// Solves admitted after that chunk was queued have no record in it yet.
hjw_status process_chunk(hjw_server* s) {
    const int64_t c = s->inflight.front();
    s->inflight.pop_front();
    const DevState* rec_all = s->h_rec[c % kInFlight];
    HIP_TRY(hipEventSynchronize(s->rec_ev[c % kInFlight]));
    hjw_status st = finish_downloads(s, false);
    if (st != HJW_OK) return st;
    const int b = int(s->step_no++ & 1);
    Staging& down = s->down[b];
    st = finish_downloads(s, true, b);
    if (st != HJW_OK) return st;
    // which solves retire now: every failed one, and finished ones while their results
    // fit one staging buffer (kStageCap, or one larger result alone); the others retire
    // at the next step (their steps are closed, so the chunks between change nothing)
    std::vector<int64_t> keep, out;
    keep.reserve(s->active.size());
    size_t total = 0;
    for (int64_t id : s->active) {
        Req& q = s->reqs.at(id);
        if (q.first_chunk > c) {
            keep.push_back(id);
            continue;
        }
        const DevState& rec = rec_all[2 * q.slot + (q.par0 ^ s->flip)];
        s->stats.node_stages += 3.0 * double(q.cells) * double(rec.steps - q.steps_seen);
        q.steps_seen = rec.steps;
        const bool bad = rec.bad != 0;
        const size_t nb = align256(size_t(q.cells) * sizeof(double));
        if ((!bad && rec.t < q.r.t_final) || (!bad && total > 0 && total + nb > kStageCap)) {
            keep.push_back(id);
            continue;
        }
        q.info.steps = rec.steps;
        q.info.t = rec.t;
        q.info.last_dt = rec.dt;
        q.info.alpha_x = rec.alpha_x;
        q.info.alpha_y = rec.alpha_y;
        for (int k = 0; k < 4; ++k) q.info.range[k] = rec.range[k];
        q.status = bad ? HJW_ENONFINITE : HJW_OK;
        if (!bad) {
            q.res_off = total;
            total += nb;
        }
        out.push_back(id);
    }
    st = reserve(down, total);
    if (st != HJW_OK) return st;
    for (int64_t id : out) {
        Req& q = s->reqs.at(id);
        const size_t n = size_t(q.cells);
        char* w = s->base + s->heap_off + q.off;
        if (q.status != HJW_OK) {
            q.state = 2;
            q.t_finish = seconds_since(s->t0);
            s->completed.push_back(id);
            s->stats.failed += 1;
        } else {
            const void* src = w;
            if (s->prec == HJW_FP32) {
                double* stage = reinterpret_cast<double*>(w + 2 * align256(n * 4));
                hipLaunchKernelGGL(k_f2d, dim3(256), dim3(256), 0, s->stream,
                                   reinterpret_cast<const float*>(w), stage, int64_t(n));
                HIP_TRY(hipGetLastError());
                src = stage;
            }
            HIP_TRY(hipMemcpyAsync(down.p + q.res_off, src, n * sizeof(double),
                                   hipMemcpyDeviceToHost, s->stream));
            q.state = 3;
            q.res_buf = b;
            down.ids.push_back(id);
            s->stats.done += 1;
        }
        s->heap.release(q.off, q.bytes);
        s->in_use -= q.bytes;
        s->free_slots.push_back(q.slot);
        q.slot = -1;
        s->table_dirty = true;
    }
    if (!down.ids.empty()) {
        HIP_TRY(hipEventRecord(down.ev, s->stream));
        down.pending = true;
    }
    s->active.swap(keep);
    return admit(s, s->up[b]);
}

}  // namespace

extern "C" {

hjw_status hjw_server_footprint(int prec, const hjw_request* req, size_t* bytes) {
    if (!req || !bytes) return fail(HJW_EINVAL, "NULL argument");
    if (prec < HJW_FP64 || prec > HJW_FP32) return fail(HJW_EINVAL, "unknown precision %d", prec);
    hjw_status st = validate(*req);
    if (st != HJW_OK) return st;
    *bytes = footprint(prec, *req);
    return HJW_OK;
}

hjw_status hjw_server_create(int prec, void* pool, size_t pool_bytes, int max_active,
                             void* stream, hjw_server** out) {
    hjw::last_error().clear();
    if (!out || !pool) return fail(HJW_EINVAL, "NULL argument");
    *out = nullptr;
    if (prec < HJW_FP64 || prec > HJW_FP32) return fail(HJW_EINVAL, "unknown precision %d", prec);
    if (max_active < 1 || max_active > 1024) return fail(HJW_EINVAL, "max_active must be 1..1024");
    if (reinterpret_cast<uintptr_t>(pool) % 256 != 0)
        return fail(HJW_EINVAL, "pool must be 256-byte aligned");
    const size_t ctl = align256(size_t(max_active) * entry_bytes(prec)) +
                       align256(size_t(max_active + 1) * sizeof(int)) + align256(sizeof(int)) +
                       align256(2 * size_t(max_active) * sizeof(DevState)) +
                       align256(size_t(max_active) * sizeof(RangeSlots));
    if (pool_bytes < ctl + 4096) return fail(HJW_ENOMEM, "pool too small for %d slots", max_active);
    hjw_server* s = new (std::nothrow) hjw_server();
    if (!s) return fail(HJW_ENOMEM, "host allocation failed");
    s->prec = prec;
    s->base = static_cast<char*>(pool);
    s->bytes = pool_bytes;
    s->max_active = max_active;
    size_t o = 0;
    s->d_table = s->base + o;
    o += align256(size_t(max_active) * entry_bytes(prec));
    s->d_tile_start = reinterpret_cast<int*>(s->base + o);
    o += align256(size_t(max_active + 1) * sizeof(int));
    s->d_ngrids = reinterpret_cast<int*>(s->base + o);
    o += align256(sizeof(int));
    s->d_states = reinterpret_cast<DevState*>(s->base + o);
    o += align256(2 * size_t(max_active) * sizeof(DevState));
    s->d_slots = reinterpret_cast<RangeSlots*>(s->base + o);
    o += align256(size_t(max_active) * sizeof(RangeSlots));
    s->heap_off = o;
    s->heap_bytes = pool_bytes - o;
    s->heap.reset(s->heap_bytes / 256 * 256);
    // the inbox is an optimisation: without it phi0 waits in ordinary host memory
    const size_t inbox = std::min(kInboxMax, s->heap_bytes / 4 / 256 * 256);
    if (inbox >= (size_t(1) << 20)) {
        if (hipHostMalloc(reinterpret_cast<void**>(&s->inbox), inbox, hipHostMallocDefault) ==
            hipSuccess) {
            // touch every page now: the first writes to fresh pinned pages cost a page
            // fault each, which would otherwise fall on the first burst of submissions
            std::memset(s->inbox, 0, inbox);
            s->inbox_map.reset(inbox);
        } else {
            s->inbox = nullptr;
            (void)hipGetLastError();   // leave no error behind for the next check
        }
    }
    for (int k = max_active - 1; k >= 0; --k) s->free_slots.push_back(k);
    hjw_status st = HJW_OK;
    s->stream = static_cast<hipStream_t>(stream);
    if (!s->stream) {
        if (hipStreamCreate(&s->stream) != hipSuccess) st = fail(HJW_EHIP, "hipStreamCreate failed");
        s->own_stream = true;
    }
    if (st == HJW_OK && hipStreamCreate(&s->capture) != hipSuccess) {
        s->capture = nullptr;
        st = fail(HJW_EHIP, "hipStreamCreate failed");
    }
    auto pinned = [](void* p, size_t bytes) {
        return hipHostMalloc(reinterpret_cast<void**>(p), bytes, hipHostMallocDefault) ==
               hipSuccess;
    };
    auto event = [](hipEvent_t* e) {
        return hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess;
    };
    for (int b = 0; b < 2 && st == HJW_OK; ++b) {
        if (!pinned(&s->h_table[b], size_t(max_active) * entry_bytes(prec)) ||
            !pinned(&s->h_tile_start[b], size_t(max_active + 1) * sizeof(int)) ||
            !pinned(&s->h_ngrids[b], sizeof(int)))
            st = fail(HJW_EHIP, "hipHostMalloc failed");
        else if (!event(&s->tab_ev[b]) || !event(&s->up[b].ev) || !event(&s->down[b].ev))
            st = fail(HJW_EHIP, "hipEventCreate failed");
    }
    for (int b = 0; b < kInFlight && st == HJW_OK; ++b) {
        if (!pinned(&s->h_rec[b], 2 * size_t(max_active) * sizeof(DevState)))
            st = fail(HJW_EHIP, "hipHostMalloc failed");
        else if (!event(&s->rec_ev[b]))
            st = fail(HJW_EHIP, "hipEventCreate failed");
    }
    if (st == HJW_OK) st = upload_table(s);
    if (st == HJW_OK && hipStreamSynchronize(s->stream) != hipSuccess)
        st = fail(HJW_EHIP, "hipStreamSynchronize failed");
    if (st != HJW_OK) {
        hjw_server_destroy(s);
        return st;
    }
    s->stats.pool_bytes = s->heap_bytes;
    *out = s;
    return HJW_OK;
}

hjw_status hjw_server_submit(hjw_server* s, const hjw_request* req, const double* phi0,
                             int64_t* id) {
    if (!s || !req || !phi0 || !id) return fail(HJW_EINVAL, "NULL argument");
    hjw_status st = validate(*req);
    if (st != HJW_OK) return st;
    const size_t bytes = footprint(s->prec, *req);
    if (bytes > s->heap_bytes)
        return fail(HJW_ENOMEM, "request needs %zu pool bytes, the pool has %zu", bytes,
                    s->heap_bytes);
    const int64_t n = req->n[0] * req->n[1];
    Req q;
    // phi0 goes to the pinned inbox when a block is free (after returning the blocks of
    // uploads that have completed), else to host memory of its own
    const size_t in_bytes = align256(size_t(n) * sizeof(double));
    if (s->inbox) {
        q.in_off = s->inbox_map.alloc(in_bytes);
        for (int b = 0; b < 2 && q.in_off == SIZE_MAX; ++b) {
            Staging& up = s->up[b];
            if (!up.pending) continue;
            const hipError_t e = hipEventQuery(up.ev);
            if (e == hipErrorNotReady) continue;
            if (e != hipSuccess) return fail(HJW_EHIP, "hipEventQuery: %s", hipGetErrorString(e));
            up.pending = false;
            reclaim_inbox(s, up);
            q.in_off = s->inbox_map.alloc(in_bytes);
        }
    }
    if (q.in_off != SIZE_MAX) {
        q.in_bytes = in_bytes;
        if (!copy_finite(reinterpret_cast<double*>(s->inbox + q.in_off), phi0, n)) {
            s->inbox_map.release(q.in_off, in_bytes);
            return fail(HJW_ENONFINITE, "phi0 holds non-finite values");
        }
    } else {
        q.phi0.resize(size_t(n));
        if (!copy_finite(q.phi0.data(), phi0, n))
            return fail(HJW_ENONFINITE, "phi0 holds non-finite values");
    }
    q.id = s->next_id++;
    q.r = *req;
    q.t_submit = seconds_since(s->t0);
    q.bytes = bytes;
    q.cells = n;
    q.tiles = int(((req->n[0] + kTX - 1) / kTX) * ((req->n[1] + kTY - 1) / kTY));
    *id = q.id;
    s->queue.push_back(q.id);
    s->reqs.emplace(q.id, std::move(q));
    s->stats.submitted += 1;
    return HJW_OK;
}

hjw_status hjw_server_run(hjw_server* s, int chunks, int64_t* active, int64_t* queued) {
    if (!s) return fail(HJW_EINVAL, "NULL server");
    hjw_status st = HJW_OK;
    if (s->inflight.empty()) st = admit(s, s->up[s->step_no & 1]);
    for (int c = 0; st == HJW_OK && c < chunks && !(s->active.empty() && s->inflight.empty());
         ++c) {
        // keep kInFlight chunks queued while anything is admitted, then wait for the oldest
        while (st == HJW_OK && !s->active.empty() && int(s->inflight.size()) < kInFlight)
            st = launch_chunk(s);
        if (st == HJW_OK) st = process_chunk(s);
    }
    // with nothing admitted, let the queued chunks end and every result reach host memory
    while (st == HJW_OK && s->active.empty() && !s->inflight.empty()) st = process_chunk(s);
    if (st == HJW_OK && s->active.empty()) st = finish_downloads(s, true);
    if (active) *active = int64_t(s->active.size());
    if (queued) *queued = int64_t(s->queue.size());
    return st;
}

hjw_status hjw_server_completed(hjw_server* s, int64_t* ids, int cap, int* count) {
    if (!s || !count || (cap > 0 && !ids)) return fail(HJW_EINVAL, "NULL argument");
    const int n = std::min<int>(cap, int(s->completed.size()));
    for (int k = 0; k < n; ++k) ids[k] = s->completed[k];
    s->completed.erase(s->completed.begin(), s->completed.begin() + n);
    *count = n;
    return HJW_OK;
}

hjw_status hjw_server_result(hjw_server* s, int64_t id, double* phi_out, hjw_info* info,
                             double* t_submit, double* t_finish) {
    if (!s) return fail(HJW_EINVAL, "NULL server");
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return fail(HJW_EINVAL, "unknown request %lld", (long long)id);
    Req& q = it->second;
    if (q.state != 2) return fail(HJW_ESTATE, "request %lld is not finished", (long long)id);
    if (phi_out && !q.result.empty()) std::memcpy(phi_out, q.result.data(), q.result.size() * 8);
    if (info) *info = q.info;
    if (t_submit) *t_submit = q.t_submit;
    if (t_finish) *t_finish = q.t_finish;
    const hjw_status st = q.status;
    s->reqs.erase(it);
    if (st != HJW_OK) return fail(st, "request %lld produced non-finite values", (long long)id);
    return HJW_OK;
}

hjw_status hjw_server_get_stats(const hjw_server* s, hjw_server_stats* out) {
    if (!s || !out) return fail(HJW_EINVAL, "NULL argument");
    *out = s->stats;
    out->queued = int64_t(s->queue.size());
    out->active = int64_t(s->active.size());
    out->pool_in_use = s->in_use;
    out->pool_peak = s->peak;
    return HJW_OK;
}

double hjw_server_clock(const hjw_server* s) { return s ? seconds_since(s->t0) : 0.0; }

void hjw_server_destroy(hjw_server* s) {
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    drop_graphs(s);
    auto unpin = [](void* p) {
        if (p) (void)hipHostFree(p);
    };
    auto drop = [](hipEvent_t e) {
        if (e) (void)hipEventDestroy(e);
    };
    for (int b = 0; b < 2; ++b) {
        unpin(s->h_table[b]);
        unpin(s->h_tile_start[b]);
        unpin(s->h_ngrids[b]);
        unpin(s->up[b].p);
        unpin(s->down[b].p);
        drop(s->tab_ev[b]);
        drop(s->up[b].ev);
        drop(s->down[b].ev);
    }
    for (int b = 0; b < kInFlight; ++b) {
        unpin(s->h_rec[b]);
        drop(s->rec_ev[b]);
    }
    unpin(s->inbox);
    if (s->capture) (void)hipStreamDestroy(s->capture);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

}  // extern "C"
