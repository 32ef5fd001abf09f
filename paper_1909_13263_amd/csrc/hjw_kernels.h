// hjw_kernels.h - device kernels of one RK3 step (templates shared by the grid API
// and the batched server).
//
// One TVD-RK3 step (Rathan & Biswas, arXiv:1909.13263, Step 5) is three launches:
//   stage<Pre>   WENO-L derivatives of phi^n (Steps 1-4), writes Hbar = H(ubar,vbar),
//                Dx = (u+ - u-)/2, Dy = (v+ - v-)/2 and folds the workgroup's min/max
//                of u+-, v+- into range slots;
//   stage<Mid>   every workgroup reduces the slots -> alpha_x, alpha_y (eq. LF, maximum
//                of |H_p| over the box) -> dt (CFL rule); rebuilds
//                phi_1 = phi^n - dt (Hbar - ax Dx - ay Dy) on the tile and its halo,
//                derivatives of phi_1, phi_2 = 3/4 phi^n + 1/4 (phi_1 + dt L);
//   stage<Last>  derivatives of phi_2, phi^{n+1} = 1/3 phi^n + 2/3 (phi_2 + dt L),
//                written in place over phi^n.
// The step state lives on the device (two records per grid, by step parity), so whole
// steps are captured once in a HIP graph and replayed; kernels of a step past t_final
// exit at once.
#pragma once

#include <climits>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "hjw_common.h"
#include "hjw_tile.h"

namespace hjw {

// ------------------------------------------------------------------ kernels
// Wave-wide min/max with DPP lane moves (no LDS round trip per step): two quad
// permutations, then the half-row and row mirrors, leave every lane of each 16-lane row
// with that row's fold; two row broadcasts (lane 15 into rows 1 and 3, then lane 31 into
// rows 2 and 3) carry the folds of rows 0-2 into row 3, whose last lane holds the wave's
// fold; it is read out with readlane, so the result is uniform over the wave.  The moves
// leave the lanes they do not write undefined (rows outside a broadcast's mask hold
// values no later step reads), which lets the compiler fuse each move into the min/max
// that uses it.  All 64 lanes must be active.
template <int CTRL, int ROWS = 0xF>
__device__ inline int dpp_move(int x) {
    return __builtin_amdgcn_mov_dpp(x, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS = 0xF>
__device__ inline float dpp_move(float x) {
    return __int_as_float(dpp_move<CTRL, ROWS>(__float_as_int(x)));
}
template <int CTRL, int ROWS = 0xF>
__device__ inline double dpp_move(double x) {
    const int lo = dpp_move<CTRL, ROWS>(__double2loint(x));
    const int hi = dpp_move<CTRL, ROWS>(__double2hiint(x));
    return __hiloint2double(hi, lo);
}
__device__ inline float read_lane(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}
__device__ inline double read_lane(double x, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                            __builtin_amdgcn_readlane(__double2loint(x), l));
}
template <bool MAX, typename T>
__device__ inline T wave_fold(T x) {
    const auto f = [](T p, T q) { return MAX ? fmax(p, q) : fmin(p, q); };
    x = f(x, dpp_move<0xB1>(x));        // quad_perm [1,0,3,2]
    x = f(x, dpp_move<0x4E>(x));        // quad_perm [2,3,0,1]
    x = f(x, dpp_move<0x141>(x));       // row_half_mirror: lane i <- lane 7-i of its half row
    x = f(x, dpp_move<0x140>(x));       // row_mirror: lane i <- lane 15-i of its row
    x = f(x, dpp_move<0x142, 0xA>(x));  // row_bcast:15, rows 1 and 3
    x = f(x, dpp_move<0x143, 0xC>(x));  // row_bcast:31, rows 2 and 3
    return read_lane(x, 63);
}
// FP32: the fold runs on order-preserving integer keys (x >= +0 keeps its bits, x <= -0
// has its magnitude bits flipped, so -0 < +0 and the order is total), whose integer
// min/max need no NaN quieting of the moved values and take each move as an operand.
__device__ inline int float_key(float x) {
    const int b = __float_as_int(x);
    return b ^ ((b >> 31) & 0x7fffffff);
}
__device__ inline float key_float(int k) { return __int_as_float(k ^ ((k >> 31) & 0x7fffffff)); }
// A lane the move does not write keeps the fold's identity, so the compiler can fuse the
// move into the min/max.
template <bool MAX, int CTRL, int ROWS = 0xF>
__device__ inline int fold_step(int k) {
    constexpr int kIdentity = MAX ? INT_MIN : INT_MAX;
    const int m = __builtin_amdgcn_update_dpp(kIdentity, k, CTRL, ROWS, 0xF, false);
    return MAX ? max(k, m) : min(k, m);
}
template <bool MAX>
__device__ inline float wave_fold(float x) {
    int k = float_key(x);
    k = fold_step<MAX, 0xB1>(k);
    k = fold_step<MAX, 0x4E>(k);
    k = fold_step<MAX, 0x141>(k);
    k = fold_step<MAX, 0x140>(k);
    k = fold_step<MAX, 0x142, 0xA>(k);
    k = fold_step<MAX, 0x143, 0xC>(k);
    return key_float(__builtin_amdgcn_readlane(k, 63));
}
template <typename T>
__device__ inline T wave_min(T x) { return wave_fold<false>(x); }
template <typename T>
__device__ inline T wave_max(T x) { return wave_fold<true>(x); }

__device__ inline bool step_open(const DevState& s) {
    // the fields are read together, in one round trip (a short-circuit test would read them
    // one after another)
    const int bad = s.bad;
    const double t = s.t, t_final = s.t_final;
    const int64_t left = s.steps_left;
    return (bad == 0) & (t < t_final) & (left > 0);
}

__device__ inline int tile_of_block(int bid, int nb, int remap) {
    // Blocks are dealt to the 8 XCDs round-robin; give each XCD a contiguous run of
    // tiles so that tile halos are shared through that XCD's L2.
    return remap ? (bid % 8) * (nb / 8) + bid / 8 : bid;
}

// Range accumulators: the first stage of a step folds each workgroup's min/max of
// the one-sided derivatives into one of kSlots slots with integer atomics on an
// order-preserving key of the FP64 value (exact, independent of order); the second
// stage reduces the slots in every workgroup and derives the same time step.
constexpr int kSlots = 64;
struct RangeSlots {
    unsigned long long key[4][kSlots];   // min u, max u, min v, max v
    unsigned int bad[kSlots];
};

// Monotone map from doubles to unsigned 64-bit keys and back.
__device__ inline unsigned long long order_key(double x) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(x));
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ inline double key_value(unsigned long long k) {
    const unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double(static_cast<long long>(b));
}

template <int NW, typename T, typename P>
__device__ inline void fold_range(const StageArgs<T, P>& a, int bid, T lu, T hu, T lv, T hv,
                                  bool bad) {
    __shared__ double red[NW][4];
    __shared__ int red_bad[NW];
    const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
    lu = wave_min(lu);
    hu = wave_max(hu);
    lv = wave_min(lv);
    hv = wave_max(hv);
    const bool wave_bad = __any(bad);
    if (lane == 0) {
        red[w][0] = double(lu);
        red[w][1] = double(hu);
        red[w][2] = double(lv);
        red[w][3] = double(hv);
        red_bad[w] = wave_bad ? 1 : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double r0 = red[0][0], r1 = red[0][1], r2 = red[0][2], r3 = red[0][3];
        int anybad = red_bad[0];
        for (int k = 1; k < NW; ++k) {
            r0 = fmin(r0, red[k][0]);
            r1 = fmax(r1, red[k][1]);
            r2 = fmin(r2, red[k][2]);
            r3 = fmax(r3, red[k][3]);
            anybad |= red_bad[k];
        }
        RangeSlots* sl = static_cast<RangeSlots*>(a.slots);
        const int k = bid % kSlots;
        atomicMin(&sl->key[0][k], order_key(r0));
        atomicMax(&sl->key[1][k], order_key(r1));
        atomicMin(&sl->key[2][k], order_key(r2));
        atomicMax(&sl->key[3][k], order_key(r3));
        if (anybad) atomicOr(&sl->bad[k], 1u);
    }
}

// Second stage: every workgroup reduces the slots and plans the step from the step
// record st[par] (read-only during this launch); workgroup 0 publishes the result in
// st[par ^ 1].  plan_finish returns whether the step is taken; dt and the dissipation
// go to the references.
// The plan's inputs are read first (plan_issue) and used later (plan_finish), so that
// a caller can issue its own loads in between and their latencies overlap.  With the
// plan published by its own launch (plan_ready) every thread reads the record's
// outcome; otherwise the first wave reads the range slots and the record.
struct PlanIn {
    DevState s;                   // the step's record (first wave)
    unsigned long long key[4];    // one range slot per lane of the first wave
    unsigned int bad;
    int ready_active;             // the published outcome (plan_ready), kept apart from s
    double ready_dt, ready_ax, ready_ay;   // so that no value merges the two paths
};

template <typename T, typename P>
__device__ inline void plan_issue(const StageArgs<T, P>& a, PlanIn& in) {
    if (a.plan_ready) {
        const DevState& n = a.st[a.par ^ 1];
        in.ready_active = n.active;
        in.ready_dt = n.dt;
        in.ready_ax = n.alpha_x;
        in.ready_ay = n.alpha_y;
        return;
    }
    if (threadIdx.x < 64) {
        const RangeSlots* sl = static_cast<const RangeSlots*>(a.slots);
        const int k = threadIdx.x;
        // every lane reads the record (one address): no branch whose result must be
        // copied, which would wait for the loads here
        in.s = a.st[a.par];
        for (int q = 0; q < 4; ++q) in.key[q] = sl->key[q][k];
        in.bad = sl->bad[k];
    }
}

template <typename T, typename P>
__device__ inline bool plan_finish(const StageArgs<T, P>& a, int bid, const PlanIn& in,
                                   double& dt, double& ax, double& ay) {
    if (a.plan_ready) {
        dt = in.ready_dt;
        ax = in.ready_ax;
        ay = in.ready_ay;
        return in.ready_active != 0;
    }
    __shared__ DevState s_plan;
    if (threadIdx.x < 64) {
        DevState s = in.s;
        double r0 = key_value(in.key[0]), r1 = key_value(in.key[1]);
        double r2 = key_value(in.key[2]), r3 = key_value(in.key[3]);
        unsigned int b = in.bad;
        // an empty fence: the test of b below cannot be moved up to the load of b (it
        // would wait there for the loads a caller issues between plan_issue and here)
        asm volatile("" : "+v"(b));
        // an FP32 stencil's ranges are FP32 values (widened exactly): they fold as FP32
        // keys; NaNs of empty slots sort past every value, as fmin/fmax ignore them
        if (std::is_same<T, float>::value) {
            r0 = double(wave_min(float(r0)));
            r1 = double(wave_max(float(r1)));
            r2 = double(wave_min(float(r2)));
            r3 = double(wave_max(float(r3)));
        } else {
            r0 = wave_min(r0);
            r1 = wave_max(r1);
            r2 = wave_min(r2);
            r3 = wave_max(r3);
        }
        b = __any(b != 0u) ? 1u : 0u;
        if (threadIdx.x == 0) {
            if (step_open(s)) {
                const double r[4] = {r0, r1, r2, r3};
                if (b != 0u || !(finite_t(r0) && finite_t(r1) && finite_t(r2) && finite_t(r3))) {
                    s.bad = 1;
                    s.active = 0;
                } else {
                    plan_step(s, a.ham, a.hpD, a.dim, a.ihxD, a.ihyD, r);
                    s.active = s.bad ? 0 : 1;
                }
            } else {
                s.active = 0;   // nothing to do: carry the record over unchanged
            }
            s_plan = s;
            if (bid == 0) a.st[a.par ^ 1] = s;
        }
    }
    __syncthreads();
    dt = s_plan.dt;
    ax = s_plan.alpha_x;
    ay = s_plan.alpha_y;
    return s_plan.active != 0;
}

template <typename T, typename P>
__device__ inline bool plan_in_block(const StageArgs<T, P>& a, int bid, double& dt, double& ax,
                                     double& ay) {
    PlanIn in;
    plan_issue(a, in);
    return plan_finish(a, bid, in, dt, ax, ay);
}

// Third stage, workgroup 0: empty the slots for the next step's first stage.
template <typename T, typename P>
__device__ inline void clear_slots(const StageArgs<T, P>& a, int bid) {
    if (bid == 0 && threadIdx.x < kSlots) {
        RangeSlots* sl = static_cast<RangeSlots*>(a.slots);
        const int k = threadIdx.x;
        sl->key[0][k] = ~0ull;
        sl->key[1][k] = 0ull;
        sl->key[2][k] = ~0ull;
        sl->key[3][k] = 0ull;
        sl->bad[k] = 0u;
    }
}

// Entry of a stage kernel: whether this workgroup has work, and the step's dt and
// dissipation for the second and third stages.
template <int STAGE, typename T, typename P>
__device__ inline bool stage_entry(const StageArgs<T, P>& a, int bid, double& dt, double& ax,
                                   double& ay) {
    dt = ax = ay = 0.0;
    if (STAGE == kStagePre) return step_open(a.st[a.par]);
    if (STAGE == kStageMid) {
        if (!a.plan_ready) return plan_in_block(a, bid, dt, ax, ay);
        const DevState& n = a.st[a.par ^ 1];
        if (!n.active) return false;
        dt = n.dt;
        ax = n.alpha_x;
        ay = n.alpha_y;
        return true;
    }
    if (STAGE == kStageLast) {
        // the plan's outcome and values in one round trip: the empty asm keeps the loads of
        // dt and the dissipation ahead of the test of active
        const DevState& n = a.st[a.par ^ 1];
        const int active = n.active;
        double d = n.dt, x = n.alpha_x, y = n.alpha_y;
        asm volatile("" : "+v"(d), "+v"(x), "+v"(y));
        if (!active) return false;
        dt = d;
        ax = x;
        ay = y;
        clear_slots(a, bid);
        return true;
    }
    return true;
}

// One workgroup's share of a stage on a 2-D grid: bid is the workgroup's index among
// the grid's nbx * nby tiles; threads2d(TY, S) threads, half row and half column
// threads, each marching S nodes.
template <typename T, typename P, int STAGE, int TY, int S, bool TIMED>
__device__ inline void stage_tile2d(const StageArgs<T, P>& a, int bid) {
    using TL = Tile<T, P, kTX, TY, S, S>;
    static_assert(TL::kThreads == threads2d(TY, S), "launch bounds");
    constexpr bool kCenter = STAGE == kStageMid || STAGE == kStageLast;
    __shared__ P phiL[TL::kPhiElems];
    __shared__ T uL[TL::kUElems];
    __shared__ P pnL[kCenter ? TL::kCenterElems : 1];
    __shared__ T vL[TL::kVElems];
    const int nb = a.nbx * a.nby;
    const int tile = tile_of_block(bid, nb, a.remap);
    const int64_t x0 = int64_t(tile % a.nbx) * kTX;
    const int64_t y0 = int64_t(tile / a.nbx) * TY;
    // the workgroup is exactly the tile's threads: with the range known, the compiler
    // resolves at compile time which rounds of the load cover the tile's own nodes
    const int tid = threadIdx.x;
    __builtin_assume(tid >= 0 && tid < TL::kThreads);
    double dt, ax, ay;
    const bool interior = TL::inside(a, x0, y0);
    // periodic edge tiles take the same path on the FP32 stencil; on FP64 the second
    // gather's code made the stage slower (the edge tiles load after the plan instead)
    constexpr bool kEdgeEarly = sizeof(T) == 4;
    if (STAGE == kStageMid &&
        (interior || (kEdgeEarly && a.bcx == kBcPeriodic && a.bcy == kBcPeriodic))) {
        // the plan's loads, then the tile's, then the plan: the plan waits only for its
        // own loads (they were issued first) while the tile's are still in flight
        PlanIn pin;
        plan_issue(a, pin);
        typename TL::Gathered gth;
        if (!kEdgeEarly || interior)
            TL::template gather<false>(tid, a, x0, y0, gth);
        else
            TL::template gather<kEdgeEarly>(tid, a, x0, y0, gth);
        dt = ax = ay = 0.0;
        if (!plan_finish(a, bid, pin, dt, ax, ay)) return;   // uniform over the workgroup
        TL::make_phi1(tid, a, dt, ax, ay, phiL, pnL, gth);
    } else {
        // a step past its end returns before loading anything
        if (!stage_entry<STAGE>(a, bid, dt, ax, ay)) return;
        TL::template load<STAGE>(tid, a, x0, y0, dt, ax, ay, phiL, pnL);
    }
    TL::template load_corners<STAGE>(tid, a, x0, y0, dt, ax, ay, phiL);
    __syncthreads();
    T vm[S], vp[S];
    const bool rows = tid < TL::kHalf;   // wave-uniform: the first half of the waves march rows
    if (rows) {
        TL::sweep_x(tid, a, phiL, uL);
    } else {
        TL::sweep_y(tid - TL::kHalf, a, phiL, vm, vp, vL);
    }
    __syncthreads();
    Finisher<STAGE, T, P, TIMED> fin(a, x0, y0, dt, ax, ay, 2);
    TL::finish(rows ? tid : tid - TL::kHalf, !rows, uL, vm, vp, vL, phiL,
               kCenter ? pnL : nullptr, fin);

    if (STAGE == kStagePre) {
        fold_range<TL::kThreads / 64>(a, bid, fin.lo_u, fin.hi_u, fin.lo_v, fin.hi_v, fin.bad);
    } else if (STAGE == kStageLast) {
        // any wave that met a non-finite value raises the flag (the same store from each)
        if (__any(fin.bad) && tid % 64 == 0) a.st[a.par ^ 1].bad = 1;
    }
}

// TIMED: the grid's Hamiltonian may be the time- and phi-dependent family; the kernels of
// every other family are compiled without its code.
template <typename T, typename P, int STAGE, int TY, int S, bool TIMED>
__global__ __launch_bounds__(threads2d(TY, S), fp64_waves(sizeof(T), TY)) void k_stage2d(
    StageArgs<T, P> a) {
    stage_tile2d<T, P, STAGE, TY, S, TIMED>(a, int(blockIdx.x));
}

template <typename T, typename P, int STAGE, bool TIMED>
__global__ __launch_bounds__(256) void k_stage1d(StageArgs<T, P> a) {
    using TL = Tile1D<T, P, kTX1, kS1>;
    constexpr bool kCenter = STAGE == kStageMid || STAGE == kStageLast;
    __shared__ P phiL[TL::kPhiElems];
    __shared__ T uL[TL::kUElems];
    __shared__ P pnL[kCenter ? TL::kCenterElems : 1];
    double dt, ax, ay;
    if (!stage_entry<STAGE>(a, int(blockIdx.x), dt, ax, ay)) return;
    const int64_t x0 = int64_t(blockIdx.x) * kTX1;
    const int tid = threadIdx.x;
    __builtin_assume(tid >= 0 && tid < 256);
    TL::template load<STAGE>(tid, a, x0, dt, ax, 0.0, phiL, pnL);
    __syncthreads();
    TL::sweep_x(tid, a, phiL, uL);
    __syncthreads();
    Finisher<STAGE, T, P, TIMED> fin(a, x0, 0, dt, ax, 0.0, 1);
    const int mode = fin.mode();
    if (TIMED && mode == kNodeTimed) {
        for (int c = tid; c < kTX1; c += 256)
            fin.template node<TIMED ? kNodeTimed : kNodePlain>(
                c, 0, uL[c], uL[kTX1 + c], T(0), T(0), phiL[c + 3], kCenter ? pnL[c] : P(0));
    } else if (mode == kNodeExtended) {
        for (int c = tid; c < kTX1; c += 256)
            fin.template node<kNodeExtended>(c, 0, uL[c], uL[kTX1 + c], T(0), T(0),
                                             phiL[c + 3], kCenter ? pnL[c] : P(0));
    } else {
        for (int c = tid; c < kTX1; c += 256)
            fin.template node<kNodePlain>(c, 0, uL[c], uL[kTX1 + c], T(0), T(0), phiL[c + 3],
                                          kCenter ? pnL[c] : P(0));
    }
    if (STAGE == kStagePre) {
        fold_range<4>(a, int(blockIdx.x), fin.lo_u, fin.hi_u, T(0), T(0), fin.bad);
    } else if (STAGE == kStageLast) {
        // any wave that met a non-finite value raises the flag (the same store from each)
        if (__any(fin.bad) && tid % 64 == 0) a.st[a.par ^ 1].bad = 1;
    }
}

// The step plan as a launch of its own (one wave): on large grids, planning once
// costs less than planning in every workgroup of the second stage.
template <typename T, typename P>
__global__ __launch_bounds__(64) void k_plan(StageArgs<T, P> a) {
    double dt, ax, ay;
    a.plan_ready = 0;   // the second stage's arguments say the plan is published: by this
    (void)plan_in_block(a, 0, dt, ax, ay);
}

// Keeps one wave busy for about `ticks` of the constant-rate wall clock (at most 2^22
// short sleeps), so that the launches the host enqueues meanwhile then run back to back.
static __global__ void k_hold(int64_t ticks) {
    const long long t0 = wall_clock64();
    for (int k = 0; k < (1 << 22); ++k) {
        if (wall_clock64() - t0 >= ticks) break;
        __builtin_amdgcn_s_sleep(8);
    }
}

static __global__ void k_set_target(DevState* st, double t_final, double cfl, int64_t steps_left) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->t_final = t_final;
        st->cfl = cfl;
        st->steps_left = steps_left;
        st->active = 0;
    }
}

// Both step records to t = 0 and empty range slots.
static __global__ void k_reset(DevState* st, RangeSlots* sl) {
    if (blockIdx.x == 0 && threadIdx.x < 2) {
        DevState s;
        s.t = 0.0;
        s.t_final = 0.0;
        s.cfl = 0.0;
        s.dt = 0.0;
        s.alpha_x = 0.0;
        s.alpha_y = 0.0;
        for (int k = 0; k < 4; ++k) s.range[k] = 0.0;
        s.steps = 0;
        s.steps_left = 0;
        s.active = 0;
        s.bad = 0;
        s.pad[0] = s.pad[1] = 0;
        st[threadIdx.x] = s;
    }
    if (blockIdx.x == 0 && threadIdx.x < kSlots) {
        const int k = threadIdx.x;
        sl->key[0][k] = ~0ull;
        sl->key[1][k] = 0ull;
        sl->key[2][k] = ~0ull;
        sl->key[3][k] = 0ull;
        sl->bad[k] = 0u;
    }
}

static __global__ void k_d2f(const double* in, float* out, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        out[i] = float(in[i]);
}

static __global__ void k_f2d(const float* in, double* out, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        out[i] = double(in[i]);
}

static __global__ void k_check_finite(const double* in, int64_t n, DevState* st) {
    int bad = 0;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        if (!finite_t(in[i])) bad = 1;
    if (__syncthreads_or(bad) && threadIdx.x == 0) st->bad = 1;
}

}  // namespace hjw
