// hjw_emulate.hip - CPU execution of the GPU tile phases (test support).
//
// Runs Tile::load / sweep_x / sweep_y and the node finisher of hjw_tile.h for
// every workgroup and thread index, phase by phase, on host memory.  The LDS
// arrays are re-filled with NaN for every workgroup and every global array
// sits between NaN guard zones, so a read of anything the tile did not stage
// surfaces as a NaN in the results; index ranges are also checked explicitly.
// Used only by the CPU tests to check the kernels' indexing and arithmetic
// before they run on a GPU.  Built as its own library, never linked into libhjw.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

#include "hjw_tile.h"

using namespace hjw;

namespace {

int g_tile_rows = 32;  // 2-D tile height being emulated (32 or 16)
int g_segment = 8;     // nodes per thread in the 2-D sweeps (8, or 4 with 16-row tiles)
int g_scheme = 0;      // kSchemeL or kSchemeJP
int g_llf = 0;         // the local dissipation (HJW_OPT_DISSIPATION = 1)
double g_origin[2] = {0.0, 0.0};   // coordinates of node (0, 0)
constexpr size_t kGuard = 4096;

template <typename X>
struct Guarded {
    std::vector<X> buf;
    size_t n;
    explicit Guarded(size_t n_) : buf(n_ + 2 * kGuard, X(NAN)), n(n_) {}
    X* data() { return buf.data() + kGuard; }
    bool guards_intact() const {
        for (size_t k = 0; k < kGuard; ++k)
            if (!std::isnan(double(buf[k])) || !std::isnan(double(buf[kGuard + n + k])))
                return false;
        return true;
    }
};

struct Problem {
    int dim;
    int64_t nx, ny;
    double dx, dy;
    int bcx, bcy;
    int ham;
    double hp[4];
};

template <typename T, typename P>
struct Emu {
    const Problem& pr;
    size_t n;
    Guarded<P> phi, phi2;
    Guarded<T> flux;
    Guarded<double> partials;
    Guarded<double> d0, d1, d2, d3;
    DevState st[2]{};   // the step's record and the planned one, as on the GPU
    int nbx, nby;
    bool overrun = false;

    explicit Emu(const Problem& p)
        : pr(p), n(size_t(p.nx * p.ny)), phi(n), phi2(n), flux(3 * n),
          partials(size_t(tiles(p)) * kPartialStride), d0(n), d1(n), d2(n), d3(n) {
        nbx = p.dim == 2 ? int((p.nx + kTX - 1) / kTX) : int((p.nx + kTX1 - 1) / kTX1);
        nby = p.dim == 2 ? int((p.ny + g_tile_rows - 1) / g_tile_rows) : 1;
    }
    static int64_t tiles(const Problem& p) {
        return p.dim == 2 ? ((p.nx + kTX - 1) / kTX) * ((p.ny + 15) / 16)
                          : (p.nx + kTX1 - 1) / kTX1;
    }

    StageArgs<T, P> args() {
        StageArgs<T, P> a{};
        a.phi_n = phi.data();
        a.phi_s = phi2.data();
        a.flux = flux.data();
        a.dout0 = d0.data();
        a.dout1 = d1.data();
        a.dout2 = d2.data();
        a.dout3 = d3.data();
        a.st = st;
        a.par = 0;
        a.slots = nullptr;
        a.nx = pr.nx;
        a.ny = pr.ny;
        a.bcx = pr.bcx;
        a.bcy = pr.bcy;
        a.ihx = P(1.0 / pr.dx);
        a.ihy = P(1.0 / pr.dy);
        a.ihxT = T(1.0 / pr.dx);
        a.ihyT = T(1.0 / pr.dy);
        a.epsx = T(weight_eps(g_scheme, pr.dx));
        a.epsy = T(weight_eps(g_scheme, pr.dy));
        a.scheme = g_scheme;
        a.llf = g_llf;
        a.x0 = g_origin[0];
        a.y0 = g_origin[1];
        a.dxD = pr.dx;
        a.dyD = pr.dy;
        a.ham = pr.ham;
        for (int k = 0; k < 4; ++k) {
            a.hpT[k] = T(pr.hp[k]);
            a.hpD[k] = pr.hp[k];
        }
        a.nbx = nbx;
        a.nby = nby;
        a.remap = 0;
        a.dim = pr.dim;
        return a;
    }

    // Run one stage over all tiles, the way the kernel does.
    template <int STAGE>
    void stage(StageArgs<T, P> a, double dt, double ax, double ay) {
        if (pr.dim == 2 && g_tile_rows == 16 && g_segment == 4)
            stage2d<STAGE, 16, 4>(a, dt, ax, ay);
        else if (pr.dim == 2 && g_tile_rows == 16)
            stage2d<STAGE, 16, 8>(a, dt, ax, ay);
        else if (pr.dim == 2)
            stage2d<STAGE, 32, 8>(a, dt, ax, ay);
        else
            stage1d<STAGE>(a, dt, ax, ay);
    }

    template <int STAGE, int TY, int S>
    void stage2d(StageArgs<T, P> a, double dt, double ax, double ay) {
        using TL = Tile<T, P, kTX, TY, S, S>;
        const int nb = nbx * nby;
        std::vector<P> phiL(TL::kPhiElems), pnL(TL::kCenterElems);
        std::vector<T> uL(TL::kUElems);
        constexpr bool kCenter = STAGE == kStageMid || STAGE == kStageLast;
        for (int b = 0; b < nb; ++b) {
            const int64_t x0 = int64_t(b % nbx) * kTX, y0 = int64_t(b / nbx) * TY;
            std::fill(phiL.begin(), phiL.end(), P(NAN));
            std::fill(pnL.begin(), pnL.end(), P(NAN));
            std::fill(uL.begin(), uL.end(), T(NAN));
            const bool interior = TL::inside(a, x0, y0);
            if (STAGE == kStageMid &&
                (interior ||
                 (sizeof(T) == 4 && a.bcx == kBcPeriodic && a.bcy == kBcPeriodic))) {
                // the kernel's split second stage: gather, plan, then phi_1 in place
                std::vector<typename TL::Gathered> gth(TL::kThreads);
                for (int t = 0; t < TL::kThreads; ++t) {
                    if (interior)
                        TL::template gather<false>(t, a, x0, y0, gth[t]);
                    else
                        TL::template gather<true>(t, a, x0, y0, gth[t]);
                }
                for (int t = 0; t < TL::kThreads; ++t)
                    TL::make_phi1(t, a, dt, ax, ay, phiL.data(), pnL.data(), gth[t]);
            } else {
                for (int t = 0; t < TL::kThreads; ++t)
                    TL::template load<STAGE>(t, a, x0, y0, dt, ax, ay, phiL.data(), pnL.data());
            }
            for (int t = 0; t < TL::kThreads; ++t)
                TL::template load_corners<STAGE>(t, a, x0, y0, dt, ax, ay, phiL.data());
            // the row threads and the column threads, then the barrier, then the finish
            std::vector<T> vm(size_t(TL::kHalf) * S), vp(size_t(TL::kHalf) * S);
            std::vector<T> vL(TL::kVElems, T(NAN));
            for (int t = 0; t < TL::kHalf; ++t) TL::sweep_x(t, a, phiL.data(), uL.data());
            for (int t = 0; t < TL::kHalf; ++t)
                TL::sweep_y(t, a, phiL.data(), &vm[size_t(t) * S], &vp[size_t(t) * S], vL.data());
            double lu = INFINITY, hu = -INFINITY, lv = INFINITY, hv = -INFINITY;
            bool bad = false;
            for (int t = 0; t < TL::kThreads; ++t) {
                // row threads (t < kHalf) finish from the stash, column threads from registers
                const bool col_half = t >= TL::kHalf;
                const int u = col_half ? t - TL::kHalf : t;
                Finisher<STAGE, T, P, true> fin(a, x0, y0, dt, ax, ay, 2);
                TL::finish(u, col_half, uL.data(), &vm[size_t(u) * S], &vp[size_t(u) * S],
                           vL.data(), phiL.data(), kCenter ? pnL.data() : nullptr, fin);
                lu = std::fmin(lu, double(fin.lo_u));
                hu = std::fmax(hu, double(fin.hi_u));
                lv = std::fmin(lv, double(fin.lo_v));
                hv = std::fmax(hv, double(fin.hi_v));
                bad = bad || fin.bad;
            }
            write_partial(b, lu, hu, lv, hv, bad);
        }
    }

    template <int STAGE>
    void stage1d(StageArgs<T, P> a, double dt, double ax, double ay) {
        using TL = Tile1D<T, P, kTX1, kS1>;
        const int nb = nbx * nby;
        std::vector<P> phiL(TL::kPhiElems), pnL(TL::kCenterElems);
        std::vector<T> uL(TL::kUElems);
        for (int b = 0; b < nb; ++b) {
            const int64_t x0 = int64_t(b) * kTX1;
            std::fill(phiL.begin(), phiL.end(), P(NAN));
            std::fill(pnL.begin(), pnL.end(), P(NAN));
            std::fill(uL.begin(), uL.end(), T(NAN));
            for (int t = 0; t < TL::kThreads; ++t)
                TL::template load<STAGE>(t, a, x0, dt, ax, 0.0, phiL.data(), pnL.data());
            for (int t = 0; t < TL::kThreads; ++t) TL::sweep_x(t, a, phiL.data(), uL.data());
            Finisher<STAGE, T, P, true> fin(a, x0, 0, dt, ax, 0.0, 1);
            for (int c = 0; c < kTX1; ++c)
                fin(c, 0, uL[c], uL[kTX1 + c], T(0), T(0), phiL[c + 3], pnL[c]);
            write_partial(b, double(fin.lo_u), double(fin.hi_u), 0.0, 0.0, fin.bad);
        }
    }

    void write_partial(int b, double lu, double hu, double lv, double hv, bool bad) {
        double* p = partials.data() + size_t(b) * kPartialStride;
        p[0] = lu;
        p[1] = hu;
        p[2] = lv;
        p[3] = hv;
        p[4] = bad ? 1.0 : 0.0;
    }

    bool guards() const {
        return phi.guards_intact() && phi2.guards_intact() && flux.guards_intact() &&
               partials.guards_intact() && d0.guards_intact() && d1.guards_intact() &&
               d2.guards_intact() && d3.guards_intact();
    }
};

Problem make_problem(int dim, int64_t nx, int64_t ny, double dx, double dy, int bcx, int bcy,
                     int ham, const double* hp) {
    Problem p{};
    p.dim = dim;
    p.nx = nx;
    p.ny = dim == 2 ? ny : 1;
    p.dx = dx;
    p.dy = dim == 2 ? dy : 1.0;
    p.bcx = bcx;
    p.bcy = dim == 2 ? bcy : kBcPeriodic;
    p.ham = ham;
    for (int k = 0; k < 4; ++k) p.hp[k] = hp ? hp[k] : 0.0;
    return p;
}

template <typename T, typename P>
int derivs(const Problem& pr, const double* phi, double* um, double* up, double* vm,
           double* vp) {
    Emu<T, P> e(pr);
    for (size_t k = 0; k < e.n; ++k) e.phi.data()[k] = P(phi[k]);
    e.template stage<kStageDeriv>(e.args(), 0.0, 0.0, 0.0);
    for (size_t k = 0; k < e.n; ++k) {
        um[k] = e.d0.data()[k];
        up[k] = e.d1.data()[k];
        if (pr.dim == 2) {
            vm[k] = e.d2.data()[k];
            vp[k] = e.d3.data()[k];
        }
    }
    return e.guards() ? 0 : -7;
}

// One RK3 step; info = {t, dt, alpha_x, alpha_y, range[4], bad}.
template <typename T, typename P>
int step(const Problem& pr, double* phi, double t, double t_final, double cfl, double* info) {
    Emu<T, P> e(pr);
    for (size_t k = 0; k < e.n; ++k) e.phi.data()[k] = P(phi[k]);
    e.st[0].t = t;
    e.st[0].t_final = t_final;
    e.st[0].cfl = cfl;
    e.st[0].steps_left = 1;
    e.st[1] = e.st[0];
    StageArgs<T, P> a = e.args();
    e.template stage<kStagePre>(a, 0.0, 0.0, 0.0);
    // the finalize kernel, serially
    double r[4] = {INFINITY, -INFINITY, INFINITY, -INFINITY};
    bool bad = false;
    const int nb = e.nbx * e.nby;
    for (int b = 0; b < nb; ++b) {
        const double* p = e.partials.data() + size_t(b) * kPartialStride;
        r[0] = std::fmin(r[0], p[0]);
        r[1] = std::fmax(r[1], p[1]);
        r[2] = std::fmin(r[2], p[2]);
        r[3] = std::fmax(r[3], p[3]);
        bad = bad || p[4] != 0.0;
    }
    DevState& ns = e.st[1];   // st[0] keeps t_n for the stages
    if (!bad) plan_step(ns, pr.ham, pr.hp, pr.dim, 1.0 / pr.dx, 1.0 / pr.dy, r);
    if (bad || ns.bad) {
        info[8] = 1.0;
        return -5;
    }
    a.out = e.phi2.data();
    e.template stage<kStageMid>(a, ns.dt, ns.alpha_x, ns.alpha_y);
    a.out = e.phi.data();
    e.template stage<kStageLast>(a, ns.dt, ns.alpha_x, ns.alpha_y);
    for (size_t k = 0; k < e.n; ++k) phi[k] = double(e.phi.data()[k]);
    info[0] = ns.t;
    info[1] = ns.dt;
    info[2] = ns.alpha_x;
    info[3] = ns.alpha_y;
    for (int k = 0; k < 4; ++k) info[4 + k] = ns.range[k];
    info[8] = 0.0;
    return e.guards() ? 0 : -7;
}

}  // namespace

extern "C" {

// Height of the emulated 2-D tile (32 or 16), as HJW_OPT_TILE_ROWS selects on the GPU.
int hjw_emu_set_tile_rows(int rows) {
    if (rows != 16 && rows != 32) return -1;
    if (rows == 32 && g_segment != 8) return -1;
    g_tile_rows = rows;
    return 0;
}

// Coordinates of node (0, 0) for the position-dependent Hamiltonian.
void hjw_emu_set_origin(double x0, double y0) {
    g_origin[0] = x0;
    g_origin[1] = y0;
}

// Dissipation of the emulated kernels: 0 the step's global alpha, 1 per node (local LF).
int hjw_emu_set_dissipation(int local) {
    if (local != 0 && local != 1) return -1;
    g_llf = local;
    return 0;
}

// Scheme of the emulated kernels: 0 WENO-L, 1 WENO-JP.
int hjw_emu_set_scheme(int scheme) {
    if (scheme != kSchemeL && scheme != kSchemeJP) return -1;
    g_scheme = scheme;
    return 0;
}

// Nodes per thread in the emulated 2-D sweeps (8, or 4 with 16-row tiles), as
// HJW_OPT_SEGMENT selects on the GPU.
int hjw_emu_set_segment(int seg) {
    if (seg != 4 && seg != 8) return -1;
    if (seg == 4 && g_tile_rows != 16) return -1;
    g_segment = seg;
    return 0;
}

// prec: 0 FP64, 1 FP32 stencil with FP64 phi, 2 FP32 phi.  Returns 0, or -7 if
// a guard zone was written.
int hjw_emu_derivatives(int dim, int64_t nx, int64_t ny, double dx, double dy, int bcx, int bcy,
                        int prec, const double* phi, double* um, double* up, double* vm,
                        double* vp) {
    const Problem pr = make_problem(dim, nx, ny, dx, dy, bcx, bcy, 0, nullptr);
    if (prec == 0) return derivs<double, double>(pr, phi, um, up, vm, vp);
    if (prec == 1) return derivs<float, double>(pr, phi, um, up, vm, vp);
    return derivs<float, float>(pr, phi, um, up, vm, vp);
}

int hjw_emu_step(int dim, int64_t nx, int64_t ny, double dx, double dy, int bcx, int bcy,
                 int prec, int ham, const double* hp, double* phi, double t, double t_final,
                 double cfl, double* info) {
    const Problem pr = make_problem(dim, nx, ny, dx, dy, bcx, bcy, ham, hp);
    if (prec == 0) return step<double, double>(pr, phi, t, t_final, cfl, info);
    if (prec == 1) return step<float, double>(pr, phi, t, t_final, cfl, info);
    return step<float, float>(pr, phi, t, t_final, cfl, info);
}

}  // extern "C"
