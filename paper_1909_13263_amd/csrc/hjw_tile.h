// hjw_tile.h - the fused WENO-L stage, written as host+device tile phases.
//
// One workgroup owns a TX x TY tile of output nodes.  Phase 0 stages the stage
// input phi_s over the tile plus a three-node plus-shaped halo into LDS; phase X
// marches each row segment and leaves phi_x^-, phi_x^+ in LDS; phase Y marches
// each column segment, forms phi_y^-, phi_y^+ and finishes the node (flux,
// Runge-Kutta combination or stage-1 outputs).  The phases are plain functions of
// the thread index so that the same code also runs in a CPU emulation with
// bounds-checked buffers.
//
// The scheme (Rathan & Biswas, arXiv:1909.13263, Section 2):
//   Step 2   three third-order candidates per side from Delta^+ phi;
//   Step 4   beta_k = (arc length over the cell of the derivative of the
//            sub-stencil reconstruction)^2, eqs. (newbeta), (length);
//            omega_k = alpha_k / sum alpha, alpha_k = d_k/(eps+beta_k)^2, eq. (WLOC1);
//   eq. (LF) Lax-Friedrichs flux; Step 5 TVD-RK3.
//
// Reformulation used here (identical in exact arithmetic):
//   p_i^k' is linear on the cell; its end values are second derivatives of the
//   cubic through the sub-stencil: C_j (central), B_j (one-sided backward) and
//   F_j (one-sided forward), in terms of v_j = Delta^+ phi_j:
//     C_j = (v_j - v_{j-1})/h,  B_j = (v_{j-3} - 3 v_{j-2} + 2 v_{j-1})/h,
//     F_j = (-2 v_j + 3 v_{j+1} - v_{j+2})/h.
//   For the cell [x_{i-1}, x_i] the three pairs are (C_{i-1}, B_i), (C_{i-1}, C_i),
//   (F_{i-1}, C_i) for k = 0, 1, 2 of phi_{x,i}^-; by the mirror symmetry the same
//   three cell lengths serve phi_{x,i-1}^+ with their weights reversed.  So each
//   cell's three lengths are computed once and used twice.
//   L = h * M(a, b), M = mean of sqrt(1+s^2) for s between the end values; M is
//   evaluated from a Taylor series about the midpoint when the pair is close
//   (relative half-gap below TAU) and from the antiderivative otherwise.
//   With t_k = (eps/h^2 + M_k^2)^2 the weights become products of the other two
//   t's (one division per side); in FP32 the t's are first scaled by 1/max t.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace hjw {

constexpr int kBcPeriodic = 0;
constexpr int kBcExtrap = 1;
constexpr int kHLinear = 0;
constexpr int kHBurgers = 1;
constexpr int kHNegcos = 2;
constexpr int kHNorm = 3;

// Stage kinds of one Runge-Kutta step.
constexpr int kStagePre = 0;    // derivatives of phi^n -> Hbar, Dx, Dy, block ranges
constexpr int kStageMid = 1;    // phi_1 rebuilt on the fly -> phi_2
constexpr int kStageLast = 2;   // phi_2 -> phi^{n+1}, in place over phi^n
constexpr int kStageDeriv = 3;  // derivatives only (u-, u+, v-, v+ as FP64)

constexpr double kEps = 1.0e-6;  // epsilon of eq. (WLOC1)

// Step state kept on the device so that whole steps can be replayed from a graph.
struct DevState {
    double t;
    double t_final;
    double cfl;
    double dt;
    double alpha_x;
    double alpha_y;
    double range[4];
    int64_t steps;
    int64_t steps_left;
    int32_t active;    // the current step is being taken
    int32_t bad;       // a non-finite value was seen
    int32_t pad[2];
};

// Block partials written by the pre-stage: min/max of u+-, v+- and a bad flag.
constexpr int kPartialStride = 5;

// ---------------------------------------------------------------- math helpers
// Host and device overloads of the few primitives whose fast device form is a
// builtin; everything else is ordinary C++ arithmetic.
__device__ inline float rsqrt_t(float x) { return __builtin_amdgcn_rsqf(x); }
__host__ inline float rsqrt_t(float x) { return 1.0f / std::sqrt(x); }
__device__ inline double rsqrt_t(double x) { return rsqrt(x); }
__host__ inline double rsqrt_t(double x) { return 1.0 / std::sqrt(x); }
__device__ inline float rcp_t(float x) { return __builtin_amdgcn_rcpf(x); }
__host__ inline float rcp_t(float x) { return 1.0f / x; }
__host__ __device__ inline double rcp_t(double x) { return 1.0 / x; }
__device__ inline float asinh_t(float x) { return asinhf(x); }
__host__ inline float asinh_t(float x) { return std::asinh(x); }
__device__ inline double asinh_t(double x) { return asinh(x); }
__host__ inline double asinh_t(double x) { return std::asinh(x); }
__device__ inline float sqrt_t(float x) { return sqrtf(x); }
__host__ inline float sqrt_t(float x) { return std::sqrt(x); }
__device__ inline double sqrt_t(double x) { return sqrt(x); }
__host__ inline double sqrt_t(double x) { return std::sqrt(x); }
__device__ inline float cos_t(float x) { return cosf(x); }
__host__ inline float cos_t(float x) { return std::cos(x); }
__device__ inline double cos_t(double x) { return cos(x); }
__host__ inline double cos_t(double x) { return std::cos(x); }
__device__ inline bool any_lane(bool p) { return __any(p ? 1 : 0) != 0; }
__host__ inline bool any_lane(bool p) { return p; }
// Products that are rounded on their own (never fused into an add), so that sums
// like a*u + b*v are symmetric under exchanging (a,u) and (b,v) bit for bit.
__device__ inline float mul_rn(float a, float b) { return __fmul_rn(a, b); }
__host__ inline float mul_rn(float a, float b) { return a * b; }
__device__ inline double mul_rn(double a, double b) { return __dmul_rn(a, b); }
__host__ inline double mul_rn(double a, double b) { return a * b; }

template <typename T>
__host__ __device__ inline bool finite_t(T x) {
    return x - x == T(0);  // false for inf and NaN
}

// Relative half-gap below which M comes from the midpoint series, and the
// series length: the truncation error stays below one unit in the last place
// (4 terms to 2e-2 in FP64, 3 terms to 1e-1 in FP32).
template <typename T> struct SeriesCfg;
template <> struct SeriesCfg<double> { static constexpr double tau2 = 4.0e-4; };
template <> struct SeriesCfg<float> { static constexpr float tau2 = 1.0e-2f; };

// Mean of sqrt(1+s^2) over [m-h, m+h] from the midpoint expansion
//   M = S (1 + y/6 + y^2 (12 m^2 - 3)/120 + y^3 45 (8 m^4 - 12 m^2 + 1)/5040),
//   S = sqrt(1+m^2), y = (h/(1+m^2))^2.
__host__ __device__ inline double mean_series(double m, double h) {
    const double q = 1.0 + m * m;
    const double r = rsqrt_t(q);
    const double S = q * r;
    const double g = h * r * r;
    const double y = g * g;
    const double m2 = m * m;
    const double c2 = (12.0 * m2 - 3.0) * (1.0 / 120.0);
    const double c3 = (45.0 / 5040.0) * ((8.0 * m2 - 12.0) * m2 + 1.0);
    return S + S * y * ((1.0 / 6.0) + y * (c2 + y * c3));
}
__host__ __device__ inline float mean_series(float m, float h) {
    const float q = 1.0f + m * m;
    const float r = rsqrt_t(q);
    const float S = q * r;
    const float g = h * r * r;
    const float y = g * g;
    const float c2 = (12.0f * m * m - 3.0f) * (1.0f / 120.0f);
    return S + S * y * ((1.0f / 6.0f) + y * c2);
}

// Antiderivative of sqrt(1+s^2).
template <typename T>
__host__ __device__ inline T prim(T s) {
    return T(0.5) * (s * sqrt_t(T(1) + s * s) + asinh_t(s));
}

// Means for the three pairs of one cell: (c0, b1), (c0, c1), (f0, c1).
template <typename T>
__host__ __device__ inline void cell_means(T c0, T b1, T c1, T f0, T& MA, T& MB, T& MC) {
    const T tau2 = SeriesCfg<T>::tau2;
    const T hA = T(0.5) * (b1 - c0), mA = T(0.5) * (b1 + c0);
    const T hB = T(0.5) * (c1 - c0), mB = T(0.5) * (c1 + c0);
    const T hC = T(0.5) * (c1 - f0), mC = T(0.5) * (c1 + f0);
    const bool wideA = hA * hA >= tau2 * (T(1) + mA * mA);
    const bool wideB = hB * hB >= tau2 * (T(1) + mB * mB);
    const bool wideC = hC * hC >= tau2 * (T(1) + mC * mC);
    MA = mean_series(mA, hA);
    MB = mean_series(mB, hB);
    MC = mean_series(mC, hC);
    if (any_lane(wideA || wideB || wideC)) {
        const T Pc0 = prim(c0), Pb1 = prim(b1), Pc1 = prim(c1), Pf0 = prim(f0);
        if (wideA) MA = (Pb1 - Pc0) / (b1 - c0);
        if (wideB) MB = (Pc1 - Pc0) / (c1 - c0);
        if (wideC) MC = (Pc1 - Pf0) / (c1 - f0);
    }
}

// Products of the weight denominators (see the file comment).
__host__ __device__ inline void weight_products(double MA, double MB, double MC, double epsp,
                                                double& pAB, double& pAC, double& pBC) {
    double tA = epsp + MA * MA, tB = epsp + MB * MB, tC = epsp + MC * MC;
    tA *= tA;
    tB *= tB;
    tC *= tC;
    pAB = tA * tB;
    pAC = tA * tC;
    pBC = tB * tC;
}
__host__ __device__ inline void weight_products(float MA, float MB, float MC, float epsp,
                                                float& pAB, float& pAC, float& pBC) {
    float tA = epsp + MA * MA, tB = epsp + MB * MB, tC = epsp + MC * MC;
    const float s = rcp_t(fmaxf(tA, fmaxf(tB, tC)));
    tA *= s;
    tB *= s;
    tC *= s;
    tA *= tA;
    tB *= tB;
    tC *= tC;
    pAB = tA * tB;
    pAC = tA * tC;
    pBC = tB * tC;
}

template <typename T>
__host__ __device__ inline T wdiv(T num, T den) {
    return num / den;
}
template <>
__host__ __device__ inline float wdiv<float>(float num, float den) {
    return num * rcp_t(den);
}

// March along one line.  line[k*stride] is phi_s at position p0-3+k,
// k = 0..S+5; writes phi^-(p0+k) to um[k] and phi^+(p0+k) to up[k], k < S.
// Differences are formed in the storage precision P and then cast to T.
template <typename T, typename P, int S>
__host__ __device__ inline void sweep(const P* line, int stride, P ihP, T ih, T epsp, T* um,
                                      T* up) {
    T v[S + 5];
#pragma unroll
    for (int k = 0; k < S + 5; ++k)
        v[k] = T((line[(k + 1) * stride] - line[k * stride]) * ihP);
    constexpr T c13 = T(1.0 / 3.0), c76 = T(7.0 / 6.0), c116 = T(11.0 / 6.0);
    constexpr T c16 = T(1.0 / 6.0), c56 = T(5.0 / 6.0);
#pragma unroll
    for (int it = 0; it <= S; ++it) {
        // the cell [x_{i-1}, x_i], i = p0 + it, sees v_{i-3..i+1}
        const T a = v[it], b = v[it + 1], c = v[it + 2], d = v[it + 3], e = v[it + 4];
        const T c0 = (c - b) * ih;                       // C_{i-1}
        const T c1 = (d - c) * ih;                       // C_i
        const T b1 = (a - T(3) * b + T(2) * c) * ih;     // B_i
        const T f0 = (T(3) * d - T(2) * c - e) * ih;     // F_{i-1}
        T MA, MB, MC;
        cell_means(c0, b1, c1, f0, MA, MB, MC);
        T pAB, pAC, pBC;
        weight_products(MA, MB, MC, epsp, pAB, pAC, pBC);
        if (it < S) {  // phi^- at node i: weights (1/10, 6/10, 3/10) on (A, B, C)
            const T q0 = c13 * a - c76 * b + c116 * c;
            const T q1 = -c16 * b + c56 * c + c13 * d;
            const T q2 = c13 * c + c56 * d - c16 * e;
            const T w0 = T(0.1) * pBC, w1 = T(0.6) * pAC, w2 = T(0.3) * pAB;
            um[it] = wdiv(w0 * q0 + w1 * q1 + w2 * q2, w0 + w1 + w2);
        }
        if (it > 0) {  // phi^+ at node i-1: the mirrored sub-stencils, (1/10, 6/10, 3/10) on (C, B, A)
            const T q0 = c13 * e - c76 * d + c116 * c;
            const T q1 = -c16 * d + c56 * c + c13 * b;
            const T q2 = c13 * c + c56 * b - c16 * a;
            const T w0 = T(0.1) * pAB, w1 = T(0.6) * pAC, w2 = T(0.3) * pBC;
            up[it - 1] = wdiv(w0 * q0 + w1 * q1 + w2 * q2, w0 + w1 + w2);
        }
    }
}

// ---------------------------------------------------------------- Hamiltonians
template <typename T>
__host__ __device__ inline T hamiltonian(int kind, const T* p, T u, T v) {
    switch (kind) {
    case kHLinear:
        return mul_rn(p[0], u) + mul_rn(p[1], v);
    case kHBurgers: {
        const T s = (mul_rn(p[0], u) + mul_rn(p[1], v)) + p[2];
        return T(0.5) * s * s;
    }
    case kHNegcos:
        return -cos_t((mul_rn(p[0], u) + mul_rn(p[1], v)) + p[2]);
    default:
        return p[0] * sqrt_t((mul_rn(u, u) + mul_rn(v, v)) + p[1]);
    }
}

// max of |sin s| on [lo, hi]: 1 when a zero of cos lies inside.
__host__ __device__ inline double max_abs_sin(double lo, double hi) {
    const double pi = 3.141592653589793238462643383279502884;
    if (hi - lo >= pi) return 1.0;
    const double k = floor((hi - 0.5 * pi) / pi);  // last pi/2 + k pi at or below hi
    if (0.5 * pi + k * pi >= lo) return 1.0;
    return fmax(fabs(sin(lo)), fabs(sin(hi)));
}

// alpha_x = max |dH/du|, alpha_y = max |dH/dv| over the box [A,B] x [C,D].
__host__ __device__ inline void dissipation(int kind, const double* p, int dim, double A,
                                            double B, double C, double D, double& ax,
                                            double& ay) {
    if (dim == 1) {
        C = 0.0;
        D = 0.0;
    }
    if (kind == kHLinear) {
        ax = fabs(p[0]);
        ay = fabs(p[1]);
    } else if (kind == kHBurgers || kind == kHNegcos) {
        // s = p0 u + p1 v + p2 takes its extremes on the box at corners
        const double s0 = mul_rn(p[0], A) + mul_rn(p[1], C);
        const double s1 = mul_rn(p[0], A) + mul_rn(p[1], D);
        const double s2 = mul_rn(p[0], B) + mul_rn(p[1], C);
        const double s3 = mul_rn(p[0], B) + mul_rn(p[1], D);
        const double lo = fmin(fmin(s0, s1), fmin(s2, s3)) + p[2];
        const double hi = fmax(fmax(s0, s1), fmax(s2, s3)) + p[2];
        const double m = (kind == kHBurgers) ? fmax(fabs(lo), fabs(hi)) : max_abs_sin(lo, hi);
        ax = fabs(p[0]) * m;
        ay = fabs(p[1]) * m;
    } else {
        // |dH/du| = |p0| |u| / sqrt(u^2+v^2+p1): largest at max |u| and min |v|
        const double umax = fmax(fabs(A), fabs(B)), vmax = fmax(fabs(C), fabs(D));
        const double umin = (A <= 0.0 && 0.0 <= B) ? 0.0 : fmin(fabs(A), fabs(B));
        const double vmin = (C <= 0.0 && 0.0 <= D) ? 0.0 : fmin(fabs(C), fabs(D));
        const double qx = (mul_rn(umax, umax) + mul_rn(vmin, vmin)) + p[1];
        const double qy = (mul_rn(vmax, vmax) + mul_rn(umin, umin)) + p[1];
        ax = fabs(p[0]) * (qx > 0.0 ? umax / sqrt(qx) : 1.0);
        ay = dim == 2 ? fabs(p[0]) * (qy > 0.0 ? vmax / sqrt(qy) : 1.0) : 0.0;
    }
}

// Advance the step state once the ranges of phi^n's derivatives are known:
// dt = cfl / (ax/dx + ay/dy), landing exactly on t_final.
__host__ __device__ inline void plan_step(DevState& s, int kind, const double* p, int dim,
                                          double ihx, double ihy, const double range[4]) {
    double ax, ay;
    dissipation(kind, p, dim, range[0], range[1], range[2], range[3], ax, ay);
    const double rate = mul_rn(ax, ihx) + (dim == 2 ? mul_rn(ay, ihy) : 0.0);
    const double remaining = s.t_final - s.t;
    double dt = rate > 0.0 ? s.cfl / rate : remaining;
    double tn = s.t + dt;
    if (!(dt < remaining)) {
        dt = remaining;
        tn = s.t_final;
    }
    s.alpha_x = ax;
    s.alpha_y = ay;
    for (int k = 0; k < 4; ++k) s.range[k] = range[k];
    s.dt = dt;
    s.t = tn;
    s.steps += 1;
    s.steps_left -= 1;
    if (!(finite_t(dt) && finite_t(ax) && finite_t(ay))) s.bad = 1;
}

// ---------------------------------------------------------------- stage arguments
template <typename T, typename P>
struct StageArgs {
    const P* phi_n;   // phi^n
    const P* phi_s;   // stage input of the last stage (phi_2)
    P* out;           // stage output (phi_2, or phi^{n+1} over phi^n)
    T* hbar;          // pre-stage outputs: H(ubar, vbar), (u+ - u-)/2, (v+ - v-)/2
    T* dxa;
    T* dya;
    double* dout0;    // derivative outputs (kStageDeriv)
    double* dout1;
    double* dout2;
    double* dout3;
    double* partials;
    DevState* st;
    int64_t nx, ny;
    int bcx, bcy;
    P ihx, ihy;       // 1/dx, 1/dy in the storage precision
    T ihxT, ihyT;
    T epsx, epsy;     // eps/dx^2, eps/dy^2
    int ham;
    T hpT[4];
    double hpD[4];    // the same parameters in FP64 (dissipation, time step)
    double ihxD, ihyD;
    int nbx, nby;
    int remap;        // nonzero: spread neighbouring tiles over one XCD
    int dim;
};

// Stage input at a node inside the grid.
template <int STAGE, typename T, typename P>
__host__ __device__ inline P node_value(const StageArgs<T, P>& a, int64_t idx, double dt,
                                        double ax, double ay) {
    if (STAGE == kStageMid) {
        // phi_1 = phi^n + dt L(phi^n), L = -(Hbar - ax Dx - ay Dy)
        const double ry = a.dim == 2 ? mul_rn(ay, double(a.dya[idx])) : 0.0;
        const double r = double(a.hbar[idx]) - (mul_rn(ax, double(a.dxa[idx])) + ry);
        return P(double(a.phi_n[idx]) - dt * r);
    } else if (STAGE == kStageLast) {
        return a.phi_s[idx];
    } else {
        return a.phi_n[idx];
    }
}

// Wrap or extrapolate one index; returns the real index and, for an
// extrapolated ghost g = 1..3 beyond the edge, g (0 otherwise).  Indices far
// outside (only in the unused part of a partial tile) are clamped.
__host__ __device__ inline int64_t resolve(int64_t i, int64_t n, int bc, int& ghost,
                                           int& side) {
    ghost = 0;
    side = 0;
    if (i >= 0 && i < n) return i;
    if (bc == kBcPeriodic) {
        int64_t r = i % n;
        return r < 0 ? r + n : r;
    }
    if (i < 0) {
        ghost = int(-i);
        side = -1;
        if (ghost > 3) ghost = 3;
        return 0;
    }
    ghost = int(i - n + 1);
    side = 1;
    if (ghost > 3) ghost = 3;
    return n - 1;
}

// Value of the stage input at (i, j), ghosts included.  Only one of the two
// indices is outside the grid on the halo of the plus-shaped stencil; where
// both are (the unused corner of a partial tile) the value is clamped.
template <int STAGE, typename T, typename P>
__host__ __device__ inline P stage_value(const StageArgs<T, P>& a, int64_t i, int64_t j,
                                         double dt, double ax, double ay) {
    int gx, sx, gy, sy;
    const int64_t ri = resolve(i, a.nx, a.bcx, gx, sx);
    const int64_t rj = resolve(j, a.ny, a.bcy, gy, sy);
    const P f0 = node_value<STAGE>(a, rj * a.nx + ri, dt, ax, ay);
    if (gx > 0 && gy == 0) {
        // linear extrapolation along x through the two edge nodes
        const int64_t ri1 = ri - sx;  // the neighbour inside
        const P f1 = node_value<STAGE>(a, rj * a.nx + ri1, dt, ax, ay);
        return P(f0 + P(gx) * (f0 - f1));
    }
    if (gy > 0 && gx == 0) {
        const int64_t rj1 = rj - sy;
        const P f1 = node_value<STAGE>(a, rj1 * a.nx + ri, dt, ax, ay);
        return P(f0 + P(gy) * (f0 - f1));
    }
    return f0;
}

// ---------------------------------------------------------------- the tile
// 512 threads: threads [0, 256) march the rows (phase X) while threads [256, 512)
// march the columns (phase Y) at the same time; after a barrier the column threads
// combine their phi_y^-+ with the phi_x^-+ left in LDS by the row threads.
template <typename T, typename P, int TX, int TY, int SX, int SY>
struct Tile {
    static constexpr int kThreads = 512;
    static constexpr int kHalf = 256;
    static constexpr int PW = TX + 7;      // pitch of the phi tile (odd: fewer bank conflicts)
    static constexpr int PH = TY + 6;
    static constexpr int UW = TX + 1;      // pitch of the phi_x results
    static constexpr int kPhiElems = PH * PW;
    static constexpr int kUElems = 2 * TY * UW;
    static_assert(TY * (TX / SX) == kHalf, "phase X covers the tile rows");
    static_assert(TX * (TY / SY) == kHalf, "phase Y covers the tile columns");

    // Phase 0: phi_s over rows [y0-3, y0+TY+3) x columns [x0-3, x0+TX+3), plus-shaped.
    template <int STAGE>
    __host__ __device__ static void load(int tid, const StageArgs<T, P>& a, int64_t x0,
                                         int64_t y0, double dt, double ax, double ay, P* phiL) {
        constexpr int kRowElems = TY * (TX + 6);   // rows of the tile with the x halo
        constexpr int kColElems = 6 * TX;          // the three rows above and below
        for (int e = tid; e < kRowElems + kColElems; e += kThreads) {
            int r, c;
            if (e < kRowElems) {
                r = e / (TX + 6) + 3;
                c = e % (TX + 6);
            } else {
                const int f = e - kRowElems;
                const int rr = f / TX;                 // 0..5
                r = rr < 3 ? rr : TY + rr;             // 0,1,2, TY+3..TY+5
                c = f % TX + 3;
            }
            phiL[r * PW + c] = stage_value<STAGE>(a, x0 + c - 3, y0 + r - 3, dt, ax, ay);
        }
    }

    // Phase X, t in [0, 256): (row, segment); phi_x^- / phi_x^+ into uL[0|1][row][x].
    __host__ __device__ static void sweep_x(int t, const StageArgs<T, P>& a, const P* phiL,
                                            T* uL) {
        const int row = t % TY;
        const int seg = t / TY;
        T um[SX], up[SX];
        sweep<T, P, SX>(phiL + (row + 3) * PW + seg * SX, 1, a.ihx, a.ihxT, a.epsx, um, up);
#pragma unroll
        for (int k = 0; k < SX; ++k) {
            uL[row * UW + seg * SX + k] = um[k];
            uL[TY * UW + row * UW + seg * SX + k] = up[k];
        }
    }

    // Phase Y, t in [0, 256): (column, segment); phi_y^- / phi_y^+ into registers.
    __host__ __device__ static void sweep_y(int t, const StageArgs<T, P>& a, const P* phiL, T* vm,
                                            T* vp) {
        const int col = t % TX;
        const int seg = t / TX;
        sweep<T, P, SY>(phiL + seg * SY * PW + col + 3, PW, a.ihy, a.ihyT, a.epsy, vm, vp);
    }

    // After the barrier: fin(col, row, um, up, vm, vp) for the thread's SY nodes.
    template <class Fin>
    __host__ __device__ static void finish(int t, const T* uL, const T* vm, const T* vp, Fin& fin) {
        const int col = t % TX;
        const int seg = t / TX;
#pragma unroll
        for (int k = 0; k < SY; ++k) {
            const int row = seg * SY + k;
            fin(col, row, uL[row * UW + col], uL[TY * UW + row * UW + col], vm[k], vp[k]);
        }
    }
};

// One-dimensional tile: TX nodes, S per thread in the sweep.
template <typename T, typename P, int TX, int S>
struct Tile1D {
    static constexpr int kThreads = 256;
    static constexpr int PW = TX + 6;
    static constexpr int kPhiElems = PW;
    static constexpr int kUElems = 2 * TX;
    static_assert(TX / S == kThreads, "sweep covers the tile");

    template <int STAGE>
    __host__ __device__ static void load(int tid, const StageArgs<T, P>& a, int64_t x0,
                                         double dt, double ax, double ay, P* phiL) {
        for (int c = tid; c < PW; c += kThreads)
            phiL[c] = stage_value<STAGE>(a, x0 + c - 3, 0, dt, ax, ay);
    }

    __host__ __device__ static void sweep_x(int tid, const StageArgs<T, P>& a, const P* phiL,
                                            T* uL) {
        T um[S], up[S];
        sweep<T, P, S>(phiL + tid * S, 1, a.ihx, a.ihxT, a.epsx, um, up);
#pragma unroll
        for (int k = 0; k < S; ++k) {
            uL[tid * S + k] = um[k];
            uL[TX + tid * S + k] = up[k];
        }
    }
};

// ---------------------------------------------------------------- node finish
// Per-node work after both sweeps, for each stage kind.  Holds running
// min/max of the derivatives for the pre-stage.
template <int STAGE, typename T, typename P>
struct Finisher {
    const StageArgs<T, P>& a;
    int64_t x0, y0;
    double dt, ax, ay;
    T lo_u, hi_u, lo_v, hi_v;
    bool bad;
    int dim;

    __host__ __device__ Finisher(const StageArgs<T, P>& args, int64_t x0_, int64_t y0_,
                                 double dt_, double ax_, double ay_, int dim_)
        : a(args), x0(x0_), y0(y0_), dt(dt_), ax(ax_), ay(ay_), lo_u(T(INFINITY)),
          hi_u(T(-INFINITY)), lo_v(T(INFINITY)), hi_v(T(-INFINITY)), bad(false), dim(dim_) {}

    __host__ __device__ void operator()(int col, int row, T um, T up, T vm, T vp) {
        const int64_t i = x0 + col, j = y0 + row;
        if (i >= a.nx || j >= a.ny) return;
        const int64_t idx = j * a.nx + i;
        if (STAGE == kStageDeriv) {
            a.dout0[idx] = double(um);
            a.dout1[idx] = double(up);
            if (dim == 2) {
                a.dout2[idx] = double(vm);
                a.dout3[idx] = double(vp);
            }
            return;
        }
        const T ub = T(0.5) * (up + um), vb = T(0.5) * (vp + vm);
        const T Dx = T(0.5) * (up - um), Dy = T(0.5) * (vp - vm);
        const T H = hamiltonian(a.ham, a.hpT, ub, vb);
        if (STAGE == kStagePre) {
            a.hbar[idx] = H;
            a.dxa[idx] = Dx;
            if (dim == 2) a.dya[idx] = Dy;
            lo_u = fmin(lo_u, fmin(um, up));
            hi_u = fmax(hi_u, fmax(um, up));
            lo_v = fmin(lo_v, fmin(vm, vp));
            hi_v = fmax(hi_v, fmax(vm, vp));
            if (!(finite_t(H) && finite_t(Dx) && finite_t(Dy))) bad = true;
            return;
        }
        // L = -(H - (ax Dx + ay Dy)); the sum is symmetric in x and y
        const T R = H - (mul_rn(T(ax), Dx) + mul_rn(T(ay), Dy));
        const double pn = double(a.phi_n[idx]);
        double res;
        if (STAGE == kStageMid) {
            const double p1 = double(node_value<kStageMid>(a, idx, dt, ax, ay));
            res = 0.75 * pn + 0.25 * (p1 - dt * double(R));
        } else {
            const double p2 = double(a.phi_s[idx]);
            res = (1.0 / 3.0) * pn + (2.0 / 3.0) * (p2 - dt * double(R));
        }
        const P outv = P(res);
        a.out[idx] = outv;
        if (!finite_t(outv)) bad = true;
    }
};

}  // namespace hjw
