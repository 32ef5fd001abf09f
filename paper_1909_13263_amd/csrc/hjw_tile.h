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
//   L = h * M(a, b), M = mean of sqrt(1+s^2) for s between the end values; M^2 is
//   evaluated from a Taylor series about the midpoint when the pair is close
//   (relative half-gap below TAU; no square root needed) and from the antiderivative
//   otherwise.  With t_k = (eps/h^2 + M_k^2)^2 the weights become products of the
//   other two t's (one division per side); in FP32 the t's are first scaled by 1/max t.
//   The weighted sum is formed as the central candidate plus a correction made
//   of two third differences (see sweep()).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace hjw {

constexpr int kBcPeriodic = 0;
constexpr int kBcExtrap = 1;
// Dirichlet: the three outermost node layers of the axis hold boundary data; they keep
// their values, and their derivatives enter neither the ranges nor the update.  Loads
// treat the axis as extrapolated: only those layers read the ghosts.
constexpr int kBcDirichlet = 2;
constexpr int kHLinear = 0;
constexpr int kHBurgers = 1;
constexpr int kHNegcos = 2;
constexpr int kHNorm = 3;
constexpr int kHQuartic = 4;
constexpr int kHControl = 5;
constexpr int kHCurvature = 6;   // NORM plus the curvature term of Example 3.13
constexpr int kHTimed = 7;       // cos(w t)(a u + b v) + lam phi: depends on t and phi

// Node variants of the finish (Finisher::mode): plain; with held Dirichlet layers or the
// curvature term; the time- and phi-dependent family (held layers possible).
constexpr int kNodePlain = 0;
constexpr int kNodeExtended = 1;
constexpr int kNodeTimed = 2;   // also every launch with the local dissipation (llf)

// Stage kinds of one Runge-Kutta step.
constexpr int kStagePre = 0;    // derivatives of phi^n -> Hbar, Dx, Dy, block ranges
constexpr int kStageMid = 1;    // phi_1 rebuilt on the fly -> phi_2
constexpr int kStageLast = 2;   // phi_2 -> phi^{n+1}, in place over phi^n
constexpr int kStageDeriv = 3;  // derivatives only (u-, u+, v-, v+ as FP64)

constexpr double kEps = 1.0e-6;  // epsilon of eq. (WLOC1)

// Schemes: WENO-L (the paper's arc-length indicators) and WENO-JP (the comparison
// scheme of Section 3: Jiang and Peng's indicators, same candidates and weights).
constexpr int kSchemeL = 0;
constexpr int kSchemeJP = 1;

// The additive constant of t_k = (eps' + X_k)^2 in the weights, per scheme: WENO-L
// works with X = (2M)^2 = 4 beta / h^2, so eps' = 4 eps / h^2; WENO-JP's indicators are
// used as defined, so eps' = eps.
inline double weight_eps(int scheme, double h) {
    return scheme == kSchemeJP ? kEps : 4.0 * kEps / (h * h);
}

// Tile shapes: 64 x TY nodes per workgroup in 2-D (TY = 16 or 32), each thread
// marching a segment of S nodes along a row or a column (S = 8, or S = 4 for twice
// the threads on grids too small to fill the GPU) and then finishing S/2 nodes;
// 1024 nodes in 1-D (segments of 4).
constexpr int kTX = 64;
constexpr int kTX1 = 1024, kS1 = 4;
// Threads of a 2-D workgroup: as many row threads as column threads.
constexpr int threads2d(int ty, int seg) { return 2 * (kTX / seg) * ty; }
// Waves per SIMD asked of the FP64 16-row stage kernels (3 tiles a CU; VGPRs <= 168).
constexpr int fp64_waves(int elem, int ty) { return elem == 8 && ty == 16 ? 3 : 1; }

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

// Block partials of the CPU emulation: min/max of u+-, v+- and a bad flag.
constexpr int kPartialStride = 5;

// ---------------------------------------------------------------- math helpers
// Host and device overloads of the few primitives whose fast device form is a
// builtin; everything else is ordinary C++ arithmetic.
__device__ inline float rcp_t(float x) { return __builtin_amdgcn_rcpf(x); }
__host__ inline float rcp_t(float x) { return 1.0f / x; }
__host__ __device__ inline double rcp_t(double x) { return 1.0 / x; }
__device__ inline double log_t(double x) { return log(x); }
__host__ inline double log_t(double x) { return std::log(x); }
__device__ inline float sqrt_t(float x) { return sqrtf(x); }
__host__ inline float sqrt_t(float x) { return std::sqrt(x); }
__device__ inline double sqrt_t(double x) { return sqrt(x); }
__host__ inline double sqrt_t(double x) { return std::sqrt(x); }
__device__ inline float sin_t(float x) { return sinf(x); }
__host__ inline float sin_t(float x) { return std::sin(x); }
__device__ inline double sin_t(double x) { return sin(x); }
__host__ inline double sin_t(double x) { return std::sin(x); }
__device__ inline float cos_t(float x) { return cosf(x); }
__host__ inline float cos_t(float x) { return std::cos(x); }
__device__ inline double cos_t(double x) { return cos(x); }
__host__ inline double cos_t(double x) { return std::cos(x); }
__device__ inline bool any_lane(bool p) { return __any(p ? 1 : 0) != 0; }
__host__ inline bool any_lane(bool p) { return p; }
// A value the caller knows to be the same on every lane of the wave (a wave's index, a row
// of a wave's task): taken from the first lane, so the compiler keeps it, and the index
// arithmetic built on it, in scalar registers.
__device__ inline int uniform_int(int x) { return __builtin_amdgcn_readfirstlane(x); }
__host__ inline int uniform_int(int x) { return x; }
// Product of two values below 2^24 (grid sides are at most 2^20): one full-rate multiply.
__device__ inline uint32_t mul_u24(uint32_t x, uint32_t y) { return __umul24(x, y); }
__host__ inline uint32_t mul_u24(uint32_t x, uint32_t y) { return x * y; }
// Element `off` of an array that starts at `base`, the offset taken in bytes as a 32-bit
// unsigned value: with a base that is uniform over the wave, the load or store addresses
// it as a scalar base plus a 32-bit vector offset, with no 64-bit arithmetic per element.
// Callers keep off * sizeof(X) below 2^32 (offsets inside a tile's rows of one grid).
template <typename X>
__host__ __device__ inline const X& at(const X* base, uint32_t off) {
    return *reinterpret_cast<const X*>(reinterpret_cast<const char*>(base) +
                                       off * uint32_t(sizeof(X)));
}
template <typename X>
__host__ __device__ inline X& at(X* base, uint32_t off) {
    return *reinterpret_cast<X*>(reinterpret_cast<char*>(base) + off * uint32_t(sizeof(X)));
}
// Products that are rounded on their own (never fused into an add), so that sums
// like a*u + b*v are symmetric under exchanging (a,u) and (b,v) bit for bit.
// (The pragma takes the product out of FMA contraction; __fmul_rn does not.)
__host__ __device__ inline float mul_rn(float a, float b) {
#pragma clang fp contract(off)
    return a * b;
}
__host__ __device__ inline double mul_rn(double a, double b) {
#pragma clang fp contract(off)
    return a * b;
}
// Fused multiply-adds written out.  Together with mul_rn they leave the compiler no
// choice of which product to fuse into which sum: a choice it makes from the use counts
// and placement of the products, which differ between the instantiations of one march.
__device__ inline float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__host__ inline float fma_t(float a, float b, float c) { return std::fma(a, b, c); }
__host__ __device__ inline double fma_t(double a, double b, double c) {
    return __builtin_fma(a, b, c);
}

template <typename T>
__host__ __device__ inline bool finite_t(T x) {
    return __builtin_isfinite(x);  // one class test on the device
}

// Relative half-gap below which M comes from the midpoint series, and the
// series length: the truncation error stays below one unit in the last place
// (4 terms to 2e-2 in FP64, 3 terms to 1e-1 in FP32).
template <typename T> struct SeriesCfg;
template <> struct SeriesCfg<double> { static constexpr double tau2 = 4.0e-4; };
template <> struct SeriesCfg<float> { static constexpr float tau2 = 1.0e-2f; };

// The square of twice the mean of sqrt(1+s^2) between a and b, from the sum sg = a + b
// and the difference dl = b - a, by the midpoint expansion
//   2M = sqrt(q4) X,  X = 1 + g^2 (2/3 + g^2 (2/5 (sg^2-1) + g^2 2/7 (sg^4 - 6 sg^2 + 2))),
//   q4 = 4 + sg^2, g = dl / q4
// (the Taylor series of the mean about m = sg/2 with y = (h/(1+m^2))^2 = 4 g^2), so
// (2M)^2 = q4 X^2 needs no square root.  xx receives the squared relative gap dl^2 / q4.
__host__ __device__ inline double mean2sq_series(double sg, double dl, double q4, double& xx) {
    const double g = dl / q4;
    xx = dl * g;
    const double g2 = g * g;
    const double s2 = mul_rn(sg, sg);
    const double t3 = (2.0 / 7.0) * fma_t(s2, s2 - 6.0, 2.0);
    const double inner = fma_t(g2, fma_t(g2, t3, mul_rn(0.4, s2 - 1.0)), 2.0 / 3.0);
    const double X = fma_t(g2, inner, 1.0);
    return mul_rn(q4 * X, X);   // rounded alone: the weights add eps to it on every path
}
__host__ __device__ inline float mean2sq_series(float sg, float dl, float q4, float& xx) {
    const float g = dl * rcp_t(q4);
    xx = dl * g;
    const float g2 = g * g;
    const float inner = fma_t(g2, 0.4f * fma_t(sg, sg, -1.0f), 2.0f / 3.0f);
    const float X = fma_t(g2, inner, 1.0f);
    return mul_rn(q4 * X, X);
}

// Antiderivative of sqrt(1+s^2): (s sqrt(1+s^2) + asinh s) / 2, with
// asinh s = sign(s) ln(|s| + sqrt(1+s^2)): the logarithm's argument is >= 1 (no
// cancellation) and the square root serves both terms.  Only pairs with a wide relative
// gap use it, so that the difference of two values is divided by a gap of at least
// tau sqrt(4 + sg^2): the rounding is amplified by a small factor only.
__host__ __device__ inline double prim(double s) {
    const double r = sqrt_t(fma_t(s, s, 1.0));
    return 0.5 * fma_t(s, r, copysign(log_t(fabs(s) + r), s));
}
// FP32: the same from the hardware square root and base-2 logarithm (about 1 ulp each).
__device__ inline float prim(float s) {
    const float r = __builtin_amdgcn_sqrtf(fmaf(s, s, 1.0f));
    const float l = __builtin_amdgcn_logf(fabsf(s) + r) * 0.693147180559945309f;
    return 0.5f * fma_t(s, r, copysignf(l, s));
}
__host__ inline float prim(float s) {
    const float r = std::sqrt(std::fma(s, s, 1.0f));
    const float l = std::log2(std::fabs(s) + r) * 0.693147180559945309f;
    return 0.5f * fma_t(s, r, std::copysign(l, s));
}

// Quotients: exact division in FP64; in FP32 a product with the hardware reciprocal.
template <typename T>
__host__ __device__ inline T wdiv(T num, T den) {
    return num / den;
}
template <>
__host__ __device__ inline float wdiv<float>(float num, float den) {
    return num * rcp_t(den);
}
// q + num / den: in FP32 one fused multiply-add with the reciprocal.
__host__ __device__ inline double add_quot(double q, double num, double den) {
    return q + num / den;
}
__host__ __device__ inline float add_quot(float q, float num, float den) {
    return fma_t(num, rcp_t(den), q);
}

// Squares of the doubled means for the three pairs of one cell: (c0, b1), (c0, c1),
// (f0, c1).  A pair whose relative half-gap is not small takes the antiderivative
// instead; the wave takes that branch only when one of its lanes needs it.  The
// squares are rounded on their own (mul_rn), so that a lane's value does not depend
// on whether its wave took the branch (a product fused into the weights' sums on one
// path only would round differently).
template <typename T>
__host__ __device__ inline void cell_means(T c0, T b1, T c1, T f0, T& MA2, T& MB2, T& MC2) {
    const T tau2 = SeriesCfg<T>::tau2;
    const T sA = c0 + b1, dA = b1 - c0;
    const T sB = c0 + c1, dB = c1 - c0;
    const T sC = f0 + c1, dC = c1 - f0;
    const T qA = fma_t(sA, sA, T(4)), qB = fma_t(sB, sB, T(4)), qC = fma_t(sC, sC, T(4));
    // half-gap dl/2 against tau sqrt(1 + m^2) = tau sqrt(q4)/2: wide when dl^2/q4 >= tau^2
    T xA, xB, xC;
    MA2 = mean2sq_series(sA, dA, qA, xA);
    MB2 = mean2sq_series(sB, dB, qB, xB);
    MC2 = mean2sq_series(sC, dC, qC, xC);
    if (any_lane(fmax(xA, fmax(xB, xC)) >= tau2)) {
        const T Pc0 = prim(c0), Pb1 = prim(b1), Pc1 = prim(c1), Pf0 = prim(f0);
        if (xA >= tau2) {
            const T M = wdiv(T(2) * (Pb1 - Pc0), dA);
            MA2 = mul_rn(M, M);
        }
        if (xB >= tau2) {
            const T M = wdiv(T(2) * (Pc1 - Pc0), dB);
            MB2 = mul_rn(M, M);
        }
        if (xC >= tau2) {
            const T M = wdiv(T(2) * (Pc1 - Pf0), dC);
            MC2 = mul_rn(M, M);
        }
    }
}

// WENO-JP indicators of the three sub-stencils of one cell from the second differences
// (divided by h) e1..e4 = Delta^- Delta^+ phi_{i-2..i+1} / h:
//   IS_A = 13 (e1-e2)^2 + 3 (e1-3 e2)^2, IS_B = 13 (e2-e3)^2 + 3 (e2+e3)^2,
//   IS_C = 13 (e3-e4)^2 + 3 (3 e3-e4)^2;
// as for WENO-L, the same three serve phi^-_i and, reversed, phi^+_{i-1}.
template <typename T>
__host__ __device__ inline void jp_indicators(T e1, T e2, T e3, T e4, T& IA, T& IB, T& IC) {
    const T a0 = e1 - e2, a1 = fma_t(T(-3), e2, e1);
    const T b0 = e2 - e3, b1 = e2 + e3;
    const T c0 = e3 - e4, c1 = fma_t(T(3), e3, -e4);
    IA = fma_t(T(13), a0 * a0, mul_rn(T(3), a1 * a1));
    IB = fma_t(T(13), b0 * b0, mul_rn(T(3), b1 * b1));
    IC = fma_t(T(13), c0 * c0, mul_rn(T(3), c1 * c1));
}

// Products of the weight denominators: with t_k = (eps/h^2 + M_k^2)^2 (up to a
// common factor), omega_k of eq. (WLOC1) is proportional to d_k times the product
// of the other two t's.  Inputs are the squared doubled means and eps4 = 4 eps / h^2.
__host__ __device__ inline void weight_products(double MA2, double MB2, double MC2, double eps4,
                                                double& pAB, double& pAC, double& pBC) {
    double tA = eps4 + MA2, tB = eps4 + MB2, tC = eps4 + MC2;
    tA *= tA;
    tB *= tB;
    tC *= tC;
    pAB = tA * tB;
    pAC = tA * tC;
    pBC = tB * tC;
}
// FP32: the t's are first scaled by 1/max t so that no product overflows.
__host__ __device__ inline void weight_products(float MA2, float MB2, float MC2, float eps4,
                                                float& pAB, float& pAC, float& pBC) {
    float tA = eps4 + MA2, tB = eps4 + MB2, tC = eps4 + MC2;
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


// March along one line.  line[k*stride] is phi_s at position p0-3+k,
// k = 0..S+5; hands phi^-(p0+k) to emit.minus(k, .) and phi^+(p0+k) to emit.plus(k, .),
// k < S, as soon as the march has formed each (sweep() collects them in um[k], up[k]).
// Differences are formed in the storage precision P and then cast to T.
//
// With v_j = Delta^+ phi_j and the cell [x_{i-1}, x_i] seeing (a,b,c,d,e) =
// v_{i-3..i+1}, first differences e1..e4 of (a..e) give
//   C_{i-1} = e2/h, C_i = e3/h, B_i = (2 e2 - e1)/h, F_{i-1} = (2 e3 - e4)/h,
// and the candidates of Step 2 differ from the central one by third differences:
//   q0 - q1 = D3a/3, q2 - q1 = D3b/6, D3a = a - 3b + 3c - d, D3b = b - 3c + 3d - e,
//   q1 = c + (e2 + 2 e3)/6 for phi^- at x_i, and mirrored for phi^+ at x_{i-1}:
//   qp1 = c - (e3 + 2 e2)/6, qp0 - qp1 = -D3b/3, qp2 - qp1 = -D3a/6.
// So phi^- = q1 + (w0 (q0-q1) + w2 (q2-q1)) / (w0 + w1 + w2), and likewise phi^+.
template <typename T, typename P, int S, int SCHEME, class Emit>
__host__ __device__ inline void sweep_emit(const P* line, int stride, P ihP, T ih, T eps4,
                                           Emit&& emit) {
    // The quotients are rounded on their own: fused into the differences that follow,
    // they would round differently at the ends of a segment than inside it.
    T v[S + 5];
#pragma unroll
    for (int k = 0; k < S + 5; ++k)
        v[k] = T(mul_rn(line[(k + 1) * stride] - line[k * stride], ihP));
    T e1 = v[1] - v[0], e2 = v[2] - v[1], e3 = v[3] - v[2];
    // The end values are rounded on their own too: C_i is carried to the next cell, and a
    // product fused into a sum in one iteration but not in another would make a node's
    // value depend on where its segment starts.
    T c0 = mul_rn(e2, ih);
#pragma unroll
    for (int it = 0; it <= S; ++it) {
        const T c = v[it + 2];
        const T e4 = v[it + 4] - v[it + 3];
        const T B1 = T(2) * e2 - e1;          // h B_i
        const T F0 = T(2) * e3 - e4;          // h F_{i-1}
        const T c1 = mul_rn(e3, ih);          // C_i
        const T b1 = mul_rn(B1, ih);          // B_i
        const T f0 = mul_rn(F0, ih);          // F_{i-1}
        T XA, XB, XC;   // squared doubled means (WENO-L) or indicators (WENO-JP)
        if (SCHEME == kSchemeJP)
            jp_indicators(e1, e2, e3, e4, XA, XB, XC);
        else
            cell_means(c0, b1, c1, f0, XA, XB, XC);
        T pAB, pAC, pBC;
        weight_products(XA, XB, XC, eps4, pAB, pAC, pBC);
        const T D3a = B1 - e3;                // a - 3b + 3c - d
        const T D3b = F0 - e2;                // b - 3c + 3d - e
        // numerators and denominators below are six times those of the weighted sums
        const T xa = mul_rn(pBC, D3a), xb = mul_rn(pAB, D3b);
        const T p36AC = mul_rn(T(36), pAC);
        if (it < S) {  // phi^- at node i: weights (1/10, 6/10, 3/10) on (A, B, C)
            const T q1 = fma_t(e2 + T(2) * e3, T(1.0 / 6.0), c);
            const T num = fma_t(T(3), xb, xa + xa);             // 6 (pBC D3a/3 + pAB D3b/2)
            const T den = fma_t(T(18), pAB, fma_t(T(6), pBC, p36AC));
            emit.minus(it, add_quot(q1, num, den));
        }
        if (it > 0) {  // phi^+ at node i-1: the mirrored sub-stencils, (1/10, 6/10, 3/10) on (C, B, A)
            const T qp1 = fma_t(-(e3 + T(2) * e2), T(1.0 / 6.0), c);
            const T num = fma_t(T(3), xa, xb + xb);             // 6 (pAB D3b/3 + pBC D3a/2)
            const T den = fma_t(T(18), pBC, fma_t(T(6), pAB, p36AC));
            emit.plus(it - 1, add_quot(qp1, -num, den));
        }
        e1 = e2;
        e2 = e3;
        e3 = e4;
        c0 = c1;
    }
}
template <typename T>
struct ToArrays {
    T* um;
    T* up;
    __host__ __device__ void minus(int k, T v) const { um[k] = v; }
    __host__ __device__ void plus(int k, T v) const { up[k] = v; }
};
template <typename T, typename P, int S, int SCHEME>
__host__ __device__ inline void sweep(const P* line, int stride, P ihP, T ih, T eps4, T* um,
                                      T* up) {
    sweep_emit<T, P, S, SCHEME>(line, stride, ihP, ih, eps4, ToArrays<T>{um, up});
}

// ---------------------------------------------------------------- Hamiltonians
// H(u, v) at the node (x, y); only the control Hamiltonian of Example 3.11 depends on
// the position (the family that depends on t and phi, TIMED, is evaluated by the
// finisher, which holds the stage time):
//   LINEAR a u + b v; BURGERS s^2/2; NEGCOS -cos s; QUARTIC (s^2-1)(s^2-4)/4 with
//   s = a u + b v + c; NORM and CURVATURE k0 sqrt(u^2 + v^2 + k1) (the curvature term
//   is added by the finisher);
//   CONTROL sin(y) u + (sin(x) + sign v) v - sin(y)^2/2 - (1 - cos x).
template <typename T>
__host__ __device__ inline T hamiltonian(int kind, const T* p, T u, T v, T x, T y) {
    switch (kind) {
    case kHLinear:
        return mul_rn(p[0], u) + mul_rn(p[1], v);
    case kHBurgers: {
        const T s = (mul_rn(p[0], u) + mul_rn(p[1], v)) + p[2];
        return T(0.5) * s * s;
    }
    case kHNegcos:
        return -cos_t((mul_rn(p[0], u) + mul_rn(p[1], v)) + p[2]);
    case kHQuartic: {
        const T s = (mul_rn(p[0], u) + mul_rn(p[1], v)) + p[2];
        const T s2 = s * s;
        return T(0.25) * ((s2 - T(1)) * (s2 - T(4)));
    }
    case kHControl: {
        const T sy = sin_t(y);
        const T sgn = T((v > T(0)) - (v < T(0)));
        return sy * u + (sin_t(x) + sgn) * v - T(0.5) * sy * sy - (T(1) - cos_t(x));
    }
    default:
        return p[0] * sqrt_t((mul_rn(u, u) + mul_rn(v, v)) + p[1]);
    }
}

// max of |s^3 - 5s/2| (the slope of the quartic in s) on [lo, hi]: the ends and the
// critical points +-sqrt(5/6) that lie inside.
__host__ __device__ inline double max_abs_quartic_slope(double lo, double hi) {
    const double sc = 0.91287092917527685576;   // sqrt(5/6)
    double m = 0.0;
    const double cand[4] = {lo, hi, -sc, sc};
    for (int k = 0; k < 4; ++k) {
        const double s = cand[k];
        if (s >= lo && s <= hi) m = fmax(m, fabs(s * s * s - 2.5 * s));
    }
    return m;
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
    if (kind == kHLinear || kind == kHTimed) {
        // TIMED: |H_u| = |a cos(w t)| <= |a| at every stage time
        ax = fabs(p[0]);
        ay = fabs(p[1]);
    } else if (kind == kHControl) {
        // |H_u| = |sin y| <= 1, |H_v| = |sin x + sign v| <= 2 wherever the nodes lie
        ax = 1.0;
        ay = dim == 2 ? 2.0 : 0.0;
    } else if (kind == kHBurgers || kind == kHNegcos || kind == kHQuartic) {
        // s = p0 u + p1 v + p2 takes its extremes on the box at corners
        const double s0 = mul_rn(p[0], A) + mul_rn(p[1], C);
        const double s1 = mul_rn(p[0], A) + mul_rn(p[1], D);
        const double s2 = mul_rn(p[0], B) + mul_rn(p[1], C);
        const double s3 = mul_rn(p[0], B) + mul_rn(p[1], D);
        const double lo = fmin(fmin(s0, s1), fmin(s2, s3)) + p[2];
        const double hi = fmax(fmax(s0, s1), fmax(s2, s3)) + p[2];
        const double m = kind == kHBurgers  ? fmax(fabs(lo), fabs(hi))
                         : kind == kHNegcos ? max_abs_sin(lo, hi)
                                            : max_abs_quartic_slope(lo, hi);
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
// dt = cfl / (ax/dx + ay/dy) (plus the curvature term's limit), landing exactly on t_final.
__host__ __device__ inline void plan_step(DevState& s, int kind, const double* p, int dim,
                                          double ihx, double ihy, const double range[4]) {
    double ax, ay;
    dissipation(kind, p, dim, range[0], range[1], range[2], range[3], ax, ay);
    double rate = mul_rn(ax, ihx) + (dim == 2 ? mul_rn(ay, ihy) : 0.0);
    // the curvature term diffuses with a coefficient of at most eps = p[2]
    if (kind == kHCurvature) rate += 2.0 * p[2] * (mul_rn(ihx, ihx) + mul_rn(ihy, ihy));
    // the zero-order term lam phi of TIMED: |lam| dt <= cfl
    if (kind == kHTimed) rate += fabs(p[3]);
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
template <typename T>
struct Flux3 {
    T h, dx, dy;
};

template <typename T, typename P>
struct StageArgs {
    const P* phi_n;   // phi^n
    const P* phi_s;   // stage input of the last stage (phi_2)
    P* out;           // stage output (phi_2, or phi^{n+1} over phi^n)
    T* flux;          // pre-stage outputs per node, interleaved:
                      // [3 i] = H(ubar, vbar), [3 i + 1] = (u+ - u-)/2, [3 i + 2] = (v+ - v-)/2
    double* dout0;    // derivative outputs (kStageDeriv)
    double* dout1;
    double* dout2;
    double* dout3;
    DevState* st;     // two step records; this step reads st[par] and writes st[par ^ 1]
    int par;
    void* slots;      // range accumulators of the first stage (see the kernels)
    int64_t nx, ny;
    int bcx, bcy;
    P ihx, ihy;       // 1/dx, 1/dy in the storage precision
    T ihxT, ihyT;
    T epsx, epsy;     // weight_eps(scheme, dx), weight_eps(scheme, dy)
    int ham;
    T hpT[4];
    double hpD[4];    // the same parameters in FP64 (dissipation, time step)
    double ihxD, ihyD;
    int nbx, nby;
    int remap;        // nonzero: spread neighbouring tiles over one XCD
    int dim;
    int plan_ready;   // nonzero: the step plan was published by its own launch
    int scheme;       // kSchemeL or kSchemeJP
    double x0, y0;    // coordinates of node (0, 0)
    double dxD, dyD;  // spacing in FP64
    int llf;          // nonzero: alpha of eq. (LF) per node over its own pair (local LF)
};

// Stage input at a node inside the grid.
template <int STAGE, typename T, typename P>
__host__ __device__ inline P node_value(const StageArgs<T, P>& a, int64_t idx, double dt,
                                        double ax, double ay) {
    if (STAGE == kStageMid) {
        // phi_1 = phi^n + dt L(phi^n), L = -(Hbar - (ax Dx + ay Dy))
        // f.dy and ay are 0 on a 1-D grid, so no test of the dimension: a load under such a
        // test is issued late and waited for at once, one memory round trip per node
        const Flux3<T> f = reinterpret_cast<const Flux3<T>*>(a.flux)[idx];
        const double r = double(f.h) - (mul_rn(ax, double(f.dx)) + mul_rn(ay, double(f.dy)));
        return P(fma(-dt, r, double(a.phi_n[idx])));
    } else if (STAGE == kStageLast) {
        return a.phi_s[idx];
    } else {
        return a.phi_n[idx];
    }
}

// The same, for the node `off` elements after the node `base` (a tile's uniform origin).
template <int STAGE, typename T, typename P>
__host__ __device__ inline P node_value_at(const StageArgs<T, P>& a, int64_t base, uint32_t off,
                                           double dt, double ax, double ay) {
    if (STAGE == kStageMid) {
        const Flux3<T> f = at(reinterpret_cast<const Flux3<T>*>(a.flux) + base, off);
        const double r = double(f.h) - (mul_rn(ax, double(f.dx)) + mul_rn(ay, double(f.dy)));
        return P(fma(-dt, r, double(at(a.phi_n + base, off))));
    } else if (STAGE == kStageLast) {
        return at(a.phi_s + base, off);
    } else {
        return at(a.phi_n + base, off);
    }
}

// Wrap or extrapolate one index; returns the real index and, for an
// extrapolated ghost g = 1..3 beyond the edge, g (0 otherwise).  Indices far
// outside (only in the unused part of a partial tile) are clamped.
// Coordinates are 32-bit: a side has at most 2^30 nodes.
__host__ __device__ inline int resolve(int i, int n, int bc, int& ghost, int& side) {
    ghost = 0;
    side = 0;
    if (i >= 0 && i < n) return i;
    if (bc == kBcPeriodic) {
        // one wrap reaches every node a real node's stencil needs (they lie within 3 of
        // the grid, and n >= 8); nodes further out belong to the unused part of a partial
        // tile and are clamped
        const int r = i < 0 ? i + n : i - n;
        return r < 0 ? 0 : (r >= n ? n - 1 : r);
    }
    if (i < 0) {
        ghost = int(-i);
        side = -1;
        if (ghost > 3) ghost = 3;
        return 0;
    }
    ghost = i - n + 1;
    side = 1;
    if (ghost > 3) ghost = 3;
    return n - 1;
}

// Index of node (i, j) of a grid nx wide (0 <= i, j < 2^31, nx < 2^32): one 32 x 32-bit
// multiply-add into 64 bits.
__host__ __device__ inline int64_t grid_index(int j, int i, int64_t nx) {
    return int64_t(uint64_t(uint32_t(j)) * uint64_t(uint32_t(nx)) + uint64_t(uint32_t(i)));
}

// Where the stage input at (i, j) comes from, ghosts included: idx0 is the node (the
// edge node for a ghost) and, for a ghost g = 1..3 beyond an edge along one axis, idx1 is
// its neighbour inside, the value being extrapolated linearly through the two; otherwise
// idx1 = idx0 and g = 0.  Only one of the two indices is outside the grid on the halo of
// the plus-shaped stencil; where both are (the unused corner of a partial tile) the value
// is clamped.
template <typename T, typename P>
__host__ __device__ inline void ghost_pair(const StageArgs<T, P>& a, int64_t i, int64_t j,
                                           int64_t& idx0, int64_t& idx1, int& g) {
    int gx, sx, gy, sy;
    const int ri = resolve(int(i), int(a.nx), a.bcx, gx, sx);
    const int rj = resolve(int(j), int(a.ny), a.bcy, gy, sy);
    const bool ex = gx > 0 && gy == 0, ey = gy > 0 && gx == 0;
    idx0 = grid_index(rj, ri, a.nx);
    idx1 = grid_index(ey ? rj - sy : rj, ex ? ri - sx : ri, a.nx);
    g = ex ? gx : (ey ? gy : 0);
}

template <typename P>
__host__ __device__ inline P extrapolate(P f0, P f1, int g) {
    return g ? P(f0 + P(g) * (f0 - f1)) : f0;
}

// Value of the stage input at (i, j), ghosts included.  Both values are loaded
// unconditionally (the same node twice when there is no ghost), so that the loads do
// not wait on a branch.
template <int STAGE, typename T, typename P>
__host__ __device__ inline P stage_value(const StageArgs<T, P>& a, int64_t i, int64_t j,
                                         double dt, double ax, double ay) {
    int64_t i0, i1;
    int g;
    ghost_pair(a, i, j, i0, i1, g);
    const P f0 = node_value<STAGE>(a, i0, dt, ax, ay);
    const P f1 = node_value<STAGE>(a, i1, dt, ax, ay);
    return extrapolate(f0, f1, g);
}

// ---------------------------------------------------------------- the tile
// 2 * kHalf threads: threads [0, kHalf) march the rows (phase X) while threads
// [kHalf, 2 kHalf) march the columns (phase Y) at the same time; after a barrier the
// column threads combine their phi_y^-+ with the phi_x^-+ left in LDS by the row threads.
template <typename T, typename P, int TX, int TY, int SX, int SY>
struct Tile {
    static constexpr int kHalf = TY * (TX / SX);
    static constexpr int kThreads = 2 * kHalf;
    static constexpr int PW = TX + 7;      // pitch of the phi tile (odd: fewer bank conflicts)
    static constexpr int PH = TY + 6;
    static constexpr int UW = TX + 1;      // pitch of the phi_x results
    static constexpr int kPhiElems = PH * PW;
    static constexpr int kUElems = 2 * TY * UW;
    static constexpr int kCenterElems = TX * TY;   // phi^n on the tile (second/third stage)
    static_assert(TX * (TY / SY) == kHalf, "phase Y covers the tile columns with as many threads");
    static_assert(kHalf % 64 == 0, "row and column threads are whole waves");

    // Phase 0: phi_s over rows [y0-3, y0+TY+3) x columns [x0-3, x0+TX+3), plus-shaped.
    // Tiles whose halo lies inside the grid index it directly (TX and TY are powers of
    // two, so the index arithmetic is shifts and masks); tiles at an edge resolve each
    // point through the boundary condition.  Each thread issues all its loads before it
    // writes any of them to LDS, so their latencies overlap.
    // The second and third stages also keep phi^n of the tile's own nodes in pnL.
    template <int STAGE>
    __host__ __device__ static void load(int tid, const StageArgs<T, P>& a, int64_t x0,
                                         int64_t y0, double dt, double ax, double ay, P* phiL,
                                         P* pnL) {
        static_assert((TX & (TX - 1)) == 0 && (TY & (TY - 1)) == 0, "power-of-two tile");
        constexpr bool kCenter = STAGE == kStageMid || STAGE == kStageLast;
        // element e of this thread's j-th load; the last round is partial, and its idle
        // threads load a valid element whose value they drop
        auto element = [&](int j) {
            const int e = tid + j * kThreads;
            return e < kPlusElems ? e : kPlusElems - 1;
        };
        P val[kPerThread];
        P cen[kPerThread];
        if (inside(a, x0, y0)) {
            // global index of phiL[0], uniform; an element's offset from it is below
            // (TY + 6) nx + TX + 6 elements, which fits 32 bits in bytes
            const int64_t base = (y0 - 3) * a.nx + (x0 - 3);
#pragma unroll
            for (int j = 0; j < kPerThread; ++j) {
                int r, c;
                plus_node(element(j), r, c);
                const uint32_t off = mul_u24(uint32_t(r), uint32_t(a.nx)) + uint32_t(c);
                val[j] = node_value_at<STAGE>(a, base, off, dt, ax, ay);
                if (kCenter && j * kThreads < TY * TX) cen[j] = at(a.phi_n + base, off);
            }
        } else if (a.bcx == kBcPeriodic && a.bcy == kBcPeriodic) {
            // every halo index wraps to one node: one value per element
            const bool full = x0 + TX <= a.nx && y0 + TY <= a.ny;
            int64_t i0[kPerThread];
#pragma unroll
            for (int j = 0; j < kPerThread; ++j) {
                if (own_round(j) && full) {
                    i0[j] = own_index(tid + j * kThreads, a, x0, y0);
                } else {
                    int r, c;
                    plus_node(element(j), r, c);
                    int64_t i1;
                    int g;
                    ghost_pair(a, x0 + c - 3, y0 + r - 3, i0[j], i1, g);
                }
            }
#pragma unroll
            for (int j = 0; j < kPerThread; ++j) {
                val[j] = node_value<STAGE>(a, i0[j], dt, ax, ay);
                if (kCenter && j * kThreads < TY * TX) {
                    const int e = element(j);
                    const int i = int(x0) + (e % TX), jj = int(y0) + (e / TX);
                    const int ic = i < a.nx ? i : int(a.nx) - 1;
                    const int jc = jj < a.ny ? jj : int(a.ny) - 1;
                    cen[j] = a.phi_n[grid_index(int(jc), int(ic), a.nx)];
                }
            }
        } else {
            const bool full = x0 + TX <= a.nx && y0 + TY <= a.ny;
            int64_t i0[kPerThread], i1[kPerThread];
            int g[kPerThread];
#pragma unroll
            for (int j = 0; j < kPerThread; ++j) {
                if (own_round(j) && full) {
                    i0[j] = i1[j] = own_index(tid + j * kThreads, a, x0, y0);
                    g[j] = 0;
                } else {
                    int r, c;
                    plus_node(element(j), r, c);
                    ghost_pair(a, x0 + c - 3, y0 + r - 3, i0[j], i1[j], g[j]);
                }
            }
#pragma unroll
            for (int j = 0; j < kPerThread; ++j) {
                const P f0 = node_value<STAGE>(a, i0[j], dt, ax, ay);
                const P f1 = node_value<STAGE>(a, i1[j], dt, ax, ay);
                val[j] = extrapolate(f0, f1, g[j]);
                if (kCenter && j * kThreads < TY * TX) {
                    // the tile's own node, clamped into the grid on a partial tile
                    const int e = element(j);
                    const int i = int(x0) + (e % TX), jj = int(y0) + (e / TX);
                    const int ic = i < a.nx ? i : int(a.nx) - 1;
                    const int jc = jj < a.ny ? jj : int(a.ny) - 1;
                    cen[j] = a.phi_n[grid_index(int(jc), int(ic), a.nx)];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < kPerThread; ++j) {
            const int e = tid + j * kThreads;
            if (e < kPlusElems) {
                int r, c;
                plus_node(e, r, c);
                phiL[r * PW + c] = val[j];
                if (kCenter && e < TY * TX) pnL[e] = cen[j];
            }
        }
    }

    // The curvature term's cross difference needs the four diagonal neighbours of the
    // tile's corner nodes, which the plus-shaped region leaves out: four threads load
    // them after the rest of the tile (any boundary; on a Dirichlet axis only held nodes
    // read them).
    template <int STAGE>
    __host__ __device__ static void load_corners(int tid, const StageArgs<T, P>& a, int64_t x0,
                                                 int64_t y0, double dt, double ax, double ay,
                                                 P* phiL) {
        if (a.ham != kHCurvature || tid >= 4) return;
        const int r = (tid & 1) ? TY + 3 : 2, c = (tid & 2) ? TX + 3 : 2;
        phiL[r * PW + c] = stage_value<STAGE>(a, x0 + c - 3, y0 + r - 3, dt, ax, ay);
    }

    // Second stage on a tile whose halo lies inside the grid, split around the step
    // plan: gather() loads phi^n and the flux records of the plus-shaped region into
    // registers; after dt and the dissipation are known, make_phi1() writes phi_1 of the
    // region to phiL (and phi^n of the tile to pnL), with the same arithmetic as
    // node_value().  Element e maps to the same node in both calls.
    static constexpr int kPlusElems = TY * TX + TY * 6 + 6 * TX;
    static constexpr int kPerThread = (kPlusElems + kThreads - 1) / kThreads;
    struct Gathered {
        P pn[kPerThread];
        Flux3<T> f[kPerThread];
    };
    __host__ __device__ static void plus_node(int e, int& r, int& c) {
        if (e < TY * TX) {
            r = e / TX + 3;
            c = e % TX + 3;
        } else if (e < TY * TX + TY * 6) {
            const int f = e - TY * TX;
            r = f % TY + 3;
            const int k = f / TY;
            c = k < 3 ? k : TX + k;
        } else {
            const int f = e - TY * TX - TY * 6;
            const int k = f / TX;
            c = f % TX + 3;
            r = k < 3 ? k : TY + k;
        }
    }
    // Rounds of the load whose elements are all the tile's own nodes (plus_node maps
    // them first): on a tile that is not partial these lie inside the grid, so an edge
    // tile indexes them directly and resolves only its halo through the boundary.
    __host__ __device__ static constexpr bool own_round(int j) {
        return (j + 1) * kThreads <= TY * TX;
    }
    __host__ __device__ static int64_t own_index(int e, const StageArgs<T, P>& a, int64_t x0,
                                                 int64_t y0) {
        return grid_index(int(y0) + e / TX, int(x0) + e % TX, a.nx);
    }
    // Tiles whose halo lies inside the grid; their loads take each element's offset from
    // the tile's origin in 32 bits (load(), gather()), which rows of at most kOffsetNx
    // nodes allow: (TY + 6) rows of 24-byte flux records stay below 2^32 bytes, and the
    // row multiply below 2^24.  Tiles of wider grids take the general path.
    static constexpr int64_t kOffsetNx = int64_t(1) << 22;
    static_assert((TY + 6) * kOffsetNx * 24 < (int64_t(1) << 32), "32-bit tile offsets");
    __host__ __device__ static bool inside(const StageArgs<T, P>& a, int64_t x0, int64_t y0) {
        return a.nx <= kOffsetNx && x0 >= 3 && y0 >= 3 && x0 + TX + 3 <= a.nx &&
               y0 + TY + 3 <= a.ny;
    }
    // Loads only, into registers (the idle threads of the last round load a valid
    // element): nothing here waits for them, so the step plan's loads, issued before,
    // and these overlap.
    // EDGE: a tile at the edge of a grid periodic in both axes, whose halo indices wrap
    // (each names one node, so the same one value per element as inside the grid).
    template <bool EDGE>
    __host__ __device__ static void gather(int tid, const StageArgs<T, P>& a, int64_t x0,
                                           int64_t y0, Gathered& g) {
        const int64_t base = (y0 - 3) * a.nx + (x0 - 3);
        const bool full = x0 + TX <= a.nx && y0 + TY <= a.ny;
#pragma unroll
        for (int j = 0; j < kPerThread; ++j) {
            const int e = tid + j * kThreads;
            int r, c;
            plus_node(e < kPlusElems ? e : kPlusElems - 1, r, c);
            if (!EDGE) {
                // a uniform base and 32-bit offsets, as in load()
                const uint32_t off = mul_u24(uint32_t(r), uint32_t(a.nx)) + uint32_t(c);
                g.pn[j] = at(a.phi_n + base, off);
                g.f[j] = at(reinterpret_cast<const Flux3<T>*>(a.flux) + base, off);
                continue;
            }
            int64_t idx;
            if (own_round(j) && full) {
                idx = own_index(e, a, x0, y0);
            } else {
                int64_t i1;
                int gg;
                ghost_pair(a, x0 + c - 3, y0 + r - 3, idx, i1, gg);
            }
            g.pn[j] = a.phi_n[idx];
            g.f[j] = reinterpret_cast<const Flux3<T>*>(a.flux)[idx];
        }
    }
    // phi_1 of the plus-shaped region into phiL and phi^n of the tile into pnL (on a
    // partial edge tile, the own nodes outside the grid get wrapped values no node uses).
    __host__ __device__ static void make_phi1(int tid, const StageArgs<T, P>& a, double dt,
                                              double ax, double ay, P* phiL, P* pnL,
                                              const Gathered& g) {
#pragma unroll
        for (int j = 0; j < kPerThread; ++j) {
            const int e = tid + j * kThreads;
            if (e < kPlusElems) {
                int r, c;
                plus_node(e, r, c);
                const Flux3<T> f = g.f[j];
                const double rr = double(f.h) - (mul_rn(ax, double(f.dx)) + mul_rn(ay, double(f.dy)));
                phiL[r * PW + c] = P(fma(-dt, rr, double(g.pn[j])));
                if (e < TY * TX) pnL[e] = g.pn[j];
            }
        }
    }

    // Phase X, t in [0, kHalf): (row, segment); phi_x^- / phi_x^+ into uL[0|1][row][x],
    // each stored as soon as the march forms it (no segment of results held in registers).
    __host__ __device__ static void sweep_x(int t, const StageArgs<T, P>& a, const P* phiL,
                                            T* uL) {
        const int row = t % TY;
        const int seg = t / TY;
        struct ToLds {
            T* base;
            __host__ __device__ void minus(int k, T v) const { base[k] = v; }
            __host__ __device__ void plus(int k, T v) const { base[TY * UW + k] = v; }
        };
        const ToLds out{uL + row * UW + seg * SX};
        if (a.scheme == kSchemeJP)
            sweep_emit<T, P, SX, kSchemeJP>(phiL + (row + 3) * PW + seg * SX, 1, a.ihx, a.ihxT,
                                            a.epsx, out);
        else
            sweep_emit<T, P, SX, kSchemeL>(phiL + (row + 3) * PW + seg * SX, 1, a.ihx, a.ihxT,
                                           a.epsx, out);
    }

    // The finish is shared by all threads: a column thread keeps phi_y^-+ of the first
    // SY/2 of its nodes in registers and stashes those of the other SY/2 in vL, where the
    // row thread of the same index picks them up after the barrier.
    static constexpr int kKeep = SY / 2;
    static constexpr int kVElems = 2 * TY * TX / 2;

    // Phase Y, t in [0, kHalf): (column, segment); phi_y^- / phi_y^+ of the kept nodes into
    // vm / vp, of the others into the stash, each as soon as the march forms it.
    __host__ __device__ static void sweep_y(int t, const StageArgs<T, P>& a, const P* phiL, T* vm,
                                            T* vp, T* vL) {
        const int col = t % TX;
        const int seg = t / TX;
        struct KeepOrStash {
            T* vm;
            T* vp;
            T* v0;
            __host__ __device__ void minus(int k, T v) const {
                if (k < kKeep) vm[k] = v; else v0[(k - kKeep) * TX] = v;
            }
            __host__ __device__ void plus(int k, T v) const {
                if (k < kKeep) vp[k] = v; else v0[kVElems / 2 + (k - kKeep) * TX] = v;
            }
        };
        const KeepOrStash out{vm, vp, vL + seg * kKeep * TX + col};
        if (a.scheme == kSchemeJP)
            sweep_emit<T, P, SY, kSchemeJP>(phiL + seg * SY * PW + col + 3, PW, a.ihy, a.ihyT,
                                            a.epsy, out);
        else
            sweep_emit<T, P, SY, kSchemeL>(phiL + seg * SY * PW + col + 3, PW, a.ihy, a.ihyT,
                                           a.epsy, out);
    }

    // After the barrier: fin(col, row, um, up, vm, vp, phi_s, phi^n) for SY/2 nodes of
    // column t % TX, with the stage input and phi^n of the node taken from LDS.  Column
    // threads (col_half) pass their registers; row threads read the stash.
    template <class Fin>
    __host__ __device__ static void finish(int t, bool col_half, const T* uL, const T* vm,
                                           const T* vp, const T* vL, const P* phiL,
                                           const P* pnL, Fin& fin) {
        fin.tileL = phiL;
        fin.pw = PW;
        const int mode = fin.mode();
        if constexpr (Fin::kTimed) {
            if (mode == kNodeTimed) {
                finish_nodes<kNodeTimed>(t, col_half, uL, vm, vp, vL, phiL, pnL, fin);
                return;
            }
        }
        if (mode == kNodeExtended)
            finish_nodes<kNodeExtended>(t, col_half, uL, vm, vp, vL, phiL, pnL, fin);
        else
            finish_nodes<kNodePlain>(t, col_half, uL, vm, vp, vL, phiL, pnL, fin);
    }
    template <int MODE, class Fin>
    __host__ __device__ static void finish_nodes(int t, bool col_half, const T* uL, const T* vm,
                                                 const T* vp, const T* vL, const P* phiL,
                                                 const P* pnL, Fin& fin) {
        // a wave's threads share seg and the half they belong to: every node row below is
        // uniform over the wave, and its global row address scalar
        const int col = t % TX;
        const int seg = uniform_int(t / TX);
        const int first = uniform_int(col_half ? 0 : kKeep);
        // the thread's LDS entries of its first node; the others lie a fixed stride further
        // (immediate offsets of the LDS reads, no address arithmetic per node)
        const int row0 = seg * SY + first;
        const T* u0 = uL + row0 * UW + col;
        const T* v0 = vL + seg * kKeep * TX + col;
        const P* s0 = phiL + (row0 + 3) * PW + col + 3;
        const P* n0 = Fin::kUsesPn ? pnL + row0 * TX + col : pnL;
#pragma unroll
        for (int j = 0; j < kKeep; ++j) {
            const T m = first == 0 ? vm[j] : v0[j * TX];   // first is uniform: a scalar test
            const T p = first == 0 ? vp[j] : v0[kVElems / 2 + j * TX];
            fin.template node<MODE>(col, row0 + j, u0[j * UW], u0[TY * UW + j * UW], m, p,
                                   s0[j * PW], Fin::kUsesPn ? n0[j * TX] : P(0));
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

    static constexpr int kCenterElems = TX;

    template <int STAGE>
    __host__ __device__ static void load(int tid, const StageArgs<T, P>& a, int64_t x0,
                                         double dt, double ax, double ay, P* phiL, P* pnL) {
        for (int c = tid; c < PW; c += kThreads)
            phiL[c] = stage_value<STAGE>(a, x0 + c - 3, 0, dt, ax, ay);
        if (STAGE == kStageMid || STAGE == kStageLast)
            for (int c = tid; c < TX; c += kThreads)
                if (x0 + c < a.nx) pnL[c] = a.phi_n[x0 + c];
    }

    __host__ __device__ static void sweep_x(int tid, const StageArgs<T, P>& a, const P* phiL,
                                            T* uL) {
        T um[S], up[S];
        if (a.scheme == kSchemeJP)
            sweep<T, P, S, kSchemeJP>(phiL + tid * S, 1, a.ihx, a.ihxT, a.epsx, um, up);
        else
            sweep<T, P, S, kSchemeL>(phiL + tid * S, 1, a.ihx, a.ihxT, a.epsx, um, up);
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
// TIMED: the launch may carry the time- and phi-dependent family (its code is compiled
// only into kernels that take it, so that it does not change the others' code).
template <int STAGE, typename T, typename P, bool TIMED>
struct Finisher {
    static constexpr bool kTimed = TIMED;
    // the second and third stages read phi^n at the node (a compile-time fact: an LDS
    // array's address may be 0, so a test of the pointer would stay in the code)
    static constexpr bool kUsesPn = STAGE == kStageMid || STAGE == kStageLast;
    const StageArgs<T, P>& a;
    int64_t x0, y0;
    int room_x, room_y;         // nodes of the grid from x0 (y0) on, capped: col < room_x
                                // and row < room_y is inside
    double dt, ax, ay;
    T axT, ayT;                 // the dissipation in the stencil precision
    T lo_u, hi_u, lo_v, hi_v;
    bool bad;
    int dim;
    const P* tileL = nullptr;   // the stage input on the tile (2-D; curvature term only)
    int pw = 0;                 // its row pitch
    T cos_wt = T(0);            // TIMED: cos(w t) at this stage's time

    __host__ __device__ Finisher(const StageArgs<T, P>& args, int64_t x0_, int64_t y0_,
                                 double dt_, double ax_, double ay_, int dim_)
        : a(args), x0(x0_), y0(y0_),
          room_x(int(args.nx - x0_ < int64_t(1) << 30 ? args.nx - x0_ : int64_t(1) << 30)),
          room_y(int(args.ny - y0_ < int64_t(1) << 30 ? args.ny - y0_ : int64_t(1) << 30)),
          dt(dt_), ax(ax_), ay(ay_), axT(T(ax_)), ayT(T(ay_)),
          lo_u(T(INFINITY)),
          hi_u(T(-INFINITY)), lo_v(T(INFINITY)), hi_v(T(-INFINITY)), bad(false), dim(dim_) {
        if (TIMED && STAGE != kStageDeriv && a.ham == kHTimed) {
            // the stages evaluate H at t_n, t_n + dt and t_n + dt/2; st[par] holds t_n for
            // the whole step (the step's new record goes to st[par ^ 1])
            const double tn = a.st[a.par].t;
            const double ts = STAGE == kStageMid ? tn + dt : STAGE == kStageLast ? tn + 0.5 * dt : tn;
            cos_wt = T(cos(a.hpD[2] * ts));
        }
    }

    // Example 3.13's curvature term N / (1 + phi_x^2 + phi_y^2) of the stage input,
    // N = (1 + phi_y^2) phi_xx - 2 phi_x phi_y phi_xy + (1 + phi_x^2) phi_yy, from central
    // differences over the node's 3 x 3 neighbourhood (differences of the stored values
    // taken in the storage precision).
    __host__ __device__ T curvature_term(int col, int row) const {
        const P* c = tileL + (row + 3) * pw + (col + 3);
        const P pc = c[0];
        const T de = T(c[1] - pc), dw = T(c[-1] - pc);
        const T dn = T(c[pw] - pc), ds = T(c[-pw] - pc);
        const T dxy = T((c[pw + 1] - c[pw - 1]) - (c[-pw + 1] - c[-pw - 1]));
        const T ihx = a.ihxT, ihy = a.ihyT;
        const T px = T(0.5) * (de - dw) * ihx, py = T(0.5) * (dn - ds) * ihy;
        const T pxx = (de + dw) * (ihx * ihx), pyy = (dn + ds) * (ihy * ihy);
        const T pxy = T(0.25) * dxy * (ihx * ihy);
        const T num = ((T(1) + py * py) * pxx - T(2) * (px * py) * pxy) + (T(1) + px * px) * pyy;
        return num / ((T(1) + px * px) + py * py);
    }

    __host__ __device__ bool held(int64_t i, int64_t j) const {
        return (a.bcx == kBcDirichlet && (i < 3 || i >= a.nx - 3)) ||
               (dim == 2 && a.bcy == kBcDirichlet && (j < 3 || j >= a.ny - 3));
    }

    // Whether a held layer or the curvature term can occur.
    __host__ __device__ bool extended() const {
        return a.bcx == kBcDirichlet ||
               (dim == 2 && (a.bcy == kBcDirichlet || a.ham == kHCurvature));
    }

    // The node variant of this launch, uniform over it: callers pick it once, outside
    // their loops over nodes.  The common case carries no test of held layers or the
    // curvature term.
    __host__ __device__ int mode() const {
        return TIMED && (a.ham == kHTimed || a.llf) ? kNodeTimed
               : extended()                          ? kNodeExtended
                                                     : kNodePlain;
    }

    __host__ __device__ void operator()(int col, int row, T um, T up, T vm, T vp, P ps, P pn_) {
        const int m = mode();
        if constexpr (TIMED) {
            if (m == kNodeTimed) {
                node<kNodeTimed>(col, row, um, up, vm, vp, ps, pn_);
                return;
            }
        }
        if (m == kNodeExtended)
            node<kNodeExtended>(col, row, um, up, vm, vp, ps, pn_);
        else
            node<kNodePlain>(col, row, um, up, vm, vp, ps, pn_);
    }

    // ps: the stage input at the node (phi_1 in the second stage, phi_2 in the third);
    // pn: phi^n at the node (second and third stages).  MODE: mode() of the launch.
    template <int MODE>
    __host__ __device__ void node(int col, int row, T um, T up, T vm, T vp, P ps, P pn_) {
        constexpr bool EXT = MODE != kNodePlain;   // held layers can occur
        const int i = int(x0) + col, j = int(y0) + row;   // sides are at most 2^30 nodes
        if (col >= room_x || row >= room_y) return;
        // the node's row in this tile starts at rbase, uniform over a wave where the row is;
        // stores address it plus the 32-bit column
        const int64_t rbase = int64_t(j) * a.nx + x0;
        const uint32_t ucol = uint32_t(col);
        if (STAGE == kStageDeriv) {
            const int64_t idx = rbase + col;
            a.dout0[idx] = double(um);
            a.dout1[idx] = double(up);
            if (dim == 2) {
                a.dout2[idx] = double(vm);
                a.dout3[idx] = double(vp);
            }
            return;
        }
        const bool hold = EXT && held(i, j);
        if (STAGE == kStagePre && hold) {
            // phi_1 = phi^n - dt (0 - 0) is phi^n exactly
            at(reinterpret_cast<Flux3<T>*>(a.flux) + rbase, ucol) = Flux3<T>{T(0), T(0), T(0)};
            return;
        }
        const T ub = T(0.5) * (up + um), vb = T(0.5) * (vp + vm);
        const T Dx = T(0.5) * (up - um), Dy = T(0.5) * (vp - vm);
        // node coordinates, for the position-dependent Hamiltonian only
        const T xn = a.ham == kHControl ? T(a.x0 + double(i) * a.dxD) : T(0);
        const T yn = a.ham == kHControl ? T(a.y0 + double(j) * a.dyD) : T(0);
        T H;
        if (MODE == kNodeTimed && a.ham == kHTimed) {
            // ps is this stage's own value at the node
            const T s = mul_rn(a.hpT[0], ub) + mul_rn(a.hpT[1], vb);
            H = mul_rn(cos_wt, s) + mul_rn(a.hpT[3], T(ps));
        } else {
            H = hamiltonian(a.ham, a.hpT, ub, vb, xn, yn);
        }
        // the curvature term enters the operator as -eps times a part of H
        if (MODE != kNodePlain && dim == 2 && a.ham == kHCurvature)
            H -= a.hpT[2] * curvature_term(col, row);
        // the dissipation: the step's global alpha, or (local LF) the max of |H_1|, |H_2|
        // over this node's own box [u-, u+] x [v-, v+]
        double lax = ax, lay = ay;
        if (MODE == kNodeTimed && a.llf)
            dissipation(a.ham, a.hpD, dim, double(fmin(um, up)), double(fmax(um, up)),
                        double(fmin(vm, vp)), double(fmax(vm, vp)), lax, lay);
        if (STAGE == kStagePre && MODE == kNodeTimed && a.llf) {
            // alpha is known here: the record holds the whole numerical Hamiltonian (the
            // second stage subtracts the global alpha times zero)
            const double r = double(H) - (mul_rn(lax, double(Dx)) + mul_rn(lay, double(Dy)));
            at(reinterpret_cast<Flux3<T>*>(a.flux) + rbase, ucol) = Flux3<T>{T(r), T(0), T(0)};
        } else if (STAGE == kStagePre) {
            at(reinterpret_cast<Flux3<T>*>(a.flux) + rbase, ucol) = Flux3<T>{H, Dx, Dy};
        }
        if (STAGE == kStagePre) {
            lo_u = fmin(lo_u, fmin(um, up));
            hi_u = fmax(hi_u, fmax(um, up));
            lo_v = fmin(lo_v, fmin(vm, vp));
            hi_v = fmax(hi_v, fmax(vm, vp));
            bad |= !(finite_t(H) && finite_t(Dx) && finite_t(Dy));
            return;
        }
        // L = -(H - (ax Dx + ay Dy)); the sum is symmetric in x and y
        const bool local = MODE == kNodeTimed && a.llf;
        const T R = H - (mul_rn(local ? T(lax) : axT, Dx) + mul_rn(local ? T(lay) : ayT, Dy));
        // The Shu-Osher combinations as explicit fused multiply-adds: every kernel
        // instantiation rounds them the same way (left to FMA contraction, the compiler
        // may fuse them differently in each)
        const double pn = double(pn_);
        const double euler = fma(-dt, double(R), double(ps));   // ps + dt L
        double res;
        if (STAGE == kStageMid) {
            res = fma(0.75, pn, 0.25 * euler);
        } else {
            res = fma(1.0 / 3.0, pn, mul_rn(2.0 / 3.0, euler));
        }
        const P outv = EXT && hold ? pn_ : P(res);
        at(a.out + rbase, ucol) = outv;
        bad |= !finite_t(outv);
    }
};

}  // namespace hjw
