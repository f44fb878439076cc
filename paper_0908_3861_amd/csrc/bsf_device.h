// Device building blocks of libbsf: double-double arithmetic, the interpolant tables,
// restart-window geometry, the on-chip pre-integrator and the localisation mesh.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "boxspline_tables.h"
#include "model_tables.h"

namespace bsf {

constexpr int kTile = 16;       // output tile edge (pixels)
constexpr int kThreads = 256;   // one output pixel per thread (per thread pair at order 3)

// Order 3 on the float32-output path shares each pixel's taps between two threads (k2
// in {0,1} and {2,3}) in workgroups of 512, so that the large order-3 windows, one
// workgroup per CU, still keep two waves per SIMD busy.  Every such tile is computed
// this way, whatever launch it lands in.  (The float64 path at order 3 needs about 500
// registers per thread and keeps one thread per pixel.)
template <int N, int PATH>
__host__ __device__ constexpr int split_of() { return (N == 3 && PATH == 1) ? 2 : 1; }
template <int N, int PATH>
__host__ __device__ constexpr int threads_of() { return kThreads * split_of<N, PATH>(); }
constexpr int kMaxWaves = 2 * kThreads / 64;
constexpr double kScaleMin = 0.5;
constexpr double kScaleMax = 1e4;

// sticky device error bits
enum : unsigned { kErrScale = 1u, kErrWindow = 2u, kErrRange = 4u };

// 1/sqrt2 as an unevaluated sum hi + lo (hi = round(1/sqrt2), lo = the rest)
constexpr double kInvSqrt2Hi = 0x1.6a09e667f3bcdp-1;
constexpr double kInvSqrt2Lo = -0x1.bdd3413b26456p-55;

// ---------------------------------------------------------------------------
// double-double (unevaluated sum of two doubles, ~106 significant bits).
// Error-free transforms: Knuth's two-sum, Dekker's fast two-sum, FMA two-product.
// ---------------------------------------------------------------------------
struct dd {
    double hi, lo;
};

__device__ __forceinline__ dd two_sum(double a, double b) {
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return {s, e};
}
__device__ __forceinline__ dd fast_two_sum(double a, double b) {  // |a| >= |b|
    double s = a + b;
    double e = b - (s - a);
    return {s, e};
}
__device__ __forceinline__ dd two_prod(double a, double b) {
    double p = a * b;
    return {p, __fma_rn(a, b, -p)};
}
__device__ __forceinline__ dd dd_add(dd a, dd b) {
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = fast_two_sum(s.hi, s.lo);
    s.lo += t.lo;
    return fast_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ dd dd_neg(dd a) { return {-a.hi, -a.lo}; }
__device__ __forceinline__ dd dd_add_d(dd a, double b) {
    dd s = two_sum(a.hi, b);
    s.lo += a.lo;
    return fast_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ dd dd_mul(dd a, dd b) {
    double p = a.hi * b.hi;
    double e = __fma_rn(a.hi, b.hi, -p);
    e = __fma_rn(a.hi, b.lo, e);
    e = __fma_rn(a.lo, b.hi, e);
    return fast_two_sum(p, e);
}
__device__ __forceinline__ dd dd_mul_d(dd a, double b) {
    double p = a.hi * b;
    double e = __fma_rn(a.hi, b, -p);
    e = __fma_rn(a.lo, b, e);
    return fast_two_sum(p, e);
}
__device__ __forceinline__ dd dd_div(dd a, dd b) {
    double q1 = a.hi / b.hi;
    dd r = dd_add(a, dd_neg(dd_mul_d(b, q1)));
    double q2 = r.hi / b.hi;
    r = dd_add(r, dd_neg(dd_mul_d(b, q2)));
    double q3 = r.hi / b.hi;
    return dd_add_d(fast_two_sum(q1, q2), q3);
}

// Compensated pair s + c (c collects the rounding errors of s).  One Horner step
// acc * x + coef costs an FMA two-product and a two-sum, and the pair keeps about twice
// the working precision (compensated Horner scheme, Graillat-Langlois-Louvet).
struct cp {
    double s, c;
};
__device__ __forceinline__ cp cp_horner(cp acc, dd x, cp coef) {
    const double p = acc.s * x.hi;
    const double pi = __fma_rn(acc.s, x.hi, -p);
    const dd t = two_sum(p, coef.s);
    const double corr = __fma_rn(acc.s, x.lo, (pi + t.lo) + coef.c);
    return {t.hi, __fma_rn(acc.c, x.hi, corr)};
}
// acc + w * v for a small integer weight w (exact as a double)
// the same step for an exact double coefficient (no low part to carry)
__device__ __forceinline__ cp cp_horner(cp acc, dd x, double coef) {
    const double p = acc.s * x.hi;
    const double pi = __fma_rn(acc.s, x.hi, -p);
    const dd t = two_sum(p, coef);
    const double corr = __fma_rn(acc.s, x.lo, pi + t.lo);
    return {t.hi, __fma_rn(acc.c, x.hi, corr)};
}
__device__ __forceinline__ cp cp_axpy(cp acc, double w, cp v) {
    const dd h = two_prod(v.s, w);
    const dd t = two_sum(acc.s, h.hi);
    return {t.hi, acc.c + ((t.lo + h.lo) + v.c * w)};
}

// ---------------------------------------------------------------------------
// Interpolant tables per order (generated, exact rationals NUM/DEN).
// ---------------------------------------------------------------------------
template <int N>
struct Tab;
template <>
struct Tab<1> {
    static constexpr int S = bsf_tables::kStencil1, M = bsf_tables::kMono1, DEG = 2;
    static constexpr bool ODD = true;  // cells centred on lattice points (anchor = round(p))
    static constexpr double DEN = bsf_tables::kDen1;
    static constexpr int SPLIT = 2, SHIFT = 32;  // int64 -> 2 exact doubles of 32 bits
    __host__ __device__ static constexpr double num(int j, int a) { return bsf_tables::kNum1[j][a]; }
    __host__ __device__ static constexpr int jx(int j) { return bsf_tables::kJ1[j][0]; }
    __host__ __device__ static constexpr int jy(int j) { return bsf_tables::kJ1[j][1]; }
    __host__ __device__ static constexpr int ma(int a) { return bsf_tables::kMonoExp1[a][0]; }
    __host__ __device__ static constexpr int mb(int a) { return bsf_tables::kMonoExp1[a][1]; }
};
template <>
struct Tab<2> {
    static constexpr int S = bsf_tables::kStencil2, M = bsf_tables::kMono2, DEG = 6;
    static constexpr bool ODD = false;  // cells centred on lattice points (anchor = round(p))
    static constexpr double DEN = bsf_tables::kDen2;
    static constexpr int SPLIT = 2, SHIFT = 32;
    __host__ __device__ static constexpr double num(int j, int a) { return bsf_tables::kNum2[j][a]; }
    __host__ __device__ static constexpr int jx(int j) { return bsf_tables::kJ2[j][0]; }
    __host__ __device__ static constexpr int jy(int j) { return bsf_tables::kJ2[j][1]; }
    __host__ __device__ static constexpr int ma(int a) { return bsf_tables::kMonoExp2[a][0]; }
    __host__ __device__ static constexpr int mb(int a) { return bsf_tables::kMonoExp2[a][1]; }
};
template <>
struct Tab<3> {
    static constexpr int S = bsf_tables::kStencil3, M = bsf_tables::kMono3, DEG = 10;
    static constexpr bool ODD = true;  // cells centred on lattice points (anchor = round(p))
    static constexpr double DEN = bsf_tables::kDen3;
    static constexpr int SPLIT = 3, SHIFT = 21;  // 21-bit parts keep every partial sum exact
    __host__ __device__ static constexpr double num(int j, int a) { return bsf_tables::kNum3[j][a]; }
    __host__ __device__ static constexpr int jx(int j) { return bsf_tables::kJ3[j][0]; }
    __host__ __device__ static constexpr int jy(int j) { return bsf_tables::kJ3[j][1]; }
    __host__ __device__ static constexpr int ma(int a) { return bsf_tables::kMonoExp3[a][0]; }
    __host__ __device__ static constexpr int mb(int a) { return bsf_tables::kMonoExp3[a][1]; }
};

// Interpolants of the continuous models of degree m = 0, 1 (Section 6, phi = beta^m x beta^m)
// for the order-1 filter, table keys 10 + m: phi * beta_b is the box spline of
// {l1^(m+2), l2, l3^(m+2), l4} (phi adds m+1 unit segments along l1 and l3), degree 2m + 4.
// Its centre (m/2 + 1, m/2 + 2) is a lattice point for even m, so its cells are centred on
// half-integer points there (anchor = floor(p)), and on lattice points for odd m.
template <>
struct Tab<10> {
    static constexpr int S = bsf_tables::kStencilM10, M = bsf_tables::kMonoM10, DEG = 4;
    static constexpr bool ODD = false;
    static constexpr double DEN = bsf_tables::kDenM10;
    static constexpr int SPLIT = 2, SHIFT = 32;
    __host__ __device__ static constexpr double num(int j, int a) { return bsf_tables::kNumM10[j][a]; }
    __host__ __device__ static constexpr int jx(int j) { return bsf_tables::kJM10[j][0]; }
    __host__ __device__ static constexpr int jy(int j) { return bsf_tables::kJM10[j][1]; }
    __host__ __device__ static constexpr int ma(int a) { return bsf_tables::kMonoExpM10[a][0]; }
    __host__ __device__ static constexpr int mb(int a) { return bsf_tables::kMonoExpM10[a][1]; }
};
template <>
struct Tab<11> {
    static constexpr int S = bsf_tables::kStencilM11, M = bsf_tables::kMonoM11, DEG = 6;
    static constexpr bool ODD = true;
    static constexpr double DEN = bsf_tables::kDenM11;
    static constexpr int SPLIT = 2, SHIFT = 32;
    __host__ __device__ static constexpr double num(int j, int a) { return bsf_tables::kNumM11[j][a]; }
    __host__ __device__ static constexpr int jx(int j) { return bsf_tables::kJM11[j][0]; }
    __host__ __device__ static constexpr int jy(int j) { return bsf_tables::kJM11[j][1]; }
    __host__ __device__ static constexpr int ma(int a) { return bsf_tables::kMonoExpM11[a][0]; }
    __host__ __device__ static constexpr int mb(int a) { return bsf_tables::kMonoExpM11[a][1]; }
};

// The table key of order n with the model of degree m (-1: phi = delta).
__host__ __device__ constexpr int table_key(int n, int m) { return m < 0 ? n : 10 + m; }
// Half-width of phi's support along each axis, (m + 1)/2 (0 for phi = delta).
template <int K>
__host__ __device__ constexpr double model_reach() { return K >= 10 ? 0.5 * (K - 10 + 1) : 0.0; }

// The reference triangle u1 >= |u2| is symmetric under u2 -> -u2 (about the cell
// centre), so stencil point j and its mirror j' = (jx, e - jy) (e = 0 odd n, 1 even n)
// carry the same polynomials up to the sign (-1)^b of the u2-power b.
// Largest B such that 2^B * max_alpha sum_j |NUM[j][alpha]| <= 2^53: when every window
// value is below 2^B in magnitude, each coefficient sum G_alpha, its products and all
// its partial sums are integers below 2^53, exact in a single double.
template <int N>
__host__ __device__ constexpr int exact_bits() {
    using T = Tab<N>;
    double l1max = 0.0;
    for (int m = 0; m < T::M; ++m) {
        double l1 = 0.0;
        for (int j = 0; j < T::S; ++j) l1 += T::num(j, m) < 0 ? -T::num(j, m) : T::num(j, m);
        l1max = l1 > l1max ? l1 : l1max;
    }
    double lim = 9007199254740992.0;  // 2^53
    int b = 0;
    double p = 1.0;
    while (p * 2.0 * l1max <= lim) {
        p *= 2.0;
        ++b;
    }
    return b;
}

template <int N>
__host__ __device__ constexpr int mirror_of(int j) {
    const int e = Tab<N>::ODD ? 0 : 1;
    for (int k = 0; k < Tab<N>::S; ++k)
        if (Tab<N>::jx(k) == Tab<N>::jx(j) && Tab<N>::jy(k) == e - Tab<N>::jy(j)) return k;
    return -1;
}
template <int N>
__host__ __device__ constexpr bool is_rep(int j) {  // representative of its mirror pair
    return 2 * Tab<N>::jy(j) >= (Tab<N>::ODD ? 0 : 1);
}

// Bounds of the stencil after the quarter turns about the cell centre (odd n: about
// the anchor; even n: about the anchor + (1/2, 1/2)).
template <int N>
__host__ __device__ constexpr int stencil_lo() {
    int lo = 0, hi = 0;
    for (int j = 0; j < Tab<N>::S; ++j) {
        lo = Tab<N>::jx(j) < lo ? Tab<N>::jx(j) : lo;
        lo = Tab<N>::jy(j) < lo ? Tab<N>::jy(j) : lo;
        hi = Tab<N>::jx(j) > hi ? Tab<N>::jx(j) : hi;
        hi = Tab<N>::jy(j) > hi ? Tab<N>::jy(j) : hi;
    }
    const int other = Tab<N>::ODD ? -hi : 1 - hi;
    return lo < other ? lo : other;
}
template <int N>
__host__ __device__ constexpr int stencil_hi() {
    return Tab<N>::ODD ? -stencil_lo<N>() : 1 - stencil_lo<N>();
}

// ---------------------------------------------------------------------------
// Restart window of an output tile.  For pixel m the taps sit at
// p = m + n*tau - x_k with p - m in [-R1 - n/2, R1 - n/2] x [-R2 - 3n/2, R2 - 3n/2],
// R1 = (n/2)(a1 + a'2 + a'4), R2 = (n/2)(a3 + a'2 + a'4); the anchor q = round(p)
// (odd n) or floor(p) (even n) and the stencil add the interpolation reach.  The
// window also holds every sample in the kernel support [m - R, m + R].
// ---------------------------------------------------------------------------
struct Window {
    int x0, y0, wq, hq;
};

// K: the interpolant's table (order N, or a continuous model of it); a model's kernel
// support reaches model_reach<K>() further along each axis.
template <int N, int K = N>
__host__ __device__ inline Window tile_window(int t1, int t2, int tw, int th, double R1, double R2) {
    const double qlo = Tab<K>::ODD ? -0.5 : -1.0, qhi = Tab<K>::ODD ? 0.5 : 0.0;
    const int jl = stencil_lo<K>(), jh = stencil_hi<K>();
    constexpr double e = model_reach<K>();
    int lx = (int)floor(-R1 - 0.5 * N + qlo) + jl, sx = (int)floor(-R1 - e);
    int hx = (int)ceil(R1 - 0.5 * N + qhi) + jh, ux = (int)ceil(R1 + e);
    int ly = (int)floor(-R2 - 1.5 * N + qlo) + jl, sy = (int)floor(-R2 - e);
    int hy = (int)ceil(R2 - 1.5 * N + qhi) + jh, uy = (int)ceil(R2 + e);
    Window w;
    w.x0 = t1 + (lx < sx ? lx : sx) - 1;
    w.y0 = t2 + (ly < sy ? ly : sy) - 1;
    const int x1 = t1 + tw - 1 + (hx > ux ? hx : ux) + 1;
    const int y1 = t2 + th - 1 + (hy > uy ? hy : uy) + 1;
    w.wq = x1 - w.x0 + 1;
    w.hq = y1 - w.y0 + 1;
    return w;
}

// elements of a window plus the right-hand extension triangle of step (4)
__host__ __device__ inline long long window_elems(const Window& w) {
    return (long long)w.hq * w.wq + (long long)w.hq * (w.hq - 1) / 2;
}

__host__ __device__ inline double reach1(int n, double a1, double a2, double a4) {
    return 0.5 * n * (a1 + (a2 + a4) * 0.70710678118654752440);
}

}  // namespace bsf
