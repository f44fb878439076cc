// Two-direction (rect) space-variant box-spline filter: Section 4, eq. def with N = 2.
//
// The box spline of scale vector (a1, a2) at angles 0 and pi/2 is the tensor product of a
// segment of length a1 along x (columns) and one of length a2 along y (rows); rect = the one
// at (1, 1).  Order n is its n-fold self-convolution, beta_a1^{n-1}(x1) beta_a2^{n-1}(x2).
// Every output pixel m is the projection of the image's continuous model
// f(x) = sum_k c[k] (beta^{n1} x beta^{n1})(x - k) onto that box spline at m's own scales
// (Section 6, with phi = beta^{n1} x beta^{n1}; n1 = -1 is phi = delta, Section 7's choice).
//
// The two steps of Section 6 with b = (1, 1), which puts the running-sum filter of eq.
// RS_filter on the lattice:
//   1. non-adaptive: g = the n-fold running sums of c along rows, then along columns (for
//      n = 1 the summed-area table);
//   2. adaptive (eq. mask): F(x) = sum_k g[k] B(x + tau - k), B = beta^D x beta^D with
//      D = n1 + n (phi convolved with the order-n box spline at b), tau = (a - 1) n / 2 per
//      axis (the shift of eq. factor), and
//      s[m] = (a1 a2)^-n sum_{j1, j2} (-1)^{j1+j2} C(n, j1) C(n, j2) F(m - (a1 j1, a2 j2)).
// The mask separates: the weights along x, d_j1 beta^D(u1(j1) - k1), are formed once per pixel
// ((n+1)(D+1) of them), and for each of the (n+1)(D+1) rows the mask reaches, the row's
// weighted sum is formed and weighted along y.
//
// Restart windows.  A workgroup owns a T x T tile and runs step 1 on a window that holds
// every sample the tile's masks reach, the running sums anchored at the window centre (each
// line's two halves, after and before the anchor, on two threads): that
// changes g by a polynomial of degree < n along each direction, which the degree-D
// interpolation reproduces and the n-th difference annihilates (same result in exact
// arithmetic, magnitudes bounded by the window instead of the image).  Both stages carry a
// compensation term (a float64 value and its rounding error): the mask cancels magnitudes of
// order (window/2)^{2n}.
//
// The degree-2 and degree-3 models first need c = f_ext * (b^{n1} x b^{n1})^{-1}: the
// one-dimensional inverse (the two-sided exponential of filter1d.h's Prefilter) along rows,
// then along columns, in two global passes over the domain the windows read.
#pragma once

namespace bsf {
namespace rect {

constexpr int kThreads = 256;

struct Args {
    // samples: the image under its border rule (SRC = 0), or the coefficient buffer (SRC = 1)
    const void* in;
    long long in_pitch;
    int dtype, border;
    const double* cbuf;  // c[(k2 - org) * cpitch + (k1 - org)], org = -left
    long long cpitch;
    const float* scales;  // (a1, a2) per pixel
    long long sc_pitch;   // in pixels
    void* out;            // float64 (path 0) or float32 (path 1)
    long long out_pitch;
    int width, height, path;
    int T, tiles_x, tiles_y;
    int left, right;      // window halos before / after a tile (both axes)
    int wx, pitch;        // window side (T + left + right) and its LDS row pitch (odd)
    float a_max;
    unsigned* err;
};

// Halos of a tile: the mask point u = x + (a-1) n/2 + (D+1)/2 - a j reads cells p - l,
// p = ceil(u) - 1, l = 0..D, over every scale in [0.5, a_max] (as the 1-D filter).
__host__ inline int halo_left(int n, int D, double a_max) {
    return (int)std::ceil((a_max + 1.0) * n * 0.5 + 0.5 * (D + 1)) + 1;
}
__host__ inline int halo_right(int n, int D, double a_max) {
    return (int)std::ceil(std::max(a_max - 1.0, 0.0) * n * 0.5 + 0.5 * (D + 1)) + 1;
}
__host__ inline int lds_pitch(int wx) { return wx | 1; }  // odd: 16-byte rows on distinct banks
__host__ inline long long lds_bytes(int T, int n, int D, double a_max) {
    const int wx = T + halo_left(n, D, a_max) + halo_right(n, D, a_max);
    return 16ll * lds_pitch(wx) * wx;
}

using f1d::cpair;
using f1d::cp_sum;

// One half of a line of the window (entries `stride` apart), n anchored running sums
// y[t] = y[t-1] + x[t] with y[anchor] = 0: the half after the anchor runs forward from it
// (back = false, positions anchor+1 .. len-1), the rest backward, y[t-1] = y[t] - x[t]
// (back = true, positions anchor .. 0).  Each fold of a half reads only that half of the
// previous fold, so the two halves are independent and run on different threads.
template <int N>
__device__ __forceinline__ void anchored_half(double2* line, int len, int stride, int anchor, bool back) {
#pragma unroll 1
    for (int fold = 0; fold < N; ++fold) {
        cpair acc = {0.0, 0.0};
        if (!back) {
            for (int t = anchor + 1; t < len; ++t) {
                const double2 x = line[t * stride];
                acc = cp_sum(acc, {x.x, x.y});
                line[t * stride] = make_double2(acc.s, acc.c);
            }
        } else {
            for (int t = anchor; t >= 0; --t) {
                const double2 x = line[t * stride];
                line[t * stride] = make_double2(acc.s, acc.c);
                acc = cp_sum(acc, {-x.x, -x.y});
            }
        }
    }
}

// w * v for a double-double weight w and a compensated value v, added to acc.
__device__ __forceinline__ cpair dd_mac(cpair acc, dd w, cpair v) {
    const dd p = two_prod(w.hi, v.s);
    const dd t = two_sum(acc.s, p.hi);
    return {t.hi, acc.c + (t.lo + __fma_rn(w.hi, v.c, __fma_rn(w.lo, v.s, p.lo)))};
}

// P_l(t) = sum_e A[l][e] t^e (D! beta^D(t + l - (D+1)/2), integer coefficients) in
// double-double, times the integer s.
template <int D>
__device__ __forceinline__ dd piece_dd(int l, double t, long long s) {
    dd acc = {0.0, 0.0};
    bool seeded = false;
#pragma unroll
    for (int e = D; e >= 0; --e) {
        const long long A = f1d::lattice_coef(D, l, e);
        if (seeded) {
            const dd p = two_prod(acc.hi, t);
            const double lo = __fma_rn(acc.lo, t, p.lo);
            const dd q = two_sum(p.hi, (double)A);
            acc = fast_two_sum(q.hi, q.lo + lo);
        } else if (A != 0) {
            acc = {(double)A, 0.0};
            seeded = true;
        }
    }
    const dd p = two_prod(acc.hi, (double)s);
    return fast_two_sum(p.hi, __fma_rn(acc.lo, (double)s, p.lo));
}

template <typename T>
__device__ __forceinline__ double sample(const Args& A, int k1, int k2) {
    const bool inside = k1 >= 0 && k1 < A.width && k2 >= 0 && k2 < A.height;
    if (A.border != 0 && !inside) return 0.0;
    const int c1 = k1 < 0 ? 0 : (k1 >= A.width ? A.width - 1 : k1);
    const int c2 = k2 < 0 ? 0 : (k2 >= A.height ? A.height - 1 : k2);
    return (double)static_cast<const T*>(A.in)[(long long)c2 * A.in_pitch + c1];
}

// One tile per workgroup (XCD-aware order), T x T outputs, threads stepping over them.
template <int N, int D, int SRC>
__global__ __launch_bounds__(kThreads) void rect_kernel(Args A) {
    extern __shared__ double2 rect_lds[];
    double2* S = rect_lds;
    const int tid = threadIdx.x;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = tile % A.tiles_x, ty = tile / A.tiles_x;
    const int X0 = tx * A.T - A.left, Y0 = ty * A.T - A.left;  // window origin
    const int wx = A.wx, P = A.pitch;
    const int nwin = wx * wx;

    // ---- the window's coefficients into LDS ----------------------------------------------
    if constexpr (SRC == 1) {
        const double* cb = A.cbuf + (long long)(Y0 + A.left) * A.cpitch + (X0 + A.left);
        for (int i = tid; i < nwin; i += kThreads) {
            const int r = i / wx, c = i - r * wx;
            S[r * P + c] = make_double2(cb[(long long)r * A.cpitch + c], 0.0);
        }
    } else {
        for (int i = tid; i < nwin; i += kThreads) {
            const int r = i / wx, c = i - r * wx;
            double v;
            if (A.dtype == 0) v = sample<unsigned char>(A, X0 + c, Y0 + r);
            else if (A.dtype == 1) v = sample<float>(A, X0 + c, Y0 + r);
            else v = sample<double>(A, X0 + c, Y0 + r);
            S[r * P + c] = make_double2(v, 0.0);
        }
    }
    __syncthreads();

    // ---- step 1: n anchored running sums along rows, then along columns ----------------------
    const int ctr = wx / 2 - 1;
    for (int h = tid; h < 2 * wx; h += kThreads) anchored_half<N>(S + (h >> 1) * P, wx, 1, ctr, h & 1);
    __syncthreads();
    for (int h = tid; h < 2 * wx; h += kThreads) anchored_half<N>(S + (h >> 1), wx, P, ctr, h & 1);
    __syncthreads();

    // ---- step 2: the separable mask at each output's own scales ------------------------------
    bool bad = false;
    constexpr int NT = (N + 1) * (D + 1);
    for (int o = tid; o < A.T * A.T; o += kThreads) {
        const int ox = o % A.T, oy = o / A.T;
        const int m1 = tx * A.T + ox, m2 = ty * A.T + oy;
        if (m1 >= A.width || m2 >= A.height) continue;
        const float2 af = *reinterpret_cast<const float2*>(A.scales + 2 * ((long long)m2 * A.sc_pitch + m1));
        const long long off = (long long)m2 * A.out_pitch + m1;
        if (!(af.x >= 0.5f && af.x <= A.a_max && af.y >= 0.5f && af.y <= A.a_max)) {  // false for NaN
            bad = true;
            if (A.path == 1) static_cast<float*>(A.out)[off] = __builtin_nanf("");
            else static_cast<double*>(A.out)[off] = __builtin_nan("");
            continue;
        }
        const double a1 = af.x, a2 = af.y;
        const double u01 = (double)(A.left + ox) + (a1 - 1.0) * (0.5 * N) + 0.5 * (D + 1);
        const double u02 = (double)(A.left + oy) + (a2 - 1.0) * (0.5 * N) + 0.5 * (D + 1);
        // weights and columns along x: d_j1 P_l(t1(j1)) at column p1(j1) - l
        dd w1[NT];
        int c1[NT];
#pragma unroll
        for (int j = 0; j <= N; ++j) {
            const double u = __fma_rn(-a1, (double)j, u01);  // exact: a1 has 24 significant bits
            const double pc = ceil(u) - 1.0;
            const double t = u - pc;
            int p = (int)pc;
            p = p < D ? D : (p > wx - 1 ? wx - 1 : p);
            const long long sgn = ((j & 1) ? -1 : 1) * f1d::binom(N, j);
#pragma unroll
            for (int l = 0; l <= D; ++l) {
                w1[j * (D + 1) + l] = piece_dd<D>(l, t, sgn);
                c1[j * (D + 1) + l] = p - l;
            }
        }
        cpair acc = {0.0, 0.0};
#pragma unroll 1
        for (int j = 0; j <= N; ++j) {
            const double u = __fma_rn(-a2, (double)j, u02);
            const double pc = ceil(u) - 1.0;
            const double t = u - pc;
            int p = (int)pc;
            p = p < D ? D : (p > wx - 1 ? wx - 1 : p);
            const long long sgn = ((j & 1) ? -1 : 1) * f1d::binom(N, j);
#pragma unroll
            for (int l = 0; l <= D; ++l) {
                const double2* row = S + (p - l) * P;
                cpair q = {0.0, 0.0};
#pragma unroll
                for (int i = 0; i < NT; ++i) {
                    const double2 v = row[c1[i]];
                    q = dd_mac(q, w1[i], {v.x, v.y});
                }
                acc = dd_mac(acc, piece_dd<D>(l, t, sgn), q);
            }
        }
        // (a1 a2)^n (D!)^2: a1 a2 is exact (48 bits); the powers and the factorial round once each
        double den = a1 * a2;
        const double base = den;
#pragma unroll
        for (int i = 1; i < N; ++i) den *= base;
        den *= (double)(f1d::factorial(D) * f1d::factorial(D));
        const double s = (acc.s + acc.c) / den;
        if (A.path == 1) static_cast<float*>(A.out)[off] = (float)s;
        else static_cast<double*>(A.out)[off] = s;
    }
    const unsigned long long bb = __ballot(bad);
    if (bb && (tid & 63) == __ffsll((long long)bb) - 1) atomicOr(A.err, kErrScale);
}

// ---- prefilter of the degree-2 and degree-3 models (two global passes) ----------------------

struct PrefArgs {
    const void* in;
    long long in_pitch;
    int dtype, border, width, height;
    double* h;        // rows pass output: rows org-K .. org+ch+K-1, columns org .. org+cw-1
    double* c;        // columns pass output: rows org .. org+ch-1
    long long pitch;  // of both (cw rounded up)
    int org, cw, ch;  // the domain c covers: k1 in [org, org + cw), k2 in [org, org + ch)
};

template <typename T>
__device__ __forceinline__ double pf_sample(const PrefArgs& A, int k1, int k2) {
    const bool inside = k1 >= 0 && k1 < A.width && k2 >= 0 && k2 < A.height;
    if (A.border != 0 && !inside) return 0.0;
    const int c1 = k1 < 0 ? 0 : (k1 >= A.width ? A.width - 1 : k1);
    const int c2 = k2 < 0 ? 0 : (k2 >= A.height ? A.height - 1 : k2);
    return (double)static_cast<const T*>(A.in)[(long long)c2 * A.in_pitch + c1];
}

// h[k2][k1] = rho sum_{|j| <= K} z^|j| f_ext[k2][k1 - j], Horner in z over the pairs.
template <int MODEL, typename T>
__device__ __forceinline__ double pf_row(const PrefArgs& A, int k1, int k2) {
    using PF = f1d::Prefilter<MODEL>;
    double acc = pf_sample<T>(A, k1 - PF::K, k2) + pf_sample<T>(A, k1 + PF::K, k2);
#pragma unroll
    for (int j = PF::K - 1; j >= 1; --j) acc = __fma_rn(acc, PF::z, pf_sample<T>(A, k1 - j, k2) + pf_sample<T>(A, k1 + j, k2));
    acc = __fma_rn(acc, PF::z, pf_sample<T>(A, k1, k2));
    return PF::rho * acc;
}

template <int MODEL>
__global__ __launch_bounds__(256) void rect_prefilter_rows(PrefArgs A) {
    using PF = f1d::Prefilter<MODEL>;
    const int rows = A.ch + 2 * PF::K;
    const long long total = (long long)rows * A.cw;
    for (long long i = blockIdx.x * 256ll + threadIdx.x; i < total; i += (long long)gridDim.x * 256) {
        const int r = (int)(i / A.cw), x = (int)(i - (long long)r * A.cw);
        const int k1 = A.org + x, k2 = A.org - PF::K + r;
        double v;
        if (A.dtype == 0) v = pf_row<MODEL, unsigned char>(A, k1, k2);
        else if (A.dtype == 1) v = pf_row<MODEL, float>(A, k1, k2);
        else v = pf_row<MODEL, double>(A, k1, k2);
        A.h[(long long)r * A.pitch + x] = v;
    }
}

template <int MODEL>
__global__ __launch_bounds__(256) void rect_prefilter_cols(PrefArgs A) {
    using PF = f1d::Prefilter<MODEL>;
    const long long total = (long long)A.ch * A.cw;
    for (long long i = blockIdx.x * 256ll + threadIdx.x; i < total; i += (long long)gridDim.x * 256) {
        const int r = (int)(i / A.cw), x = (int)(i - (long long)r * A.cw);
        const double* col = A.h + (long long)(r + PF::K) * A.pitch + x;  // h at this row
        double acc = col[-(long long)PF::K * A.pitch] + col[(long long)PF::K * A.pitch];
#pragma unroll
        for (int j = PF::K - 1; j >= 1; --j) acc = __fma_rn(acc, PF::z, col[-(long long)j * A.pitch] + col[(long long)j * A.pitch]);
        acc = __fma_rn(acc, PF::z, col[0]);
        A.c[(long long)r * A.pitch + x] = PF::rho * acc;
    }
}

}  // namespace rect
}  // namespace bsf
