// One-dimensional scale-adaptive filter (Section 3, Proposition 3.1) for batches of signals.
//
// Every output sample m is the projection of the signal's continuous model onto the
// B-spline of degree n-1 and scale a[m] centred at m.  The model is
// f(x) = sum_k c[k] beta^{n1}(x - k) with n1 in {-1, 0, 1, 2, 3} (n1 = -1: impulses at the
// samples; n1 = 0, 1: the interpolation filter is the unit impulse, c = f; n1 = 2, 3: c is the
// extended signal filtered by the inverse of b^{n1}[k] = beta^{n1}(k), the model interpolating
// the samples).  Proposition 3.1 computes it in two steps:
//   1. non-adaptive: g = n-fold running sum of c (the filter u_1^n, eq. RS with b = 1);
//   2. adaptive: F(x) = sum_k g[k] beta^D(x + tau - k) with D = n1 + n, tau = (a-1) n / 2,
//      and s[m] = Delta_a^n F(m) = a^-n sum_j (-1)^j C(n,j) F(m - a j) (eq. FD).
//
// Layout of the work.  A workgroup owns kT = 256 consecutive outputs of one signal and runs step 1
// on a restart window that holds every sample their masks reach: the running sums start from
// zero at the window's left edge, which changes g there by a polynomial of degree n-1; the
// degree-D interpolation reproduces it and the n-th difference annihilates it, so the result
// is the same in exact arithmetic, and the magnitudes the mask cancels stay bounded by the
// window length instead of the signal's.  One wave runs the sums, each lane on a contiguous
// chunk of the window in LDS, with the chunk totals combined across the wave.
// The interpolant of F on the cell (p-1, p] is a polynomial in t = x + tau + (D+1)/2 - p:
//   F = sum_e t^e G_e[p],   D! G_e[p] = sum_{l=0}^{D} A[l][e] g[p - l],
// with integer A (the piece of beta^D on [l, l+1], times D!).  The workgroup tabulates
// G_0..G_D for every window position in LDS once; each output then needs n+1 table reads and
// n+1 Horner evaluations.  All sums carry a compensation term (a float64 value plus its
// rounding error), since the mask cancels magnitudes of order (window length)^n.
#pragma once

namespace bsf {
namespace f1d {

constexpr int kThreads = 256;
constexpr int kPerThread = 1;
constexpr int kT = kThreads * kPerThread;  // outputs per workgroup
constexpr int kWindowMax = 4096;           // longest restart window

__host__ __device__ constexpr long long ipow(long long b, int e) {
    long long r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}
__host__ __device__ constexpr long long binom(int n, int k) {
    long long r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}
__host__ __device__ constexpr long long factorial(int n) { return n <= 1 ? 1 : n * factorial(n - 1); }

// D! times the coefficient of t^e in beta^D(t + l - (D+1)/2), t in (0, 1]: from the
// truncated-power form of the B-spline, only the terms i <= l are active on that piece.
__host__ __device__ constexpr long long lattice_coef(int D, int l, int e) {
    long long s = 0;
    for (int i = 0; i <= l; ++i) s += ((i & 1) ? -1 : 1) * binom(D + 1, i) * ipow(l - i, D - e);
    return binom(D, e) * s;
}

// Window geometry for outputs [m0, m0 + kT) with every scale in [0.5, a_max]: the window
// starts at m0 - left and holds W samples.  Cell index p = ceil(u) - 1 of the mask point
// u = (m - P) + tau + (D+1)/2 - a j runs over [D, W - 1].
__host__ inline int window_left(int n, int D, double a_max) {
    return (int)std::ceil((a_max + 1.0) * n * 0.5 + 0.5 * (D + 1)) + 1;
}
__host__ inline int window_len(int n, int D, double a_max) {
    const int right = (int)std::ceil(std::max(a_max - 1.0, 0.0) * n * 0.5 + 0.5 * (D + 1)) + 1;
    return kT + window_left(n, D, a_max) + right;
}
// LDS of a workgroup: the running sums (a pair per position), then the interpolant tables:
// D+1 pairs per position on the float64 path, D+1 doubles on the float32-output path.
__host__ inline long long lds_bytes(int D, int W, int path) {
    return 16ll * W + (path == 0 ? 16ll : 8ll) * W * (D + 1);
}

// The prefilter of the degree-2 and degree-3 models (Section 3, c = f * (b^{n1})^{-1}): the
// inverse of the symmetric filter (b1, b0, b1) is the two-sided exponential rho z^|k|, with
// z the root of b1 z^2 + b0 z + b1 inside the unit circle and rho = 1 / (b1 (z - 1/z)):
// z = 2 sqrt2 - 3, rho = sqrt2 for degree 2; z = sqrt3 - 2, rho = sqrt3 for degree 3.  It is
// truncated at |k| <= K: the dropped tail is at most 2 rho |z|^(K+1) / (1 - |z|) of max |f|,
// below 2^-60 for K = 24 (degree 2) and K = 32 (degree 3).
template <int M>
struct Prefilter {
    static constexpr int K = 0;
};
template <>
struct Prefilter<2> {
    static constexpr int K = 24;
    static constexpr double z = -0.1715728752538099, rho = 1.4142135623730951;
};
template <>
struct Prefilter<3> {
    static constexpr int K = 32;
    static constexpr double z = -0.2679491924311227, rho = 1.7320508075688772;
};

struct cpair {
    double s, c;
};
__device__ __forceinline__ cpair cp_sum(cpair a, cpair b) {
    const dd t = two_sum(a.s, b.s);
    return {t.hi, (a.c + b.c) + t.lo};
}
// acc * t + coef for an exact double t (compensated Horner step)
__device__ __forceinline__ cpair cp_fma(cpair acc, double t, cpair coef) {
    const double p = acc.s * t;
    const double pe = __fma_rn(acc.s, t, -p);
    const dd q = two_sum(p, coef.s);
    return {q.hi, __fma_rn(acc.c, t, (pe + q.lo) + coef.c)};
}
// acc + w * v for a small integer w
__device__ __forceinline__ cpair cp_axpy_i(cpair acc, double w, cpair v) {
    const dd h = two_prod(v.s, w);
    const dd t = two_sum(acc.s, h.hi);
    return {t.hi, acc.c + ((t.lo + h.lo) + v.c * w)};
}
// A pair moved across lanes by a DPP control (lanes without a source, or outside the row
// mask, receive zero: bound_ctrl, and zero as the kept value).
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_f64(double v) {
    unsigned long long b;
    __builtin_memcpy(&b, &v, 8);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROWMASK, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROWMASK, 0xf, true);
    b = ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
    double r;
    __builtin_memcpy(&r, &b, 8);
    return r;
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ cpair dpp_cp(cpair v) {
    return {dpp_f64<CTRL, ROWMASK>(v.s), dpp_f64<CTRL, ROWMASK>(v.c)};
}
// Inclusive compensated prefix sum over the wave's 64 lanes at register speed: shifts by 1, 2,
// 4, 8 within each row of 16 lanes, then the broadcasts of lanes 15 and 31 into the rows above
// (a lane adding a zero pair keeps its value exactly).
__device__ __forceinline__ cpair wave_scan_cp(cpair v) {
    v = cp_sum(dpp_cp<0x111, 0xf>(v), v);  // row_shr:1
    v = cp_sum(dpp_cp<0x112, 0xf>(v), v);  // row_shr:2
    v = cp_sum(dpp_cp<0x114, 0xf>(v), v);  // row_shr:4
    v = cp_sum(dpp_cp<0x118, 0xf>(v), v);  // row_shr:8
    v = cp_sum(dpp_cp<0x142, 0xa>(v), v);  // row_bcast:15 into rows 1 and 3
    v = cp_sum(dpp_cp<0x143, 0xc>(v), v);  // row_bcast:31 into rows 2 and 3
    return v;
}
// The pair of a wave-uniform lane l.
__device__ __forceinline__ double lane_f64(double v, int l) {
    unsigned long long b;
    __builtin_memcpy(&b, &v, 8);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    b = ((unsigned long long)hi << 32) | lo;
    double r;
    __builtin_memcpy(&r, &b, 8);
    return r;
}

struct Args {
    const void* in;
    long long in_pitch;
    const float* scales;
    long long sc_pitch;
    void* out;  // float64 (path 0) or float32 (path 1)
    long long out_pitch;
    int length, tiles, dtype, border, left, W;
    float a_max;
    unsigned* err;
};

// acc + w * v for an integer weight w known at compile time after unrolling: powers of two
// (the common case, +-1 and +-2) scale exactly and need no two-product.
__device__ __forceinline__ bool pow2_weight(long long w) {
    const long long a = w < 0 ? -w : w;
    return a != 0 && (a & (a - 1)) == 0;
}
__device__ __forceinline__ cpair cp_add_weighted(cpair acc, long long w, cpair v) {
    if (pow2_weight(w)) return cp_sum(acc, {v.s * (double)w, v.c * (double)w});
    return cp_axpy_i(acc, (double)w, v);
}
// w * v as the first term of a sum
__device__ __forceinline__ cpair cp_weighted(long long w, cpair v) {
    if (pow2_weight(w)) return {v.s * (double)w, v.c * (double)w};
    const dd h = two_prod(v.s, (double)w);
    return {h.hi, h.lo + v.c * (double)w};
}

// The extended samples f_ext[P + idx], idx = 0 .. count-1, handed to put(idx, value).
template <typename T, typename Put>
__device__ __forceinline__ void load_window(const Args& A, const T* row, int P, int count, Put put) {
    const int L = A.length;
    const bool zero_border = A.border != 0;
    // four samples per thread in flight at a time
    for (int base = threadIdx.x; base < count; base += 4 * kThreads) {
        double x[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int idx = base + r * kThreads;
            const int k = P + idx;
            const bool inside = k >= 0 && k < L;
            const int kc = k < 0 ? 0 : (k >= L ? L - 1 : k);
            x[r] = (idx < count && !(zero_border && !inside)) ? (double)row[kc] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int idx = base + r * kThreads;
            if (idx < count) put(idx, x[r]);
        }
    }
}

template <typename Put>
__device__ __forceinline__ void load_any(const Args& A, int b, int P, int count, Put put) {
    const long long off = (long long)b * A.in_pitch;
    if (A.dtype == 0) load_window(A, static_cast<const unsigned char*>(A.in) + off, P, count, put);
    else if (A.dtype == 1) load_window(A, static_cast<const float*>(A.in) + off, P, count, put);
    else load_window(A, static_cast<const double*>(A.in) + off, P, count, put);
}

// PATH 0: float64 output, every step compensated.  PATH 1: float32 output; the running sums
// stay compensated (they carry the largest magnitudes), the tables and the mask are plain
// float64 (their rounding errors are of order 2^-53 of the sums, far below float32).
template <int N, int D, int PATH>
__global__ __launch_bounds__(kThreads) void filter1d_kernel(Args A) {
    extern __shared__ double4 f1d_lds[];
    const int W = A.W;
    double2* gbuf = reinterpret_cast<double2*>(f1d_lds);  // [W] samples, then running sums
    double2* tab = gbuf + W;                               // PATH 0: [D+1][W] (s, c) of G_e
    double* tabd = reinterpret_cast<double*>(gbuf + W);    // PATH 1: [D+1][W] G_e

    const int tid = threadIdx.x, lane = tid & 63;
    const int b = blockIdx.x / A.tiles;
    const int tile = blockIdx.x - b * A.tiles;
    const int m0 = tile * kT;
    const int P = m0 - A.left;  // signal index of window position 0
    const int L = A.length;

    // the outputs' scales, fetched first so that their latency overlaps step 1
    float af[kPerThread];
#pragma unroll
    for (int q = 0; q < kPerThread; ++q) {
        const int m = m0 + tid + q * kThreads;
        af[q] = m < L ? A.scales[(long long)b * A.sc_pitch + m] : 1.0f;
    }

    // ---- the window's coefficients c, coalesced, into LDS -----------------------------------
    constexpr int MODEL = D - N;
    if constexpr (MODEL >= 2) {
        // c = f_ext * (b^{MODEL})^{-1} on the window: the extended samples of the window and K
        // more on each side go to the table area (free until the tables are built), then every
        // position sums its truncated two-sided exponential, Horner in z over the pairs
        // f[k-j] + f[k+j] (the terms shrink geometrically, so the sum is accurate to a few ulps).
        using PF = Prefilter<MODEL>;
        double* fx = reinterpret_cast<double*>(gbuf + W);
        load_any(A, b, P - PF::K, W + 2 * PF::K, [&](int idx, double v) { fx[idx] = v; });
        __syncthreads();
        for (int idx = tid; idx < W; idx += kThreads) {
            const double* f0 = fx + idx + PF::K;  // f_ext at this position
            double acc = f0[-PF::K] + f0[PF::K];
#pragma unroll
            for (int j = PF::K - 1; j >= 1; --j) acc = __fma_rn(acc, PF::z, f0[-j] + f0[j]);
            acc = __fma_rn(acc, PF::z, f0[0]);
            gbuf[idx] = make_double2(PF::rho * acc, 0.0);
        }
    } else {
        load_any(A, b, P, W, [&](int idx, double v) { gbuf[idx] = make_double2(v, 0.0); });
    }
    __syncthreads();

    // ---- step 1: n running sums over the window, by one wave --------------------------------
    // Lane i owns the chunk [i C, i C + C) (C odd: 16-byte LDS accesses at an odd multiple of
    // 16 bytes apart do not collide).  Each pass scans its chunk, then adds the exclusive
    // prefix of the chunk totals; the prefix of fold k is added while fold k+1 scans.
    // The wave that runs them rotates with the workgroup index: the waves of a workgroup are
    // spread over the CU's four SIMDs in the same order for every workgroup, and the sums are
    // the longest phase, so a fixed choice would load one SIMD with every workgroup's sums.
    if ((tid >> 6) == (int)(blockIdx.x & 3)) {
        const int C = ((W + 63) / 64) | 1;
        const int lo = lane * C < W ? lane * C : W;
        const int hi = lo + C < W ? lo + C : W;
        cpair pre = {0.0, 0.0};
#pragma unroll 1
        for (int fold = 0; fold < N; ++fold) {
            cpair s = {0.0, 0.0};
            // four elements per batch: their LDS reads are in flight together
            for (int i0 = lo; i0 < hi; i0 += 4) {
                double2 x[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) x[r] = i0 + r < hi ? gbuf[i0 + r] : make_double2(0.0, 0.0);
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (i0 + r < hi) {
                        // finish the previous fold (its prefix), then scan this one
                        s = cp_sum(s, fold == 0 ? cpair{x[r].x, 0.0} : cp_sum(pre, {x[r].x, x[r].y}));
                        gbuf[i0 + r] = make_double2(s.s, s.c);
                    }
                }
            }
            const cpair tot = wave_scan_cp(s);
            pre = dpp_cp<0x138, 0xf>(tot);  // wave_shr:1, lane 0 receives zero
            // Anchor this fold at the window centre: subtract its value at position ctr (the
            // owner lane's prefix plus its local sum there) from every prefix.  The later folds
            // turn that constant into a polynomial of degree < n, which the mask annihilates;
            // the sums the mask cancels shrink by about 2^n.
            const int ctr = W / 2 - 1;
            const double2 xc = gbuf[ctr];
            const cpair owner_pre = {lane_f64(pre.s, ctr / C), lane_f64(pre.c, ctr / C)};
            const cpair anchor = cp_sum(owner_pre, {xc.x, xc.y});
            pre = cp_sum(pre, {-anchor.s, -anchor.c});
        }
        for (int i = lo; i < hi; ++i) {
            const double2 x = gbuf[i];
            const cpair g = cp_sum(pre, {x.x, x.y});
            gbuf[i] = make_double2(g.s, g.c);
        }
    }
    __syncthreads();

    // ---- lattice tables G_e[p] = sum_l A[l][e] g[p - l] (the 1/D! is applied last) ---------
    if (PATH == 1) {
        for (int p = tid + D; p < W; p += kThreads) {
            double g[D + 1];
#pragma unroll
            for (int l = 0; l <= D; ++l) {
                const double2 x = gbuf[p - l];
                g[l] = x.x + x.y;
            }
#pragma unroll
            for (int e = 0; e <= D; ++e) {
                double G = 0.0;
#pragma unroll
                for (int l = 0; l <= D; ++l) {
                    const long long w = lattice_coef(D, l, e);
                    if (w != 0) G = __fma_rn((double)w, g[l], G);
                }
                tabd[e * W + p] = G;
            }
        }
    } else {
#pragma unroll 2
        for (int p = tid + D; p < W; p += kThreads) {
            cpair G[D + 1];
            bool seeded[D + 1];
#pragma unroll
            for (int e = 0; e <= D; ++e) {
                G[e] = {0.0, 0.0};
                seeded[e] = false;
            }
#pragma unroll
            for (int l = 0; l <= D; ++l) {
                const double2 x = gbuf[p - l];
                const cpair gl = {x.x, x.y};
#pragma unroll
                for (int e = 0; e <= D; ++e) {
                    const long long w = lattice_coef(D, l, e);
                    if (w == 0) continue;
                    G[e] = seeded[e] ? cp_add_weighted(G[e], w, gl) : cp_weighted(w, gl);
                    seeded[e] = true;
                }
            }
#pragma unroll
            for (int e = 0; e <= D; ++e) tab[e * W + p] = make_double2(G[e].s, G[e].c);
        }
    }
    __syncthreads();

    // ---- step 2: the finite-difference mask at each output's own scale ----------------------
    bool bad = false;
#pragma unroll
    for (int q = 0; q < kPerThread; ++q) {
        const int m = m0 + tid + q * kThreads;
        if (m >= L) continue;
        const long long o = (long long)b * A.out_pitch + m;
        if (!(af[q] >= 0.5f && af[q] <= A.a_max)) {  // false for NaN
            bad = true;
            if (PATH == 1) static_cast<float*>(A.out)[o] = __builtin_nanf("");
            else static_cast<double*>(A.out)[o] = __builtin_nan("");
            continue;
        }
        const double a = af[q];
        const double u0 = (double)(m - P) + (a - 1.0) * (0.5 * N) + 0.5 * (D + 1);
        // a^n D!: a^2 is exact (48 bits), a^3 and the factorial round once each
        double den = a;
#pragma unroll
        for (int i = 1; i < N; ++i) den *= a;
        den *= (double)factorial(D);
        if (PATH == 1) {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j <= N; ++j) {
                const double u = __fma_rn(-a, (double)j, u0);
                const double pc = ceil(u) - 1.0;
                const double t = u - pc;
                int p = (int)pc;
                p = p < D ? D : (p > W - 1 ? W - 1 : p);
                double val = tabd[D * W + p];
#pragma unroll
                for (int e = D - 1; e >= 0; --e) val = __fma_rn(val, t, tabd[e * W + p]);
                acc = j == 0 ? val : __fma_rn((double)(((j & 1) ? -1 : 1) * binom(N, j)), val, acc);
            }
            static_cast<float*>(A.out)[o] = (float)(acc / den);
            continue;
        }
        cpair acc = {0.0, 0.0};
#pragma unroll
        for (int j = 0; j <= N; ++j) {
            const double u = __fma_rn(-a, (double)j, u0);  // exact: a has 24 significant bits
            const double pc = ceil(u) - 1.0;
            const double t = u - pc;      // in (0, 1]
            int p = (int)pc;
            p = p < D ? D : (p > W - 1 ? W - 1 : p);
            double2 x = tab[D * W + p];
            cpair val = {x.x, x.y};
#pragma unroll
            for (int e = D - 1; e >= 0; --e) {
                x = tab[e * W + p];
                val = cp_fma(val, t, {x.x, x.y});
            }
            acc = j == 0 ? val : cp_add_weighted(acc, ((j & 1) ? -1 : 1) * binom(N, j), val);
        }
        static_cast<double*>(A.out)[o] = (acc.s + acc.c) / den;
    }
    const unsigned long long bb = __ballot(bad);
    if (bb && lane == __ffsll((long long)bb) - 1) atomicOr(A.err, kErrScale);
}

}  // namespace f1d
}  // namespace bsf
