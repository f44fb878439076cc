// libbsf: hand-written gfx950 kernels and the C ABI declared in include/bsf.h.
//
// One workgroup filters one 16x16 output tile:
//   1. it reads the tile's scale vectors and sizes a restart window that holds the
//      support of every pixel of the tile (local reach, not the image-wide maximum);
//   2. it loads the window (boundary rule applied) into LDS as exact int64 samples;
//   3. stage 1 (Section 7, eq. RS): n-fold running sums along (1,0), (1,1), (0,1),
//      (-1,1) on the window plus the right-hand triangle that step (4) reads;
//   4. stage 2 (eq. final_eqn, generalised to order n): each thread evaluates its
//      pixel's (n+1)^4 finite-difference taps, interpolating the pre-integrated
//      window with the lattice box spline.
#include <hip/hip_runtime.h>
#include <type_traits>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bsf.h"
#include "bsf_device.h"
#include "filter1d.h"
#include "plan.h"
#include "rep3_groups.h"

namespace bsf {

// One filter job (an image, its scale field, order, path and output).
struct JobDesc {
    const void* in;
    long long in_pitch;
    const float* scales;
    long long scale_pitch;
    void* out;
    long long out_pitch;
    int width, height;
    int in_dtype;
    int border;
    int order, path;
    int tiles_x, tiles_y;
    long long item_base;  // first work item of this job in a batched launch
    unsigned* err;        // sticky error bits of this job (a context's word, or a plan's per-job word)
};

// Launch-wide parameters.
struct Launch {
    long long lds_cap;    // int64 elements a window may use (dynamic LDS, or a scratch slice)
    unsigned long long* stats;  // [0] pixels of the float64 path evaluated split, [1] of
                                //   those evaluated again compensated (null: not counted)
    unsigned* push_count; // tiles whose window does not fit go to this list for a later,
    int2* push_list;      //   larger launch: (job, tile); push_cap = 0 flags them instead
    int push_cap;
    // test aid: dump one tile's pre-integrated window instead of filtering
    long long* dbg_window;
    int* dbg_geom;
    long long dbg_cap;
};

// XCD-aware order: consecutive workgroup ids are dealt round-robin to the 8 XCDs, so
// hand each XCD a contiguous band of tiles (neighbouring windows share their halos in
// that XCD's L2).
__device__ __forceinline__ int xcd_tile(int wg, int nwg) {
    const int per = nwg / 8;
    if (wg >= per * 8) return wg;
    return (wg % 8) * per + wg / 8;
}

// ---------------------------------------------------------------------------
// LDS window: the (wq x hq) box row-major at 0, the extension triangle after it
// (row r holds hq-1-r extra columns to the right of the box).
// ---------------------------------------------------------------------------
struct Geo {
    int wq, hq, qn;
};

__device__ __forceinline__ int waddr(const Geo& g, int r, int c) {
    return c < g.wq ? r * g.wq + c : g.qn + r * (g.hq - 1) - ((r * (r - 1)) >> 1) + (c - g.wq);
}

__device__ __forceinline__ long long add_ovf(long long a, long long b, unsigned& ovf) {
    long long s = (long long)((unsigned long long)a + (unsigned long long)b);
    ovf |= (unsigned)(((a ^ s) & (b ^ s)) < 0);
    return s;
}
__device__ __forceinline__ long long sub_ovf(long long a, long long b, unsigned& ovf) {
    long long s = (long long)((unsigned long long)a - (unsigned long long)b);
    ovf |= (unsigned)(((a ^ b) & (a ^ s)) < 0);
    return s;
}
// float64 running sums (the float32-output path): rounded, no range check
__device__ __forceinline__ double add_ovf(double a, double b, unsigned&) { return a + b; }
__device__ __forceinline__ double sub_ovf(double a, double b, unsigned&) { return a - b; }

// Walks one line of the window point by point, keeping the LDS address up to date:
// (r, c) moves by (dr, dc) with dr in {-1, 0, 1}; the box is row-major, triangle row r
// starts at T(r) = qn + r (hq - 1) - r (r - 1) / 2 and holds columns wq.. of that row.
struct LineWalk {
    int r, c, rowbase, tr, a;
};
__device__ __forceinline__ LineWalk walk_at(const Geo& g, int r, int c) {
    LineWalk w;
    w.r = r;
    w.c = c;
    w.rowbase = r * g.wq;
    w.tr = g.qn + r * (g.hq - 1) - ((r * (r - 1)) >> 1);
    w.a = c < g.wq ? w.rowbase + c : w.tr + (c - g.wq);
    return w;
}
template <int DR, int DC>
__device__ __forceinline__ void walk_step(const Geo& g, LineWalk& w, int sgn) {  // sgn = +1 forward, -1 back
    const int dr = DR * sgn, dc = DC * sgn;
    if (dr > 0) w.tr += g.hq - 1 - w.r;
    w.r += dr;
    if (dr < 0) w.tr -= g.hq - 1 - w.r;
    w.rowbase += dr * g.wq;
    w.c += dc;
    w.a = w.c < g.wq ? w.rowbase + w.c : w.tr + (w.c - g.wq);
}

// The n-fold running sum (n = NF) of one line of the window, points (r0, c0) + t (dr, dc),
// t < len, in one pass with n running states.  tref < 0: y_k[t] = sum_{s <= t} y_{k-1}[s]
// (zero initial condition at the line's start, as in the paper's recursions).  tref >=
// 0: the same recursions anchored at y_k[tref] = 0; they differ from the former by a
// polynomial of degree < n along the line, which the mesh's n-fold finite difference along
// that direction cancels, and they keep the integers small near the tile centre.  An
// anchored line is two independent recursions -- forward from tref (part 0) and backward
// from it (part 1, which also zeroes tref) -- run by different threads.  CHECK: detect
// int64 overflow (the recursions wrap modulo 2^64 either way).  B: loads in flight per
// thread (more for a window in global memory, whose latency they hide).
template <int NF, bool CHECK, int DR, int DC, int B, typename V>
__device__ void scan_line_n(V* S, const Geo& g, int r0, int c0, int len, int tref, int part, unsigned& ovf) {
    V y[NF];
#pragma unroll
    for (int k = 0; k < NF; ++k) y[k] = 0;
    auto add = [&](V a, V b) -> V {
        if constexpr (CHECK) return add_ovf(a, b, ovf);
        else return a + b;
    };
    auto sub = [&](V a, V b) -> V {
        if constexpr (CHECK) return sub_ovf(a, b, ovf);
        else return a - b;
    };
    if (part == 0) {  // forward: y_1 += x, y_k += y_{k-1}
        int t = tref + 1;
        if (t >= len) return;
        LineWalk w = walk_at(g, r0 + t * DR, c0 + t * DC);
        for (; t + B <= len; t += B) {
            int ad[B];
            V v[B];
#pragma unroll
            for (int i = 0; i < B; ++i) {
                ad[i] = w.a;
                walk_step<DR, DC>(g, w, 1);
            }
#pragma unroll
            for (int i = 0; i < B; ++i) v[i] = S[ad[i]];
#pragma unroll
            for (int i = 0; i < B; ++i) {
                y[0] = add(y[0], v[i]);
#pragma unroll
                for (int k = 1; k < NF; ++k) y[k] = add(y[k], y[k - 1]);
                S[ad[i]] = y[NF - 1];
            }
        }
        for (; t < len; ++t) {
            y[0] = add(y[0], S[w.a]);
#pragma unroll
            for (int k = 1; k < NF; ++k) y[k] = add(y[k], y[k - 1]);
            S[w.a] = y[NF - 1];
            walk_step<DR, DC>(g, w, 1);
        }
    } else {  // backward from tref: y_k[t] = y_k[t+1] - y_{k-1}[t+1], y_0 = x
        LineWalk w = walk_at(g, r0 + tref * DR, c0 + tref * DC);
        const int aref = w.a;
        V prev = S[aref];
        int t = tref - 1;
        walk_step<DR, DC>(g, w, -1);
        for (; t - B + 1 >= 0; t -= B) {
            int ad[B];
            V v[B];
#pragma unroll
            for (int i = 0; i < B; ++i) {
                ad[i] = w.a;
                walk_step<DR, DC>(g, w, -1);
            }
#pragma unroll
            for (int i = 0; i < B; ++i) v[i] = S[ad[i]];
#pragma unroll
            for (int i = 0; i < B; ++i) {
#pragma unroll
                for (int k = NF - 1; k > 0; --k) y[k] = sub(y[k], y[k - 1]);
                y[0] = sub(y[0], prev);
                prev = v[i];
                S[ad[i]] = y[NF - 1];
            }
        }
        for (; t >= 0; --t) {
#pragma unroll
            for (int k = NF - 1; k > 0; --k) y[k] = sub(y[k], y[k - 1]);
            y[0] = sub(y[0], prev);
            prev = S[w.a];
            S[w.a] = y[NF - 1];
            walk_step<DR, DC>(g, w, -1);
        }
        S[aref] = 0;
    }
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Stage 1 on the window (eq. RS steps (1)-(4), n folds each, fused into one pass per
// direction).  cen: anchor every line at the tile centre (cc, rc) instead of at its start.
// rows_done: step (1) has already run (load_rows_runsum).
template <int NF, bool CHECK, int B, typename V>
__device__ void preintegrate_window_n(V* S, const Geo& g, bool cen, int cc, int rc, unsigned& ovf,
                                      bool rows_done = false) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int W = g.wq, H = g.hq, Wt = W + H - 1;
    const int parts = cen ? 2 : 1;
    if (!rows_done) {
        for (int it = tid; it < H * parts; it += nt) {  // (1) along (1,0): rows
            const int part = it >= H, r = it - part * H;
            scan_line_n<NF, CHECK, 0, 1, B>(S, g, r, 0, Wt - r, cen ? clampi(cc, 0, Wt - r - 1) : -1, part, ovf);
        }
        __syncthreads();
    }
    const int nd = Wt + H - 1;
    for (int it = tid; it < nd * parts; it += nt) {  // (2) along (1,1): diagonals c - r = e
        const int part = it >= nd, i = it - part * nd;
        const int e = i - (H - 1);
        const int rs = e < 0 ? -e : 0;
        const int re = std::min(H - 1, (W + H - 2 - e) >> 1);
        const int len = re - rs + 1;
        scan_line_n<NF, CHECK, 1, 1, B>(S, g, rs, e + rs, len, cen ? clampi(rc - rs, 0, len - 1) : -1, part, ovf);
    }
    __syncthreads();
    for (int it = tid; it < Wt * parts; it += nt) {  // (3) along (0,1): columns
        const int part = it >= Wt, c = it - part * Wt;
        const int len = std::min(H, Wt - c);
        scan_line_n<NF, CHECK, 1, 0, B>(S, g, 0, c, len, cen ? clampi(rc, 0, len - 1) : -1, part, ovf);
    }
    __syncthreads();
    for (int it = tid; it < Wt * parts; it += nt) {  // (4) along (-1,1): anti-diagonals c + r = e, read down-right
        const int part = it >= Wt, e = it - part * Wt;
        const int len = std::min(H, e + 1);
        scan_line_n<NF, CHECK, 1, -1, B>(S, g, 0, e, len, cen ? clampi(rc, 0, len - 1) : -1, part, ovf);
    }
    __syncthreads();
}

// binom(m + n - 1, n) as a double: the largest n-fold running sum of a line of m values
// of magnitude at most 1
__device__ __forceinline__ double fold_gain(int m, int n) {
    double r = 1.0;
    for (int i = 0; i < n; ++i) r = r * (double)(m + i) / (double)(i + 1);
    return r;
}

// Whether int64 overflow is possible in stage 1: with |x| < 2^bits, every value of every
// recursion is below 2^bits * gain(Wt) * gain(hq)^3 (rows are at most Wt = wq + hq - 1
// long, the other lines at most hq).
template <int N>
__device__ __forceinline__ bool stage1_needs_check(const Geo& g, int bits) {
    const double h = fold_gain(g.hq, N);
    return !(ldexp(1.0, bits) * fold_gain(g.wq + g.hq - 1, N) * h * h * h < 0x1p62);
}

// Stage 1 with the overflow checks only where the bound above does not exclude overflow.
template <int N, int B = 8, typename V>
__device__ void preintegrate_window(V* S, const Geo& g, bool cen, int cc, int rc, int bits, unsigned& ovf) {
    bool check = false;
    if constexpr (std::is_integral<V>::value) check = stage1_needs_check<N>(g, bits);
    if (check) preintegrate_window_n<N, true, B>(S, g, cen, cc, rc, ovf);
    else preintegrate_window_n<N, false, B>(S, g, cen, cc, rc, ovf);
}

// A 64-bit value moved across the wave's lanes by a DPP control; lanes without a source, or
// in rows outside ROWMASK, receive zero.
template <int CTRL, int ROWMASK, typename V>
__device__ __forceinline__ V dpp64(V v) {
    static_assert(sizeof(V) == 8, "64-bit lanes");
    unsigned long long b;
    __builtin_memcpy(&b, &v, 8);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROWMASK, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROWMASK, 0xf, true);
    b = ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
    V r;
    __builtin_memcpy(&r, &b, 8);
    return r;
}
template <typename V>
__device__ __forceinline__ V lane64(V v, int l) {
    unsigned long long b;
    __builtin_memcpy(&b, &v, 8);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    b = ((unsigned long long)hi << 32) | lo;
    V r;
    __builtin_memcpy(&r, &b, 8);
    return r;
}
// Inclusive prefix sum over the wave's 64 lanes: shifts by 1, 2, 4, 8 within each row of 16
// lanes, then the broadcasts of lanes 15 and 31 into the rows above.
template <typename V>
__device__ __forceinline__ V wave_incl_scan(V v) {
    v += dpp64<0x111, 0xf>(v);  // row_shr:1
    v += dpp64<0x112, 0xf>(v);  // row_shr:2
    v += dpp64<0x114, 0xf>(v);  // row_shr:4
    v += dpp64<0x118, 0xf>(v);  // row_shr:8
    v += dpp64<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp64<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// The NF-fold running sums y_k[j] = sum_{i <= j} y_{k-1}[i], y_0 = x, of a sequence x(0 ..
// len-1), by one wave: lane l takes the run of K elements 64 K c + K l .. + K - 1 of chunk c,
// sums it from zero states, and learns its run's initial states from an exclusive scan, over
// the wave, of the runs' end states (fold k's end state after a run of K from initial states
// s_1..s_k is s_k + sum_{m=1}^{k-1} C(K-1+m, m) s_{k-m} plus the run's own sum from zero,
// so fold by fold the scans are plain sums); the last lane's end states carry into the next
// chunk.  put(j, y_NF[j]).  Integer sums are exact (modulo 2^64); float64 sums round in
// another order than a sequential walk.
template <int NF, int K, typename V, typename X, typename Put>
__device__ __forceinline__ void wave_runsum(int len, X x, Put put) {
    const int lane = threadIdx.x & 63;
    V carry[NF];
#pragma unroll
    for (int k = 0; k < NF; ++k) carry[k] = 0;
    for (int j0 = 0; j0 < len; j0 += 64 * K) {
        const int jb = j0 + lane * K;
        V v[K];
#pragma unroll
        for (int i = 0; i < K; ++i) v[i] = jb + i < len ? x(jb + i) : V(0);
        V l[NF][K];  // the run's own sums, from zero states
#pragma unroll
        for (int i = 0; i < K; ++i) {
            l[0][i] = i ? l[0][i - 1] + v[i] : v[i];
#pragma unroll
            for (int k = 1; k < NF; ++k) l[k][i] = i ? l[k][i - 1] + l[k - 1][i] : l[k - 1][i];
        }
        V c[NF];  // the run's initial states
#pragma unroll
        for (int k = 0; k < NF; ++k) {
            V z = l[k][K - 1];
            long long bc = 1;  // C(K-1+m, m)
#pragma unroll
            for (int m = 1; m <= k; ++m) {
                bc = bc * (K - 1 + m) / m;
                z += (V)bc * c[k - m];
            }
            const V inc = wave_incl_scan(z);
            c[k] = carry[k] + dpp64<0x138, 0xf>(inc);  // wave_shr:1, lane 0 receives zero
            carry[k] += lane64(inc, 63);
        }
#pragma unroll
        for (int i = 0; i < K; ++i) {
            if (jb + i >= len) break;
            V y = l[NF - 1][i];
            long long bc = 1;  // C(i+m, m)
#pragma unroll
            for (int m = 0; m < NF; ++m) {
                if (m) bc = bc * (i + m) / m;
                y += (V)bc * c[NF - 1 - m];
            }
            put(jb + i, y);
        }
    }
}

// The window's box loaded from the input and step (1) of stage 1 run along its rows in the
// same pass (load(r, c) gives box element (r, c); the extension triangle is zero), one wave
// per row, each row anchored at column clamp(cc) as scan_line_n anchors it: forward from the
// anchor, the n-fold sums of x[t+1], x[t+2], ...; backward, the n-fold sums of x[t], x[t-1],
// ... land n columns to the left of their last term, negated for odd n, and the n columns
// t-n+1 .. t hold zero.  Every element is written once, in runs of K per lane.
constexpr int kRowRun = 4;  // elements per lane in a run of load_rows_runsum

template <int NF, int K, typename V, typename Load>
__device__ void load_rows_runsum(V* S, const Geo& g, int cc, Load load) {
    const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6, lane = threadIdx.x & 63;
    const int W = g.wq, H = g.hq, Wt = W + H - 1;
    for (int r = wave; r < H; r += nw) {
        const int len = Wt - r, t = clampi(cc, 0, len - 1);
        const int rowbase = r * W, tr = g.qn + r * (H - 1) - ((r * (r - 1)) >> 1) - W;
        auto at = [&](int c) { return c < W ? rowbase + c : tr + c; };
        wave_runsum<NF, K, V>(
            len - t - 1, [&](int j) { return t + 1 + j < W ? load(r, t + 1 + j) : V(0); },
            [&](int j, V y) { S[at(t + 1 + j)] = y; });
        wave_runsum<NF, K, V>(
            max(t - NF + 1, 0), [&](int j) { return load(r, t - j); },
            [&](int j, V y) { S[at(t - j - NF)] = (NF & 1) ? -y : y; });
        if (lane < NF && t - lane >= 0) S[at(t - lane)] = 0;
    }
}

// ---------------------------------------------------------------------------
// Interpolation at one tap.  p = q + o + u with |u_i| <= 1/2; the quarter turn that
// brings u into the reference triangle u1 >= |u2| is applied to u and to the stencil.
// ---------------------------------------------------------------------------
template <int N>
struct TapFrame {
    int base, s1, s2;  // LDS address of stencil point j: base + jx*s1 + jy*s2
    int lo_ok;         // stencil box inside the window
};

// The cell's triangle follows from the signs of u1 + u2 and u1 - u2; the quarter turn
// R^-tri that maps it onto the reference triangle u1 >= |u2| swaps the two axes when the
// signs differ, then negates the first coordinate when u1 + u2 < 0 and the second when
// u1 - u2 < 0:  tri 0 (u1, u2), 1 (u2, -u1), 2 (-u1, -u2), 3 (-u2, u1).
struct Turn {
    bool swap, n1, n2;
};
__device__ __forceinline__ Turn cell_turn(double u1, double u2) {
    const bool sp = (u1 + u2) >= 0.0, sm = (u1 - u2) >= 0.0;
    return {sp != sm, !sp, !sm};
}

template <int N>
__device__ __forceinline__ TapFrame<N> tap_frame(int qx, int qy, Turn t, int wq, int hq) {
    // odd n rotates about the anchor, even n about the anchor + (1/2, 1/2); stencil
    // point (jx, jy) of the reference triangle sits at (jx, jy), (e - jy, jx),
    // (e - jx, e - jy) or (jy, e - jx) for tri = 0..3
    constexpr int e = Tab<N>::ODD ? 0 : 1;
    const int S1 = t.swap ? wq : 1, S2 = t.swap ? 1 : wq;
    TapFrame<N> f;
    f.s1 = t.n1 ? -S1 : S1;
    f.s2 = t.n2 ? -S2 : S2;
    f.base = (qy + (t.n1 ? e : 0)) * wq + (qx + (t.n2 ? e : 0));
    constexpr int jl = stencil_lo<N>(), jh = stencil_hi<N>();
    f.lo_ok = (qx + jl >= 0) && (qx + jh < wq) && (qy + jl >= 0) && (qy + jh < hq);
    return f;
}

template <int DEG>
__host__ __device__ constexpr int mono_index(int a, int b) {
    return a * (DEG + 1) - (a * (a - 1)) / 2 + b;
}

// Exact integer -> PARTS doubles of SHIFT bits each (the top part keeps the sign), so
// that every product with a table numerator and every partial sum stays exact.
template <int PARTS, int SHIFT>
__device__ __forceinline__ void split_int(long long x, double (&p)[PARTS]) {
    if constexpr (PARTS == 1) {
        p[0] = (double)x;
    } else {
        constexpr long long mask = (1ll << SHIFT) - 1;
#pragma unroll
        for (int i = 0; i + 1 < PARTS; ++i) p[i] = (double)((x >> (i * SHIFT)) & mask);
        p[PARTS - 1] = (double)(x >> ((PARTS - 1) * SHIFT));
    }
}

template <int PARTS, int SHIFT>
__device__ __forceinline__ cp join_parts(const double* g) {
    if constexpr (PARTS == 1) {
        return {g[0], 0.0};
    } else if constexpr (PARTS == 2) {
        const dd t = two_sum(g[1] * (double)(1ll << SHIFT), g[0]);
        return {t.hi, t.lo};
    } else {
        const dd t = dd_add_d(two_sum(g[2] * (double)(1ll << (2 * SHIFT)), g[1] * (double)(1ll << SHIFT)), g[0]);
        return {t.hi, t.lo};
    }
}

// Window values as the mesh reads them.  SRC_INT: int64 running sums, split into PARTS
// exact doubles of SHIFT bits.  SRC_DBL: the tile's values were all below
// 2^exact_bits<N>() and were converted in place to doubles; one exact part suffices.
constexpr int SRC_INT = 0, SRC_DBL = 1;

// How the coefficient sums read the window at the LDS offset of a stencil point.
// PlainRead: the value there.
struct PlainRead {
    const long long* S;
    __device__ __forceinline__ long long i64(int o) const { return S[o]; }
    __device__ __forceinline__ double dbl(int o) const { return reinterpret_cast<const double*>(S)[o]; }
};
// LatRead (integer a1 and a3): the (n+1)^2 taps (k1, k3) of one pair (k2, k4) then share
// their cell -- their anchors differ by (k1 a1, k3 a3), their offset u and quarter turn
// agree -- so the sum of their interpolants is one interpolant of the combined window
//   h[o] = sum_{k1,k3} (-1)^(k1+k3) C(n,k1) C(n,k3) g[o - k1 a1 - k3 a3 wq]
// (the finite-difference weights of eq. FD along r1 and r3).  Integer windows combine in
// wrapping int64, exact whenever |h| < 2^63; float64 windows exactly while the values
// stay below 2^53.
template <int N>
struct LatRead {
    const long long* S;
    int d1, d3;  // a1 and a3 wq: the offsets of one step of k1 and of k3
    static constexpr long long w(int k) { return (k == 0 || k == N) ? 1 : N; }  // C(n, k), n <= 3
    __device__ __forceinline__ long long i64(int o) const {
        unsigned long long h = 0;
#pragma unroll
        for (int k3 = 0; k3 <= N; ++k3) {
            unsigned long long r = 0;
#pragma unroll
            for (int k1 = 0; k1 <= N; ++k1) {
                const unsigned long long v = (unsigned long long)S[o - k1 * d1 - k3 * d3] * (unsigned long long)w(k1);
                r = (k1 & 1) ? r - v : r + v;
            }
            r *= (unsigned long long)w(k3);
            h = (k3 & 1) ? h - r : h + r;
        }
        return (long long)h;
    }
    __device__ __forceinline__ double dbl(int o) const {
        const double* Sd = reinterpret_cast<const double*>(S);
        double h = 0.0;
#pragma unroll
        for (int k3 = 0; k3 <= N; ++k3) {
            double r = 0.0;
#pragma unroll
            for (int k1 = 0; k1 <= N; ++k1)
                r = __fma_rn((k1 & 1) ? -(double)w(k1) : (double)w(k1), Sd[o - k1 * d1 - k3 * d3], r);
            h = __fma_rn((k3 & 1) ? -(double)w(k3) : (double)w(k3), r, h);
        }
        return h;
    }
};

// G_alpha = sum_j NUM[j][alpha] g[q + R j] for the monomials u1^a u2^b with ALO <= a <= AHI,
// in PARTS exact partial sums.  Mirror pairs (j, j') enter once, as g + g' for even b
// and g - g' for odd b.
template <int N, int SRC, int PARTS, int SHIFT, int ALO, int AHI, typename RD>
__device__ __forceinline__ void accumulate_chunk(const RD& rd, const TapFrame<N>& fr,
                                                 double (&G)[PARTS][mono_index<Tab<N>::DEG>(AHI, Tab<N>::DEG - AHI) -
                                                                    mono_index<Tab<N>::DEG>(ALO, 0) + 1],
                                                 unsigned& bad) {
    using T = Tab<N>;
    constexpr int DEG = T::DEG;
    constexpr int M0 = mono_index<DEG>(ALO, 0);
    constexpr int CM = mono_index<DEG>(AHI, DEG - AHI) - M0 + 1;
#pragma unroll
    for (int p = 0; p < PARTS; ++p)
#pragma unroll
        for (int c = 0; c < CM; ++c) G[p][c] = 0.0;
#pragma unroll
    for (int j = 0; j < T::S; ++j) {
        if (!is_rep<N>(j)) continue;
        const int jm = mirror_of<N>(j);
        const int o1 = fr.base + T::jx(j) * fr.s1 + T::jy(j) * fr.s2;
        const int o2 = fr.base + T::jx(jm) * fr.s1 + T::jy(jm) * fr.s2;
        double x[PARTS], xs[PARTS], xd[PARTS];
        if constexpr (SRC == SRC_DBL) {
            const double g1 = rd.dbl(o1);
            if (jm == j) {
                x[0] = g1;
            } else {
                const double g2 = rd.dbl(o2);
                xs[0] = g1 + g2;  // exact: |g| < 2^exact_bits <= 2^50
                xd[0] = g1 - g2;
            }
        } else {
            const long long g1 = rd.i64(o1);
            if (jm == j) {
                split_int<PARTS, SHIFT>(g1, x);
            } else {
                const long long g2 = rd.i64(o2);
                split_int<PARTS, SHIFT>(add_ovf(g1, g2, bad), xs);
                split_int<PARTS, SHIFT>(sub_ovf(g1, g2, bad), xd);
            }
        }
#pragma unroll
        for (int c = 0; c < CM; ++c)
            if (T::num(j, M0 + c) != 0.0) {
                const bool odd = T::mb(M0 + c) & 1;
#pragma unroll
                for (int p = 0; p < PARTS; ++p)
                    G[p][c] = __fma_rn(T::num(j, M0 + c), jm == j ? x[p] : (odd ? xd[p] : xs[p]), G[p][c]);
            }
    }
}

// Order 3: the same accumulation as runtime loops over the 36 representative stencil
// points (fully unrolled, order 3 would be tens of thousands of instructions per variant,
// and its table values up to 6e7 do not fit the literal forms of the FMA, so each would
// first be built in registers).  The points come in four groups with a common set of
// nonzero weight columns (rep3_groups.h); each group has a table in constant memory laid
// out by point -- its offsets, its mirror's, and only the group's weights, contiguous, so
// the weight loads merge -- and a loop whose body touches only those columns: 1,882 FMAs
// per part and tap instead of 2,376.  From a float64 window (one part) all 66 coefficient
// sums are formed in one pass, so the stencil is read once per tap; with three exact parts
// they are formed in two passes over u1-chunks (84 and 114 accumulators).
__host__ __device__ constexpr int rep3_ncols(int grp) {
    int n = 0;
    for (int m = 0; m < bsf_tables::kMono3; ++m) n += bsf_tables::kRep3Cols[grp][m] ? 1 : 0;
    return n;
}
__host__ __device__ constexpr int rep3_col_at(int grp, int i) {  // i-th column of the group
    for (int m = 0; m < bsf_tables::kMono3; ++m)
        if (bsf_tables::kRep3Cols[grp][m] && i-- == 0) return m;
    return -1;
}
template <int GRP>
struct Rep3ColMap {  // the group's columns in order
    int c[rep3_ncols(GRP)];
    constexpr Rep3ColMap() : c() {
        for (int i = 0; i < rep3_ncols(GRP); ++i) c[i] = rep3_col_at(GRP, i);
    }
};
template <int GRP>
struct Rep3Compact {
    static constexpr int NC = rep3_ncols(GRP);
    struct Pt {
        int jx, jy, mjx, mjy, self;
        double w[NC];
    };
    Pt r[bsf_tables::kRep3GroupSize[GRP]];
    constexpr Rep3Compact() : r() {
        int b = 0;
        for (int h = 0; h < GRP; ++h) b += bsf_tables::kRep3GroupSize[h];
        for (int k = 0; k < bsf_tables::kRep3GroupSize[GRP]; ++k) {
            const int j = bsf_tables::kRep3Points[b + k];
            const int jm = mirror_of<3>(j);
            Pt& q = r[k];
            q.jx = bsf_tables::kJ3[j][0];
            q.jy = bsf_tables::kJ3[j][1];
            q.mjx = bsf_tables::kJ3[jm][0];
            q.mjy = bsf_tables::kJ3[jm][1];
            q.self = jm == j;
            for (int i = 0; i < NC; ++i) q.w[i] = bsf_tables::kNum3[j][rep3_col_at(GRP, i)];
        }
    }
};
__constant__ Rep3Compact<0> c_rep3g0 = Rep3Compact<0>();
__constant__ Rep3Compact<1> c_rep3g1 = Rep3Compact<1>();
__constant__ Rep3Compact<2> c_rep3g2 = Rep3Compact<2>();
__constant__ Rep3Compact<3> c_rep3g3 = Rep3Compact<3>();
static_assert(bsf_tables::kRep3Groups == 4, "one compact table per group");
template <int GRP>
__device__ __forceinline__ const Rep3Compact<GRP>& rep3_compact() {
    if constexpr (GRP == 0) return c_rep3g0;
    else if constexpr (GRP == 1) return c_rep3g1;
    else if constexpr (GRP == 2) return c_rep3g2;
    else return c_rep3g3;
}

__host__ __device__ constexpr int rep3_begin(int grp) {
    int b = 0;
    for (int h = 0; h < grp; ++h) b += bsf_tables::kRep3GroupSize[h];
    return b;
}
__host__ __device__ constexpr bool rep3_col(int grp, int c) { return bsf_tables::kRep3Cols[grp][c]; }
__host__ __device__ constexpr bool rep3_groups_ok() {  // every point a representative, once,
    bool seen[bsf_tables::kStencil3] = {};              // and every nonzero weight in its columns
    for (int grp = 0; grp < bsf_tables::kRep3Groups; ++grp)
        for (int k = rep3_begin(grp); k < rep3_begin(grp + 1); ++k) {
            const int j = bsf_tables::kRep3Points[k];
            if (!is_rep<3>(j) || seen[j]) return false;
            seen[j] = true;
            for (int m = 0; m < bsf_tables::kMono3; ++m)
                if (bsf_tables::kNum3[j][m] != 0.0 && !rep3_col(grp, m)) return false;
        }
    int reps = 0;
    for (int j = 0; j < bsf_tables::kStencil3; ++j) reps += is_rep<3>(j) ? 1 : 0;
    return reps == (bsf_tables::kStencil3 + 9) / 2 && rep3_begin(bsf_tables::kRep3Groups) == reps;
}
static_assert(rep3_groups_ok(), "rep3_groups.h does not match the order-3 table");

// The address of a group table as an opaque wave-uniform value in the constant address
// space: accessed through the symbol, every 16-dword weight load rebuilt the address from
// the program counter and the relocation (five scalar instructions per eight FMAs); from
// a base register the loads take immediate offsets.
template <int GRP>
__device__ __forceinline__ const __attribute__((address_space(4))) typename Rep3Compact<GRP>::Pt* rep3_points() {
    const unsigned long long a = reinterpret_cast<unsigned long long>(static_cast<const void*>(&rep3_compact<GRP>()));
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
    return reinterpret_cast<const __attribute__((address_space(4))) typename Rep3Compact<GRP>::Pt*>(
        ((unsigned long long)hi << 32) | lo);
}

template <int GRP, int SRC, int PARTS, int SHIFT, int M0, int CM, typename RD>
__device__ __forceinline__ void accumulate_group3(const RD& rd, const TapFrame<3>& fr, double (&G)[PARTS][CM],
                                                  unsigned& bad) {
    using T = Tab<3>;
    constexpr int NC = Rep3Compact<GRP>::NC;
    constexpr Rep3ColMap<GRP> cols{};
    const auto* pts = rep3_points<GRP>();
#pragma unroll 1
    for (int k = 0; k < bsf_tables::kRep3GroupSize[GRP]; ++k) {
        const auto& q = pts[k];
        // |j| <= 3 and |s| <= wq < 2^23: the 24-bit multiply (full rate; the 32-bit one is
        // quarter rate) is exact
        const int o1 = fr.base + __mul24(q.jx, fr.s1) + __mul24(q.jy, fr.s2);
        const int o2 = fr.base + __mul24(q.mjx, fr.s1) + __mul24(q.mjy, fr.s2);
        double xs[PARTS], xd[PARTS];
        if constexpr (SRC == SRC_DBL) {
            const double g1 = rd.dbl(o1), g2 = q.self ? 0.0 : rd.dbl(o2);
            xs[0] = g1 + g2;  // exact when the window values are below 2^exact_bits
            xd[0] = g1 - g2;
        } else {
            const long long g1 = rd.i64(o1), g2 = q.self ? 0ll : rd.i64(o2);
            split_int<PARTS, SHIFT>(add_ovf(g1, g2, bad), xs);
            split_int<PARTS, SHIFT>(sub_ovf(g1, g2, bad), xd);
        }
#pragma unroll
        for (int i = 0; i < NC; ++i) {
            const int c = cols.c[i];
            if (c < M0 || c >= M0 + CM) continue;
#pragma unroll
            for (int p = 0; p < PARTS; ++p)
                G[p][c - M0] = __fma_rn(q.w[i], (T::mb(c) & 1) ? xd[p] : xs[p], G[p][c - M0]);
        }
    }
    if constexpr (GRP + 1 < bsf_tables::kRep3Groups)
        accumulate_group3<GRP + 1, SRC, PARTS, SHIFT, M0, CM>(rd, fr, G, bad);
}

template <int SRC, int PARTS, int SHIFT, int ALO, int AHI, typename RD>
__device__ __forceinline__ void accumulate_chunk3(const RD& rd, const TapFrame<3>& fr,
                                                  double (&G)[PARTS][mono_index<10>(AHI, 10 - AHI) -
                                                                     mono_index<10>(ALO, 0) + 1],
                                                  unsigned& bad) {
    constexpr int M0 = mono_index<10>(ALO, 0);
    constexpr int CM = mono_index<10>(AHI, 10 - AHI) - M0 + 1;
    asm volatile("" ::: "memory");  // keep each chunk's LDS reads local to the chunk
#pragma unroll
    for (int p = 0; p < PARTS; ++p)
#pragma unroll
        for (int c = 0; c < CM; ++c) G[p][c] = 0.0;
    accumulate_group3<0, SRC, PARTS, SHIFT, M0, CM>(rd, fr, G, bad);
}

template <typename RD>
__device__ __forceinline__ void accumulate_all3_dbl(const RD& rd, const TapFrame<3>& fr,
                                                    double (&G)[1][bsf_tables::kMono3]) {
    using T = Tab<3>;
#pragma unroll
    for (int c = 0; c < T::M; ++c) G[0][c] = 0.0;
    unsigned unused = 0;
    accumulate_group3<0, SRC_DBL, 1, 0, 0, T::M>(rd, fr, G, unused);
}

// Horner over the chunk's u1-powers AHI..ALO (compensated), continuing the running value P.
template <int N, int PARTS, int SHIFT, int ALO, int AHI, bool FIRST>
__device__ __forceinline__ void horner_chunk_dd(
    const double (&G)[PARTS][mono_index<Tab<N>::DEG>(AHI, Tab<N>::DEG - AHI) - mono_index<Tab<N>::DEG>(ALO, 0) + 1],
    dd v1, dd v2, cp& P) {
    constexpr int DEG = Tab<N>::DEG;
    constexpr int M0 = mono_index<DEG>(ALO, 0);
#pragma unroll
    for (int a = AHI; a >= ALO; --a) {
        double c[PARTS];
#pragma unroll
        for (int p = 0; p < PARTS; ++p) c[p] = G[p][mono_index<DEG>(a, DEG - a) - M0];
        cp q = join_parts<PARTS, SHIFT>(c);
#pragma unroll
        for (int b = DEG - a - 1; b >= 0; --b) {
#pragma unroll
            for (int p = 0; p < PARTS; ++p) c[p] = G[p][mono_index<DEG>(a, b) - M0];
            if constexpr (PARTS == 1) q = cp_horner(q, v2, c[0]);  // exact single-part coefficient
            else q = cp_horner(q, v2, join_parts<PARTS, SHIFT>(c));
        }
        P = (FIRST && a == AHI) ? q : cp_horner(P, v1, q);
    }
}

// A coefficient's parts as one rounded double (at most two roundings).
template <int PARTS, int SHIFT>
__device__ __forceinline__ double join_plain(const double* g) {
    if constexpr (PARTS == 1) return g[0];
    else if constexpr (PARTS == 2) return __fma_rn(g[1], (double)(1ll << SHIFT), g[0]);
    else return __fma_rn(g[2], (double)(1ll << (2 * SHIFT)), __fma_rn(g[1], (double)(1ll << SHIFT), g[0]));
}

__host__ __device__ constexpr double pow2_neg(int k) {
    double r = 1.0;
    for (int i = 0; i < k; ++i) r *= 0.5;
    return r;
}

// The same polynomial split by total degree a + b.  The terms above LOW -- the high
// differences of the pre-integrated window, small next to the low ones wherever the
// window is smooth on the scale of the cell -- go through a plain FMA Horner at the
// high words of v (PH); the terms up to LOW through the compensated Horner (PL).  With
// |v1|, |v2| <= 1/2 the plain part's error is at most gamma * B, B = sum |G_ab| 2^-(a+b)
// over its terms, where gamma covers the coefficient joins, the dropped low words of v
// and the Horner roundings along any path (at most 3 DEG + 2 units of 2^-53).
template <int N, int PARTS, int SHIFT, int ALO, int AHI, int LOW, bool FIRST>
__device__ __forceinline__ void horner_chunk_split(
    const double (&G)[PARTS][mono_index<Tab<N>::DEG>(AHI, Tab<N>::DEG - AHI) - mono_index<Tab<N>::DEG>(ALO, 0) + 1],
    dd v1, dd v2, double& PH, cp& PL, double& B) {
    constexpr int DEG = Tab<N>::DEG;
    constexpr int M0 = mono_index<DEG>(ALO, 0);
    static_assert(LOW < DEG, "the split needs a plain part");
#pragma unroll
    for (int a = AHI; a >= ALO; --a) {
        double c[PARTS];
        double qh = 0.0;
#pragma unroll
        for (int b = DEG - a; b >= 0; --b) {
            if (a + b > LOW) {
#pragma unroll
                for (int p = 0; p < PARTS; ++p) c[p] = G[p][mono_index<DEG>(a, b) - M0];
                const double x = join_plain<PARTS, SHIFT>(c);
                B = __fma_rn(fabs(x), pow2_neg(a + b), B);
                qh = (b == DEG - a) ? x : __fma_rn(qh, v2.hi, x);
            } else {
                qh = qh * v2.hi;
            }
        }
        PH = (FIRST && a == AHI) ? qh : __fma_rn(PH, v1.hi, qh);
        if (a <= LOW) {
#pragma unroll
            for (int p = 0; p < PARTS; ++p) c[p] = G[p][mono_index<DEG>(a, LOW - a) - M0];
            cp q = join_parts<PARTS, SHIFT>(c);
#pragma unroll
            for (int b = LOW - a - 1; b >= 0; --b) {
#pragma unroll
                for (int p = 0; p < PARTS; ++p) c[p] = G[p][mono_index<DEG>(a, b) - M0];
                if constexpr (PARTS == 1) q = cp_horner(q, v2, c[0]);
                else q = cp_horner(q, v2, join_parts<PARTS, SHIFT>(c));
            }
            PL = (a == LOW) ? q : cp_horner(PL, v1, q);
        }
    }
}

// Split evaluation: terms of total degree up to split_low<N>() compensated, the rest
// plain.  Order 1 (degree 2) is evaluated compensated throughout.
template <int N>
__host__ __device__ constexpr int split_low() { return (N == 1 || N >= 10) ? Tab<N>::DEG : (N == 2 ? 2 : 3); }
// a1 a2 a3 a4 from which a pixel's taps are evaluated split (see process_tile): a
// geometric-mean scale of 5 (order 2) or 4.5 (order 3)
template <int N>
__host__ __device__ constexpr double split_min_volume() { return N == 2 ? 625.0 : 410.0; }

template <int N, int SRC, int ALO, int AHI, bool FIRST, int LOW, typename RD>
__device__ __forceinline__ void interp_chunk_dd(const RD& rd, const TapFrame<N>& fr, dd v1, dd v2, cp& P,
                                                double& PH, double& B, unsigned& bad) {
    using T = Tab<N>;
    constexpr int PARTS = SRC == SRC_DBL ? 1 : T::SPLIT;
    double G[PARTS][mono_index<T::DEG>(AHI, T::DEG - AHI) - mono_index<T::DEG>(ALO, 0) + 1];
    if constexpr (N == 3 && SRC == SRC_DBL && ALO == 0 && AHI == 10)
        accumulate_all3_dbl(rd, fr, G);
    else if constexpr (N == 3)
        accumulate_chunk3<SRC, PARTS, T::SHIFT, ALO, AHI>(rd, fr, G, bad);
    else
        accumulate_chunk<N, SRC, PARTS, T::SHIFT, ALO, AHI>(rd, fr, G, bad);
    if constexpr (LOW >= T::DEG)
        horner_chunk_dd<N, PARTS, T::SHIFT, ALO, AHI, FIRST>(G, v1, v2, P);
    else
        horner_chunk_split<N, PARTS, T::SHIFT, ALO, AHI, LOW, FIRST>(G, v1, v2, PH, P, B);
}

// Horner over the chunk's u1-powers AHI..ALO in plain double, continuing P.
template <int N, int ALO, int AHI, bool FIRST>
__device__ __forceinline__ void horner_chunk_f64(
    const double (&G)[1][mono_index<Tab<N>::DEG>(AHI, Tab<N>::DEG - AHI) - mono_index<Tab<N>::DEG>(ALO, 0) + 1],
    double v1, double v2, double& P) {
    constexpr int DEG = Tab<N>::DEG;
    constexpr int M0 = mono_index<DEG>(ALO, 0);
#pragma unroll
    for (int a = AHI; a >= ALO; --a) {
        double q = G[0][mono_index<DEG>(a, DEG - a) - M0];
#pragma unroll
        for (int b = DEG - a - 1; b >= 0; --b) q = __fma_rn(q, v2, G[0][mono_index<DEG>(a, b) - M0]);
        P = (FIRST && a == AHI) ? q : __fma_rn(P, v1, q);
    }
}

template <int N, int SRC, int ALO, int AHI, bool FIRST, typename RD>
__device__ __forceinline__ void interp_chunk_f64(const RD& rd, const TapFrame<N>& fr, double v1, double v2,
                                                 double& P, unsigned& bad) {
    using T = Tab<N>;
    double G[1][mono_index<T::DEG>(AHI, T::DEG - AHI) - mono_index<T::DEG>(ALO, 0) + 1];
    if constexpr (N == 3 && SRC == SRC_DBL && ALO == 0 && AHI == 10)
        accumulate_all3_dbl(rd, fr, G);
    else if constexpr (N == 3)
        accumulate_chunk3<SRC, 1, 0, ALO, AHI>(rd, fr, G, bad);
    else
        accumulate_chunk<N, SRC, 1, 0, ALO, AHI>(rd, fr, G, bad);
    horner_chunk_f64<N, ALO, AHI, FIRST>(G, v1, v2, P);
}

// sum_j g[q+j] beta(o + u - j) = (1/DEN) sum_alpha G_alpha v^alpha: the coefficients
// accumulated exactly, the polynomial in compensated arithmetic (order 3 in u1-chunks
// to bound registers).
// With LOW below the degree, B receives the plain part's error weight (see
// horner_chunk_split) and the plain part is folded into the low word of the result.
template <int N, int SRC, int LOW, typename RD>
__device__ __forceinline__ cp interp_dd(const RD& rd, const TapFrame<N>& fr, dd v1, dd v2, double& B,
                                        unsigned& bad) {
    using T = Tab<N>;
    cp P = {0.0, 0.0};
    double PH = 0.0;
    if constexpr (N != 3 || SRC == SRC_DBL) {
        interp_chunk_dd<N, SRC, 0, T::DEG, true, LOW>(rd, fr, v1, v2, P, PH, B, bad);
    } else {  // three parts: two u1-chunks (84 and 114 accumulators)
        interp_chunk_dd<N, SRC, 4, 10, true, LOW>(rd, fr, v1, v2, P, PH, B, bad);
        interp_chunk_dd<N, SRC, 0, 3, false, LOW>(rd, fr, v1, v2, P, PH, B, bad);
    }
    if constexpr (LOW < T::DEG) P.c += PH;
    return P;
}

// the same in plain double
template <int N, int SRC, typename RD>
__device__ __forceinline__ double interp_f64(const RD& rd, const TapFrame<N>& fr, double v1, double v2,
                                             unsigned& bad) {
    using T = Tab<N>;
    double P = 0.0;
    if constexpr (N != 3 || SRC == SRC_DBL) {
        interp_chunk_f64<N, SRC, 0, T::DEG, true>(rd, fr, v1, v2, P, bad);
    } else {
        interp_chunk_f64<N, SRC, 4, 10, true>(rd, fr, v1, v2, P, bad);
        interp_chunk_f64<N, SRC, 0, 3, false>(rd, fr, v1, v2, P, bad);
    }
    return P;
}

// binom(N, k) for the finite-difference weights of eq. FD (N <= 3, k in 0..N)
template <int N>
__device__ __forceinline__ int fd_binom(int k) {
    static_assert(N >= 1 && N <= 3, "orders 1..3");
    if constexpr (N == 1) return 1;
    else if constexpr (N == 2) return k == 1 ? 2 : 1;
    else return (k == 1 || k == 2) ? 3 : 1;
}

__device__ __forceinline__ dd dd_turn(bool swap, bool neg, dd a, dd b) {  // +-(swap ? b : a)
    dd r = swap ? b : a;
    r.hi = neg ? -r.hi : r.hi;
    r.lo = neg ? -r.lo : r.lo;
    return r;
}

// One pixel of the order-N mesh (eq. final_eqn): s[m] = sum_k c_k g_I(m + n tau - x_k),
// c_k = prod_d d^n_{a_d}[k_d] (eq. FD), x_k = sum_d k_d a_d r_d (Table 1 for n = 1),
// n tau per Section 7 (the shift of eq. factor, n-fold).  Window coordinates: (mx, my)
// is the pixel relative to the window origin.  Returns s in units of the integer
// samples (the caller applies the input quantum).
//
// With LOW below the polynomial degree the taps use the split evaluation and E receives
// sum_k |c_k| B_k, which times 2^-47 bounds the error of the plain parts.
template <int N, int SRC, int LOW = Tab<N>::DEG, int K = N>
__device__ dd mesh_dd(const long long* S, int wq, int hq, int mx, int my, float4 a, int k2lo, int k2hi,
                      unsigned& bad, double& E) {
    const dd isq = {kInvSqrt2Hi, kInvSqrt2Lo};
    const double a1 = a.x, a3 = a.z;
    const dd A2 = dd_mul_d(isq, (double)a.y);  // a'_2 = a2/sqrt2 (lattice units along (1,1))
    const dd A4 = dd_mul_d(isq, (double)a.w);  // a'_4
    constexpr double h = 0.5 * N;
    // n*tau = (n/2)(a1 + a'2 - a'4 - 1, a'2 + a3 + a'4 - 3)
    const dd T1 = dd_mul_d(dd_add_d(dd_add(A2, dd_neg(A4)), a1 - 1.0), h);
    const dd T2 = dd_mul_d(dd_add_d(dd_add(A2, A4), a3 - 3.0), h);
    cp acc = {0.0, 0.0};
    for (int k2 = k2lo; k2 <= k2hi; ++k2) {
        for (int k4 = 0; k4 <= N; ++k4) {
            const int c24 = fd_binom<N>(k2) * fd_binom<N>(k4);
            const dd D2 = dd_mul_d(A2, (double)k2), D4 = dd_mul_d(A4, (double)k4);
            const dd B1 = dd_add(T1, dd_add(D4, dd_neg(D2)));        // n tau_1 - k2 a'2 + k4 a'4
            const dd B2 = dd_add(T2, dd_neg(dd_add(D2, D4)));         // n tau_2 - k2 a'2 - k4 a'4
            for (int k1 = 0; k1 <= N; ++k1) {
                const int c124 = c24 * fd_binom<N>(k1);
                const dd d1 = dd_add_d(B1, -(double)k1 * a1);
                for (int k3 = 0; k3 <= N; ++k3) {
                    const dd d2 = dd_add_d(B2, -(double)k3 * a3);
                    // anchor and local offset
                    double f1, f2;
                    if (Tab<K>::ODD) {
                        f1 = rint(d1.hi);
                        f2 = rint(d2.hi);
                    } else {
                        f1 = floor(d1.hi);
                        f2 = floor(d2.hi);
                    }
                    // u = d - (q + o) in double-double: d.hi - q alone is not exact when
                    // the anchor is floor(d) and d lies in (-1, 0)
                    const double oc = Tab<K>::ODD ? 0.0 : 0.5;
                    const dd u1 = dd_add_d(d1, -(f1 + oc));
                    const dd u2 = dd_add_d(d2, -(f2 + oc));
                    const Turn t = cell_turn(u1.hi, u2.hi);
                    const dd v1 = dd_turn(t.swap, t.n1, u1, u2);
                    const dd v2 = dd_turn(t.swap, t.n2, u2, u1);
                    const TapFrame<K> fr = tap_frame<K>(mx + (int)f1, my + (int)f2, t, wq, hq);
                    if (!fr.lo_ok) {
                        bad = 1;
                        continue;
                    }
                    double Bk = 0.0;
                    const cp P = interp_dd<K, SRC, LOW>(PlainRead{S}, fr, v1, v2, Bk, bad);
                    const int c = c124 * fd_binom<N>(k3);
                    const double cs = ((k1 + k2 + k3 + k4) & 1) ? -(double)c : (double)c;
                    acc = cp_axpy(acc, cs, P);
                    if constexpr (LOW < Tab<K>::DEG) E = __fma_rn((double)c, Bk, E);
                }
            }
        }
    }
    return fast_two_sum(acc.s, acc.c);
}

// s = acc * 2^n / DEN / (a1 a2 a3 a4)^n  (the sqrt2 weights of the two diagonal running
// sums, the table denominator and the finite-difference weights d^n_a of eq. FD)
template <int N, int K = N>
__device__ double finalize_dd(dd acc, float4 a) {
    const dd prod = two_prod((double)a.x * (double)a.y, (double)a.z * (double)a.w);  // exact
    dd pn = prod;
    for (int i = 1; i < N; ++i) pn = dd_mul(pn, prod);
    const dd den = {Tab<K>::DEN / (double)(1 << N), 0.0};
    const dd r = dd_div(dd_div(acc, den), pn);
    return r.hi + r.lo;
}

template <int N, int SRC, int K = N>
__device__ double mesh_f64(const long long* S, int wq, int hq, int mx, int my, float4 a, int k2lo, int k2hi,
                           unsigned& bad) {  // raw sum over k2 in [k2lo, k2hi]
    const double a1 = a.x, a3 = a.z;
    const double A2 = (double)a.y * kInvSqrt2Hi, A4 = (double)a.w * kInvSqrt2Hi;
    constexpr double h = 0.5 * N;
    const double T1 = h * (a1 + A2 - A4 - 1.0);
    const double T2 = h * (A2 + a3 + A4 - 3.0);
    double acc = 0.0;
    for (int k2 = k2lo; k2 <= k2hi; ++k2) {
        for (int k4 = 0; k4 <= N; ++k4) {
            const int c24 = fd_binom<N>(k2) * fd_binom<N>(k4);
            const double B1 = T1 - k2 * A2 + k4 * A4;
            const double B2 = T2 - k2 * A2 - k4 * A4;
            for (int k1 = 0; k1 <= N; ++k1) {
                const int c124 = c24 * fd_binom<N>(k1);
                const double d1 = B1 - k1 * a1;
                for (int k3 = 0; k3 <= N; ++k3) {
                    const double d2 = B2 - k3 * a3;
                    const double f1 = Tab<K>::ODD ? rint(d1) : floor(d1);
                    const double f2 = Tab<K>::ODD ? rint(d2) : floor(d2);
                    const double oc = Tab<K>::ODD ? 0.0 : 0.5;
                    const double u1 = d1 - f1 - oc, u2 = d2 - f2 - oc;
                    const Turn t = cell_turn(u1, u2);
                    const double w1 = t.swap ? u2 : u1, w2 = t.swap ? u1 : u2;
                    const double v1 = t.n1 ? -w1 : w1, v2 = t.n2 ? -w2 : w2;
                    const TapFrame<K> fr = tap_frame<K>(mx + (int)f1, my + (int)f2, t, wq, hq);
                    if (!fr.lo_ok) {
                        bad = 1;
                        continue;
                    }
                    const double P = interp_f64<K, SRC>(PlainRead{S}, fr, v1, v2, bad);
                    const int c = c124 * fd_binom<N>(k3);
                    acc = __fma_rn(((k1 + k2 + k3 + k4) & 1) ? -(double)c : (double)c, P, acc);
                }
            }
        }
    }
    return acc;
}

// Whether a pixel's (k1, k3) taps share their cell: integer a1 and a3.
__device__ __forceinline__ bool lattice_scales(float4 a) { return a.x == rintf(a.x) && a.z == rintf(a.z); }

// mesh_dd for integer a1 and a3: the (n+1)^2 taps (k1, k3) of each pair (k2, k4) as one
// interpolant of the combined window (LatRead), so one set of coefficient sums and one
// polynomial per pair instead of (n+1)^2 of each.  The geometry is mesh_dd's at k1 = k3 =
// 0 -- the other anchors follow exactly -- and the frame check covers all (k1, k3).  E
// receives sum |c24| B of the combined polynomials, which bounds the plain parts' error as
// in mesh_dd.  Integer windows need |values| < 2^(62 - 2n), float64 windows values below
// 2^(exact_bits - 2n), for the combined sums to stay exact (the caller checks).
template <int N, int SRC, int LOW = Tab<N>::DEG, int K = N>
__device__ dd mesh_dd_lat(const long long* S, int wq, int hq, int mx, int my, float4 a, int k2lo, int k2hi,
                          unsigned& bad, double& E) {
    const dd isq = {kInvSqrt2Hi, kInvSqrt2Lo};
    const double a1 = a.x;
    const int i1 = (int)a.x, i3 = (int)a.z;
    const dd A2 = dd_mul_d(isq, (double)a.y);
    const dd A4 = dd_mul_d(isq, (double)a.w);
    constexpr double h = 0.5 * N;
    constexpr int jl = stencil_lo<K>(), jh = stencil_hi<K>();
    const dd T1 = dd_mul_d(dd_add_d(dd_add(A2, dd_neg(A4)), a1 - 1.0), h);
    const dd T2 = dd_mul_d(dd_add_d(dd_add(A2, A4), (double)a.z - 3.0), h);
    const LatRead<N> rd = {S, i1, i3 * wq};
    cp acc = {0.0, 0.0};
    for (int k2 = k2lo; k2 <= k2hi; ++k2) {
        for (int k4 = 0; k4 <= N; ++k4) {
            const int c24 = fd_binom<N>(k2) * fd_binom<N>(k4);
            const dd D2 = dd_mul_d(A2, (double)k2), D4 = dd_mul_d(A4, (double)k4);
            const dd d1 = dd_add_d(dd_add(T1, dd_add(D4, dd_neg(D2))), -0.0);
            const dd d2 = dd_add_d(dd_add(T2, dd_neg(dd_add(D2, D4))), -0.0);
            const double f1 = Tab<K>::ODD ? rint(d1.hi) : floor(d1.hi);
            const double f2 = Tab<K>::ODD ? rint(d2.hi) : floor(d2.hi);
            const double oc = Tab<K>::ODD ? 0.0 : 0.5;
            const dd u1 = dd_add_d(d1, -(f1 + oc));
            const dd u2 = dd_add_d(d2, -(f2 + oc));
            const Turn t = cell_turn(u1.hi, u2.hi);
            const dd v1 = dd_turn(t.swap, t.n1, u1, u2);
            const dd v2 = dd_turn(t.swap, t.n2, u2, u1);
            const int qx = mx + (int)f1, qy = my + (int)f2;
            const TapFrame<K> fr = tap_frame<K>(qx, qy, t, wq, hq);
            if (!(qx - N * i1 + jl >= 0 && qx + jh < wq && qy - N * i3 + jl >= 0 && qy + jh < hq)) {
                bad = 1;
                continue;
            }
            double Bk = 0.0;
            const cp P = interp_dd<K, SRC, LOW>(rd, fr, v1, v2, Bk, bad);
            acc = cp_axpy(acc, ((k2 + k4) & 1) ? -(double)c24 : (double)c24, P);
            if constexpr (LOW < Tab<K>::DEG) E = __fma_rn((double)c24, Bk, E);
        }
    }
    return fast_two_sum(acc.s, acc.c);
}

// mesh_f64 for integer a1 and a3 (as mesh_dd_lat).
template <int N, int SRC, int K = N>
__device__ double mesh_f64_lat(const long long* S, int wq, int hq, int mx, int my, float4 a, int k2lo, int k2hi,
                               unsigned& bad) {
    const double a1 = a.x, a3 = a.z;
    const int i1 = (int)a.x, i3 = (int)a.z;
    const double A2 = (double)a.y * kInvSqrt2Hi, A4 = (double)a.w * kInvSqrt2Hi;
    constexpr double h = 0.5 * N;
    constexpr int jl = stencil_lo<K>(), jh = stencil_hi<K>();
    const double T1 = h * (a1 + A2 - A4 - 1.0);
    const double T2 = h * (A2 + a3 + A4 - 3.0);
    const LatRead<N> rd = {S, i1, i3 * wq};
    double acc = 0.0;
    for (int k2 = k2lo; k2 <= k2hi; ++k2) {
        for (int k4 = 0; k4 <= N; ++k4) {
            const int c24 = fd_binom<N>(k2) * fd_binom<N>(k4);
            const double d1 = T1 - k2 * A2 + k4 * A4;
            const double d2 = T2 - k2 * A2 - k4 * A4;
            const double f1 = Tab<K>::ODD ? rint(d1) : floor(d1);
            const double f2 = Tab<K>::ODD ? rint(d2) : floor(d2);
            const double oc = Tab<K>::ODD ? 0.0 : 0.5;
            const double u1 = d1 - f1 - oc, u2 = d2 - f2 - oc;
            const Turn t = cell_turn(u1, u2);
            const double w1 = t.swap ? u2 : u1, w2 = t.swap ? u1 : u2;
            const double v1 = t.n1 ? -w1 : w1, v2 = t.n2 ? -w2 : w2;
            const int qx = mx + (int)f1, qy = my + (int)f2;
            const TapFrame<K> fr = tap_frame<K>(qx, qy, t, wq, hq);
            if (!(qx - N * i1 + jl >= 0 && qx + jh < wq && qy - N * i3 + jl >= 0 && qy + jh < hq)) {
                bad = 1;
                continue;
            }
            const double P = interp_f64<K, SRC>(rd, fr, v1, v2, bad);
            acc = __fma_rn(((k2 + k4) & 1) ? -(double)c24 : (double)c24, P, acc);
        }
    }
    return acc;
}

// ---------------------------------------------------------------------------
// The mesh over a band of the window (windows held in global scratch, evaluated from LDS
// in bands of rows).  A pixel's taps come in triples (k2, k4, k3) whose three k1 taps
// share the anchor row; a triple belongs to the band when its stencil's first window row
// q2 + stencil_lo lies in [own0, own1).  The band buffer S holds window rows row0 .. row0
// + nrows - 1 at the window's pitch wq.  The tap geometry is mesh_dd's and mesh_f64's,
// operation for operation; the taps are summed triple by triple, band by band.
//
// The band's triples of a wave's 64 pixels are spread evenly over its lanes.  Each lane
// lists the triples of its pixel that the band owns (a bit per triple index i = ((k2 -
// k2lo) (N+1) + k4) (N+1) + k3); a wave scan of the counts numbers the items owner by
// owner, and the wave evaluates them 64 at a time,
// lane l taking item base + l: its owner is the last lane whose first item number is at
// most base + l, its triple the owner's set bit of that rank, its pixel (mx, my, a) read
// from the owner's lane.  Each owner then adds the values of its items, in item order,
// from the lanes that evaluated them.  A wave thus spends about (its owned triples) / 64
// triple evaluations per band instead of its busiest lane's count.  Every lane of the wave
// calls these with the same band; an inactive pixel owns nothing.
template <int N, int K, bool DD>
__device__ __forceinline__ unsigned long long band_owned(int my, float4 a, int k2lo, int k2hi, int own0, int own1) {
    constexpr int NP = N + 1;
    constexpr int jl = stencil_lo<K>();
    constexpr double h = 0.5 * N;
    const double a3 = a.z;
    unsigned long long m = 0;
    int bit = 0;
    auto own = [&](double d2hi) {
        const double f2 = Tab<K>::ODD ? rint(d2hi) : floor(d2hi);
        const int s = my + (int)f2 + jl;
        if (s >= own0 && s < own1) m |= 1ull << bit;
        ++bit;
    };
    if constexpr (DD) {  // triple_dd's d2
        const dd isq = {kInvSqrt2Hi, kInvSqrt2Lo};
        const dd A2 = dd_mul_d(isq, (double)a.y), A4 = dd_mul_d(isq, (double)a.w);
        const dd T2 = dd_mul_d(dd_add_d(dd_add(A2, A4), a3 - 3.0), h);
        for (int k2 = k2lo; k2 <= k2hi; ++k2)
#pragma unroll
            for (int k4 = 0; k4 < NP; ++k4) {
                const dd D2 = dd_mul_d(A2, (double)k2), D4 = dd_mul_d(A4, (double)k4);
                const dd B2 = dd_add(T2, dd_neg(dd_add(D2, D4)));
#pragma unroll
                for (int k3 = 0; k3 < NP; ++k3) own(dd_add_d(B2, -(double)k3 * a3).hi);
            }
    } else {  // triple_f64's d2
        const double A2 = (double)a.y * kInvSqrt2Hi, A4 = (double)a.w * kInvSqrt2Hi;
        const double T2 = h * (A2 + a3 + A4 - 3.0);
        for (int k2 = k2lo; k2 <= k2hi; ++k2)
#pragma unroll
            for (int k4 = 0; k4 < NP; ++k4) {
                const double B2 = T2 - k2 * A2 - k4 * A4;
#pragma unroll
                for (int k3 = 0; k3 < NP; ++k3) own(B2 - k3 * a3);
            }
    }
    return m;
}
__device__ __forceinline__ int wave_incl_scan_i(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);  // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);  // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true);  // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true);  // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, true);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, true);  // row_bcast:31
    return v;
}
// Index of the set bit of rank r (r < popcount(m)).
__device__ __forceinline__ int select_bit(unsigned long long m, int r) {
    int t = 0;
#pragma unroll
    for (int w = 32; w; w >>= 1) {
        const int low = __popcll(m & ((1ull << w) - 1ull));
        if (r >= low) {
            r -= low;
            m >>= w;
            t += w;
        }
    }
    return t;
}
__device__ __forceinline__ int wave_max_i(int v);
// The item loop: eval(live, t, mx, my, a) evaluates triple t of the pixel (mx, my, a) into
// the lane's item value; pull(src, take) then adds lane src's item value to the owner's sums
// when take holds (called with the same src by the whole wave, j-th item of each owner).
template <typename Eval, typename Pull>
__device__ __forceinline__ void spread_items(unsigned long long mask, int mx, int my, float4 a, Eval eval, Pull pull) {
    const int lane = threadIdx.x & 63;
    const int cnt = __popcll(mask);
    const int incl = wave_incl_scan_i(cnt);
    const int start = incl - cnt;
    const int total = __builtin_amdgcn_readlane(incl, 63);
    const unsigned mlo = (unsigned)mask, mhi = (unsigned)(mask >> 32);
    const int ax = __float_as_int(a.x), ay = __float_as_int(a.y), az = __float_as_int(a.z), aw = __float_as_int(a.w);
    for (int base = 0; base < total; base += 64) {
        const int i = base + lane;
        int o = 0;  // the item's owner
#pragma unroll
        for (int step = 32; step; step >>= 1) {
            const int p = o + step;
            if (__shfl(start, p) <= i) o = p;
        }
        const int rank = i - __shfl(start, o);
        const unsigned long long mo =
            ((unsigned long long)(unsigned)__shfl((int)mhi, o) << 32) | (unsigned)__shfl((int)mlo, o);
        const int omx = __shfl(mx, o), omy = __shfl(my, o);
        const float4 oa = make_float4(__int_as_float(__shfl(ax, o)), __int_as_float(__shfl(ay, o)),
                                      __int_as_float(__shfl(az, o)), __int_as_float(__shfl(aw, o)));
        const bool live = i < total;
        eval(live, live ? select_bit(mo, rank) : 0, omx, omy, oa);
        // the owner's items of this round: lanes [j0, j1)
        const int j0 = max(start, base) - base, j1 = min(incl, base + 64) - base;
        const int jn = max(j1 - j0, 0);
        const int jmax = __builtin_amdgcn_readfirstlane(wave_max_i(jn));
        for (int j = 0; j < jmax; ++j) pull(min(j0 + j, 63), j < jn);
    }
}

// The three k1 taps of triple (k2, k4, k3) of a pixel, float64 geometry and sums.
template <int N, int SRC, int K>
__device__ __forceinline__ double triple_f64(const long long* S, int wq, int nrows, int row0, int mx, int my,
                                             float4 a, int k2, int k4, int k3, unsigned& bad) {
    const double a1 = a.x, a3 = a.z;
    const double A2 = (double)a.y * kInvSqrt2Hi, A4 = (double)a.w * kInvSqrt2Hi;
    constexpr double h = 0.5 * N;
    const double T1 = h * (a1 + A2 - A4 - 1.0);
    const double T2 = h * (A2 + a3 + A4 - 3.0);
    const double B2 = T2 - k2 * A2 - k4 * A4;
    const double d2 = B2 - k3 * a3;
    const double f2 = Tab<K>::ODD ? rint(d2) : floor(d2);
    const int c24 = fd_binom<N>(k2) * fd_binom<N>(k4);
    const double B1 = T1 - k2 * A2 + k4 * A4;
    const double oc = Tab<K>::ODD ? 0.0 : 0.5;
    const double u2 = d2 - f2 - oc;
    double acc = 0.0;
#pragma unroll
    for (int k1 = 0; k1 <= N; ++k1) {
        const int c124 = c24 * fd_binom<N>(k1);
        const double d1 = B1 - k1 * a1;
        const double f1 = Tab<K>::ODD ? rint(d1) : floor(d1);
        const double u1 = d1 - f1 - oc;
        const Turn t = cell_turn(u1, u2);
        const double w1 = t.swap ? u2 : u1, w2 = t.swap ? u1 : u2;
        const double v1 = t.n1 ? -w1 : w1, v2 = t.n2 ? -w2 : w2;
        const TapFrame<K> fr = tap_frame<K>(mx + (int)f1, my + (int)f2 - row0, t, wq, nrows);
        if (!fr.lo_ok) {
            bad = 1;
            continue;
        }
        const double P = interp_f64<K, SRC>(PlainRead{S}, fr, v1, v2, bad);
        const int c = c124 * fd_binom<N>(k3);
        acc = __fma_rn(((k1 + k2 + k3 + k4) & 1) ? -(double)c : (double)c, P, acc);
    }
    return acc;
}
// The same in double-double geometry with compensated sums (the split evaluation's
// bound in E when LOW < DEG).
template <int N, int SRC, int LOW, int K>
__device__ __forceinline__ cp triple_dd(const long long* S, int wq, int nrows, int row0, int mx, int my, float4 a,
                                        int k2, int k4, int k3, unsigned& bad, double& E) {
    const dd isq = {kInvSqrt2Hi, kInvSqrt2Lo};
    const double a1 = a.x, a3 = a.z;
    const dd A2 = dd_mul_d(isq, (double)a.y);
    const dd A4 = dd_mul_d(isq, (double)a.w);
    constexpr double h = 0.5 * N;
    const dd T1 = dd_mul_d(dd_add_d(dd_add(A2, dd_neg(A4)), a1 - 1.0), h);
    const dd T2 = dd_mul_d(dd_add_d(dd_add(A2, A4), a3 - 3.0), h);
    const dd D2 = dd_mul_d(A2, (double)k2), D4 = dd_mul_d(A4, (double)k4);
    const dd B2 = dd_add(T2, dd_neg(dd_add(D2, D4)));
    const dd d2 = dd_add_d(B2, -(double)k3 * a3);
    const double f2 = Tab<K>::ODD ? rint(d2.hi) : floor(d2.hi);
    const int c24 = fd_binom<N>(k2) * fd_binom<N>(k4);
    const dd B1 = dd_add(T1, dd_add(D4, dd_neg(D2)));
    const double oc = Tab<K>::ODD ? 0.0 : 0.5;
    const dd u2 = dd_add_d(d2, -(f2 + oc));
    cp acc = {0.0, 0.0};
#pragma unroll
    for (int k1 = 0; k1 <= N; ++k1) {
        const int c124 = c24 * fd_binom<N>(k1);
        const dd d1 = dd_add_d(B1, -(double)k1 * a1);
        const double f1 = Tab<K>::ODD ? rint(d1.hi) : floor(d1.hi);
        const dd u1 = dd_add_d(d1, -(f1 + oc));
        const Turn t = cell_turn(u1.hi, u2.hi);
        const dd v1 = dd_turn(t.swap, t.n1, u1, u2);
        const dd v2 = dd_turn(t.swap, t.n2, u2, u1);
        const TapFrame<K> fr = tap_frame<K>(mx + (int)f1, my + (int)f2 - row0, t, wq, nrows);
        if (!fr.lo_ok) {
            bad = 1;
            continue;
        }
        double Bk = 0.0;
        const cp P = interp_dd<K, SRC, LOW>(PlainRead{S}, fr, v1, v2, Bk, bad);
        const int c = c124 * fd_binom<N>(k3);
        const double cs = ((k1 + k2 + k3 + k4) & 1) ? -(double)c : (double)c;
        acc = cp_axpy(acc, cs, P);
        if constexpr (LOW < Tab<K>::DEG) E = __fma_rn((double)c, Bk, E);
    }
    return acc;
}

// A band's float64 mesh sum of the lane's pixel (float32-output path).
template <int N, int SRC, int K = N>
__device__ double mesh_f64_band_even(const long long* S, int wq, int nrows, int row0, int own0, int own1, int mx,
                                     int my, float4 a, bool act, int k2lo, int k2hi, unsigned& bad) {
    constexpr int NP = N + 1;
    const unsigned long long mask = act ? band_owned<N, K, false>(my, a, k2lo, k2hi, own0, own1) : 0ull;
    double acc = 0.0, v = 0.0;
    unsigned vb = 0;
    spread_items(
        mask, mx, my, a,
        [&](bool live, int t, int omx, int omy, float4 oa) {
            v = 0.0;
            vb = 0;
            if (live)
                v = triple_f64<N, SRC, K>(S, wq, nrows, row0, omx, omy, oa, k2lo + t / (NP * NP), (t / NP) % NP,
                                          t % NP, vb);
        },
        [&](int src, bool take) {
            const double x = __shfl(v, src);
            const unsigned xb = (unsigned)__shfl((int)vb, src);
            if (take) {
                acc += x;
                bad |= xb;
            }
        });
    return acc;
}
// A band's double-double mesh sum of the lane's pixel, and its split bound in E.
template <int N, int SRC, int LOW = Tab<N>::DEG, int K = N>
__device__ dd mesh_dd_band_even(const long long* S, int wq, int nrows, int row0, int own0, int own1, int mx, int my,
                                float4 a, bool act, int k2lo, int k2hi, unsigned& bad, double& E) {
    constexpr int NP = N + 1;
    const unsigned long long mask = act ? band_owned<N, K, true>(my, a, k2lo, k2hi, own0, own1) : 0ull;
    cp acc = {0.0, 0.0}, v = {0.0, 0.0};
    double ve = 0.0;
    unsigned vb = 0;
    spread_items(
        mask, mx, my, a,
        [&](bool live, int t, int omx, int omy, float4 oa) {
            v = {0.0, 0.0};
            ve = 0.0;
            vb = 0;
            if (live)
                v = triple_dd<N, SRC, LOW, K>(S, wq, nrows, row0, omx, omy, oa, k2lo + t / (NP * NP), (t / NP) % NP,
                                              t % NP, vb, ve);
        },
        [&](int src, bool take) {
            const cp x = {__shfl(v.s, src), __shfl(v.c, src)};
            const double xe = __shfl(ve, src);
            const unsigned xb = (unsigned)__shfl((int)vb, src);
            if (take) {
                const dd t = two_sum(acc.s, x.s);
                acc = {t.hi, acc.c + (t.lo + x.c)};
                E += xe;
                bad |= xb;
            }
        });
    return fast_two_sum(acc.s, acc.c);
}

template <int N, int K = N>
__device__ double finalize_f64(double acc, float4 a) {
    const double prod = ((double)a.x * (double)a.y) * ((double)a.z * (double)a.w);
    double pn = prod;
    for (int i = 1; i < N; ++i) pn *= prod;
    return acc * ((double)(1 << N) / Tab<K>::DEN) / pn;
}

// ---------------------------------------------------------------------------
// The tile kernel.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// One input sample of type DT under the boundary rule, branch-free (the coordinates are
// clamped; a zero border selects 0 afterwards), so that a run of these loads can all be
// in flight at once.
template <int DT>
__device__ __forceinline__ double sample_at(const JobDesc& A, int x, int y) {
    const bool out = x < 0 || x >= A.width || y < 0 || y >= A.height;
    const long long off = (long long)clampi(y, 0, A.height - 1) * A.in_pitch + clampi(x, 0, A.width - 1);
    double v;
    if constexpr (DT == BSF_U8) v = (double)((const unsigned char*)A.in)[off];
    else if constexpr (DT == BSF_F32) v = (double)((const float*)A.in)[off];
    else v = ((const double*)A.in)[off];
    return (out && A.border == BSF_BORDER_ZERO) ? 0.0 : v;
}
__device__ __forceinline__ long long sample_u8(const JobDesc& A, int x, int y) {
    const bool out = x < 0 || x >= A.width || y < 0 || y >= A.height;
    const long long off = (long long)clampi(y, 0, A.height - 1) * A.in_pitch + clampi(x, 0, A.width - 1);
    const long long v = ((const unsigned char*)A.in)[off];
    return (out && A.border == BSF_BORDER_ZERO) ? 0ll : v;
}

// Calls f with the sample type as a compile-time constant.
template <typename F>
__device__ __forceinline__ void with_dtype(int dt, F f) {
    if (dt == BSF_U8) f(std::integral_constant<int, BSF_U8>());
    else if (dt == BSF_F32) f(std::integral_constant<int, BSF_F32>());
    else f(std::integral_constant<int, BSF_F64>());
}

// The box elements i = tid, tid + nt, ... of a window, BATCH loads per thread in flight
// together: load(r, c) for all slots of a batch first (a slot past the end of the box
// loads a valid element and is dropped), then visit(i, value).  No division per element.
template <typename T, int BATCH = 8, typename Load, typename Visit>
__device__ __forceinline__ void load_box(const Geo& g, int tid, int nt, Load load, Visit visit) {
    const int sr = nt / g.wq, sc = nt - sr * g.wq;
    int r = tid / g.wq, c = tid - r * g.wq;
    for (int i0 = tid; i0 < g.qn; i0 += BATCH * nt) {
        T v[BATCH];
#pragma unroll
        for (int b = 0; b < BATCH; ++b) {
            v[b] = load(min(r, g.hq - 1), c);
            c += sc;
            r += sr;
            if (c >= g.wq) {
                c -= g.wq;
                ++r;
            }
        }
#pragma unroll
        for (int b = 0; b < BATCH; ++b)
            if (i0 + b * nt < g.qn) visit(i0 + b * nt, v[b]);
    }
}

// Integer grid of a sample: top = exponent e with |v| < 2^e, fine = number of fractional
// bits v needs to become an integer (v = M 2^(e-53) with M a 53-bit integer).
__device__ __forceinline__ void sample_grid(double v, int& top, int& fine) {
    if (v == 0.0) {
        top = -1100;
        fine = 0;
        return;
    }
    const unsigned long long bits = __double_as_longlong(v);
    const int ex = (int)((bits >> 52) & 0x7ff);
    unsigned long long man = bits & 0xfffffffffffffull;
    int e;  // v = man' * 2^(e - 53), man' in [2^52, 2^53)
    if (ex == 0) {  // subnormal
        e = -1022 - 52 + (64 - __clzll(man)) ;
        man <<= (53 - (64 - __clzll(man)));
    } else {
        man |= 1ull << 52;
        e = ex - 1022;
    }
    top = e;
    const int low = e - 53 + __ffsll((long long)man) - 1;  // exponent of the lowest set bit
    fine = low < 0 ? -low : 0;
}

// digit k of K (B bits each; the top digit keeps the sign) of an exact integer
__device__ __forceinline__ long long digit(long long v, int k, int K, int B) {
    if (K == 1) return v;
    if (k + 1 < K) return (v >> (k * B)) & ((1ll << B) - 1);
    return v >> (k * B);
}

__device__ __forceinline__ int wave_max_i(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return v;
}

struct Shared {
    double red[2][kMaxWaves];
    int redi[2][kMaxWaves];
    int item;
};

// Order 3: the thread pair of a pixel adds its two partial tap sums, in a fixed order
// (first half + second half), and merges its error flags; the first thread keeps them.
template <int SPLIT>
__device__ __forceinline__ void combine_halves(dd& acc, unsigned& bad) {
    if constexpr (SPLIT == 2) {
        __shared__ double part[2][kThreads];
        __shared__ unsigned partbad[kThreads];
        const int pix = threadIdx.x % kThreads;
        __syncthreads();
        if (threadIdx.x >= kThreads) {
            part[0][pix] = acc.hi;
            part[1][pix] = acc.lo;
            partbad[pix] = bad;
        }
        __syncthreads();
        if (threadIdx.x < kThreads) {
            acc = dd_add(acc, dd{part[0][pix], part[1][pix]});
            bad |= partbad[pix];
        }
    }
}

// Filter one 16x16 tile of job A (index `job`) with the window in S.  blocks (tier 2, when
// tier 3 follows): tier 3 takes 2x2 blocks of tiles; one word per item (job's item_base +
// the block's first tile), cleared before tier 1, holds the block's tiles that go there
// (bit (ty & 1) * 2 + (tx & 1)), and a tile that does not fit sets its bit and pushes the
// block, (job, first tile), when it is the block's first bit.
// LAT = 1: tiles whose pixels all have integer a1, a3 take the combined-tap form of the
// mesh.  LAT = 0: every tile takes the per-tap form (the single-job tier 1 leaves the tiles
// whose pixels all have integer a1, a3 to lattice_tile_kernel, so that its per-tap kernel
// holds no code of the other form).
template <int N, int PATH, int TK = N, int LAT = 1>
__device__ __forceinline__ void process_tile(const JobDesc A, int job, int tile, const Launch L, long long* S,
                                             Shared& sh_, unsigned* blocks = nullptr) {
    auto& red = sh_.red;
    auto& redi = sh_.redi;
    constexpr int SPLIT = split_of<N, PATH>(), NT = threads_of<N, PATH>(), NW = NT / 64;
    const int tid = threadIdx.x;
    const int pix = tid % kThreads, half = tid / kThreads;  // the pixel, and the thread's share of its taps
    const int k2lo = SPLIT == 1 ? 0 : half * (N + 1) / 2, k2hi = SPLIT == 1 ? N : (half + 1) * (N + 1) / 2 - 1;
    __syncthreads();  // the previous item of this workgroup is done with S and the scratch
    const int tx = tile % A.tiles_x, ty = tile / A.tiles_x;
    const int t1 = tx * kTile, t2 = ty * kTile;
    const int tw = std::min(kTile, A.width - t1), th = std::min(kTile, A.height - t2);
    const int px = pix % kTile, py = pix / kTile;
    const int m1 = t1 + px, m2 = t2 + py;
    const bool inside = px < tw && py < th;

    // 1. the tile's scale vectors and its reach
    float4 a = make_float4(0.f, 0.f, 0.f, 0.f);
    bool valid = false;
    if (inside) {
        a = *reinterpret_cast<const float4*>(A.scales + 4 * ((long long)m2 * A.scale_pitch + m1));
        valid = true;
        const float av[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
        for (int d = 0; d < 4; ++d) valid = valid && (av[d] >= (float)kScaleMin) && (av[d] <= (float)kScaleMax);
        if (!valid) atomicOr(A.err, kErrScale);
    }
    // the combined-tap form is taken tile by tile (every call path then agrees bitwise)
    bool tile_lat = false;
    if constexpr (LAT == 1) tile_lat = __syncthreads_and(!inside || (valid && lattice_scales(a))) != 0;
    double R1 = valid ? reach1(N, a.x, a.y, a.w) : 0.0;
    double R2 = valid ? reach1(N, a.z, a.y, a.w) : 0.0;
    R1 = wave_max(R1);
    R2 = wave_max(R2);
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = R1;
        red[1][tid >> 6] = R2;
    }
    __syncthreads();
    R1 = red[0][0];
    R2 = red[1][0];
#pragma unroll
    for (int wv = 1; wv < NW; ++wv) {
        R1 = fmax(R1, red[0][wv]);
        R2 = fmax(R2, red[1][wv]);
    }

    // 2. the restart window
    const Window w = tile_window<N, TK>(t1, t2, tw, th, R1, R2);
    const long long need = window_elems(w);
    const double nan = __builtin_nan("");
    auto store = [&](double v) {
        if (!inside || half) return;
        const long long off = (long long)m2 * A.out_pitch + m1;
        if (PATH == BSF_PATH_F64)
            ((double*)A.out)[off] = v;
        else
            ((float*)A.out)[off] = (float)v;
    };
    if (need > L.lds_cap) {
        if (L.dbg_window) {
            if (tid == 0) {
                L.dbg_geom[0] = w.x0; L.dbg_geom[1] = w.y0; L.dbg_geom[2] = w.wq; L.dbg_geom[3] = w.hq;
            }
            return;
        }
        if (L.push_cap > 0) {  // a later launch with more room takes the tile
            if (tid == 0) {
                int item = tile;
                bool push = true;
                if (blocks) {  // by 2x2 blocks: the block's first flagged tile pushes it
                    item = (ty & ~1) * A.tiles_x + (tx & ~1);
                    push = atomicOr(blocks + A.item_base + item, 1u << ((ty & 1) * 2 + (tx & 1))) == 0u;
                }
                if (push) {
                    const unsigned k = atomicAdd(L.push_count, 1u);
                    if (k < (unsigned)L.push_cap) L.push_list[k] = make_int2(job, item);
                    else atomicOr(A.err, kErrWindow);
                }
            }
            return;
        }
        if (tid == 0) atomicOr(A.err, kErrWindow);
        store(nan);
        return;
    }
    const Geo g = {w.wq, w.hq, w.wq * w.hq};
    const int ntri = (g.hq * (g.hq - 1)) / 2;

    const bool cen = !L.dbg_window || L.dbg_geom[4];
    const int cc = t1 + tw / 2 - w.x0, rc = t2 + th / 2 - w.y0;  // centre of the tile's own extent
    const int mx = m1 - w.x0, my = m2 - w.y0;

    if constexpr (PATH == BSF_PATH_F32_TILED) {
        // float32 output: stage 1 in float64 (rounded running sums of the samples as they
        // are), the mesh in float64 from the window as it stands -- no integer grid, no
        // digits.  The error is the mesh's cancellation times a few float64 roundings.
        double* Sd = reinterpret_cast<double*>(S);
        with_dtype(A.in_dtype, [&](auto dt) {
            constexpr int DT = decltype(dt)::value;
            load_box<double>(g, tid, NT, [&](int r, int c) { return sample_at<DT>(A, w.x0 + c, w.y0 + r); },
                             [&](int i, double v) { Sd[i] = v; });
        });
        for (int i = tid; i < ntri; i += NT) Sd[g.qn + i] = 0.0;
        __syncthreads();
        unsigned unused = 0;
        preintegrate_window<N>(Sd, g, cen, cc, rc, 0, unused);
        __syncthreads();
        if (L.dbg_window) {  // the window as float64 bit patterns
            if (tid == 0) {
                L.dbg_geom[0] = w.x0; L.dbg_geom[1] = w.y0; L.dbg_geom[2] = w.wq; L.dbg_geom[3] = w.hq;
                L.dbg_geom[5] = 0;
                L.dbg_geom[6] = 0;
            }
            if ((long long)g.qn <= L.dbg_cap)
                for (int i = tid; i < g.qn; i += NT) L.dbg_window[i] = S[i];
            return;
        }
        unsigned bad = 0;
        dd m = {0.0, 0.0};
        // a wave whose pixels all have integer a1, a3 combines each pair's (k1, k3) taps
        // a tile whose pixels all have integer a1, a3 combines each pair's (k1, k3) taps
        const bool lat = tile_lat;
        if (inside && valid) {
            if constexpr (LAT == 1)
                m.hi = lat ? mesh_f64_lat<N, SRC_DBL, TK>(S, g.wq, g.hq, mx, my, a, k2lo, k2hi, bad)
                           : mesh_f64<N, SRC_DBL, TK>(S, g.wq, g.hq, mx, my, a, k2lo, k2hi, bad);
            else
                m.hi = mesh_f64<N, SRC_DBL, TK>(S, g.wq, g.hq, mx, my, a, k2lo, k2hi, bad);
        }
        combine_halves<SPLIT>(m, bad);
        if (!inside || half) return;
        if (!valid) {
            store(nan);
            return;
        }
        double s = finalize_f64<N, TK>(m.hi, a);
        if (bad) {
            atomicOr(A.err, kErrWindow);
            s = nan;
        }
        store(s);
        return;
    }

    // 3. an exact integer grid for the window: samples become v * 2^sh with at most 53
    //    significant bits (finer bits than 2^-53 of the window maximum are rounded)
    //    (u8 samples: integers below 2^8, no scan)
    int top = A.in_dtype == BSF_U8 ? 8 : -1100, fine = 0;
    if (A.in_dtype != BSF_U8)
        load_box<double, 1>(
            g, tid, NT,
            [&](int r, int c) {
                return A.in_dtype == BSF_F32 ? sample_at<BSF_F32>(A, w.x0 + c, w.y0 + r)
                                             : sample_at<BSF_F64>(A, w.x0 + c, w.y0 + r);
            },
            [&](int, double v) {
                int t_, f_;
                sample_grid(v, t_, f_);
                top = max(top, t_);
                fine = max(fine, f_);
            });
    top = wave_max_i(top);
    fine = wave_max_i(fine);
    __syncthreads();
    if ((tid & 63) == 0) {
        redi[0][tid >> 6] = top;
        redi[1][tid >> 6] = fine;
    }
    __syncthreads();
    top = redi[0][0];
    fine = redi[1][0];
#pragma unroll
    for (int wv = 1; wv < NW; ++wv) {
        top = max(top, redi[0][wv]);
        fine = max(fine, redi[1][wv]);
    }
    const int sh = (top + fine > 53) ? 53 - top : fine;
    const int bits = max(top + sh, 1);

    // 4. stage 1 + mesh, on K base-2^B digits of the samples when the running sums of
    //    the whole samples would leave int64 (the filter is linear in the image)
    dd acc_dd = {0.0, 0.0};
    double acc_f = 0.0;
    unsigned bad = 0;
    bool done = false;
    for (int K = 1; K <= 4 && !done; ++K) {
        const int B = (bits + K - 1) / K;
        acc_dd = {0.0, 0.0};
        acc_f = 0.0;
        bool overflowed = false;
        for (int k = 0; k < K; ++k) {
            __syncthreads();  // the previous digit's mesh has finished reading the window
            // (u8 samples four loads in flight per thread; the other types one at a time: the
            // kernel is at its register cap, and wider batches or one copy per type spilled)
            if (A.in_dtype == BSF_U8)
                load_box<long long, 4>(
                    g, tid, NT, [&](int r, int c) { return sample_u8(A, w.x0 + c, w.y0 + r); },
                    [&](int i, long long v) { S[i] = digit(v, k, K, B); });
            else
                load_box<long long, 1>(
                    g, tid, NT,
                    [&](int r, int c) {
                        const double v = A.in_dtype == BSF_F32 ? sample_at<BSF_F32>(A, w.x0 + c, w.y0 + r)
                                                               : sample_at<BSF_F64>(A, w.x0 + c, w.y0 + r);
                        return (long long)rint(ldexp(v, sh));
                    },
                    [&](int i, long long v) { S[i] = digit(v, k, K, B); });
            for (int i = tid; i < ntri; i += NT) S[g.qn + i] = 0;
            __syncthreads();
            unsigned ovf = 0;
            preintegrate_window<N>(S, g, cen, cc, rc, (K == 1 ? bits : B) + 1, ovf);
            ovf = __syncthreads_or(ovf);
            if (L.dbg_window) {
                if (tid == 0) {
                    L.dbg_geom[0] = w.x0; L.dbg_geom[1] = w.y0; L.dbg_geom[2] = w.wq; L.dbg_geom[3] = w.hq;
                    L.dbg_geom[5] = (int)ovf;
                    L.dbg_geom[6] = sh;
                }
                if ((long long)g.qn <= L.dbg_cap)
                    for (int i = tid; i < g.qn; i += NT) L.dbg_window[i] = S[i];
                return;
            }
            if (ovf) {
                overflowed = true;
                break;
            }
            // when every value the mesh reads is below 2^exact_bits, hold the box as exact
            // doubles: the coefficient sums then need one part and no conversions per tap
            unsigned long long mag = 0;
            for (int i = tid; i < g.qn; i += NT) {
                const long long v = S[i];
                mag |= (unsigned long long)(v < 0 ? -v : v);
            }
            constexpr int kExact = exact_bits<TK>();  // folded at compile time
            const bool fast = !__syncthreads_or((mag >> kExact) != 0ull);
            // a tile whose pixels all have integer a1, a3 combines each pair's (k1, k3) taps
            // (mesh_dd_lat) where the combined window stays exact
            bool lat = false;
            if constexpr (LAT == 1)
                lat = tile_lat && !__syncthreads_or((mag >> (fast ? kExact - 2 * N : 62 - 2 * N)) != 0ull);
            if (fast) {
                for (int i = tid; i < g.qn; i += NT) reinterpret_cast<double*>(S)[i] = (double)S[i];
                __syncthreads();
            }
            bool tried = false, redo = false;
            // The split is tried by whole waves whose pixels all have a geometric-mean
            // scale of at least split_min_volume^(1/4): the bound's ratio to |s| falls
            // roughly as that scale's 6th (order 2) or 7th (order 3) power and holds there
            // as a rule; below, a wave would mostly pay for both evaluations.
            const bool wave_split =
                __all(!(inside && valid) || (double)a.x * a.y * a.z * a.w >= split_min_volume<TK>()) != 0;
            if (inside && valid) {
                const double wk = ldexp(1.0, k * B);
                if (PATH == BSF_PATH_F64) {
                    dd m;
                    double E = 0.0;
                    bool done_m = false;
                    if constexpr (split_low<TK>() < Tab<TK>::DEG) {
                        if (K == 1 && wave_split) {
                            tried = true;
                            // split evaluation; a pixel whose bound on the plain parts' error,
                            // 2^-47 E, exceeds 2^-44 |s| is evaluated again, compensated
                            constexpr int LOW = split_low<TK>();
                            if (LAT == 1 && lat)
                                m = fast ? mesh_dd_lat<N, SRC_DBL, LOW, TK>(S, g.wq, g.hq, mx, my, a, k2lo, k2hi, bad, E)
                                         : mesh_dd_lat<N, SRC_INT, LOW, TK>(S, g.wq, g.hq, mx, my, a, k2lo, k2hi, bad, E);
                            else
                                m = fast ? mesh_dd<N, SRC_DBL, LOW, TK>(S, g.wq, g.hq, mx, my, a, k2lo, k2hi, bad, E)
                                         : mesh_dd<N, SRC_INT, LOW, TK>(S, g.wq, g.hq, mx, my, a, k2lo, k2hi, bad, E);
                            done_m = E <= 8.0 * fabs(m.hi);
                            redo = !done_m;
                        }
                    }
                    if (!done_m) {
                        constexpr int DEG = Tab<TK>::DEG;
                        if (LAT == 1 && lat)
                            m = fast ? mesh_dd_lat<N, SRC_DBL, DEG, TK>(S, g.wq, g.hq, mx, my, a, k2lo, k2hi, bad, E)
                                     : mesh_dd_lat<N, SRC_INT, DEG, TK>(S, g.wq, g.hq, mx, my, a, k2lo, k2hi, bad, E);
                        else
                            m = fast ? mesh_dd<N, SRC_DBL, DEG, TK>(S, g.wq, g.hq, mx, my, a, k2lo, k2hi, bad, E)
                                     : mesh_dd<N, SRC_INT, DEG, TK>(S, g.wq, g.hq, mx, my, a, k2lo, k2hi, bad, E);
                    }
                    acc_dd = dd_add(acc_dd, dd_mul_d(m, wk));
                } else {
                    const double m = fast ? mesh_f64<N, SRC_DBL, TK>(S, g.wq, g.hq, mx, my, a, k2lo, k2hi, bad)
                                          : mesh_f64<N, SRC_INT, TK>(S, g.wq, g.hq, mx, my, a, k2lo, k2hi, bad);
                    acc_f = __fma_rn(m, wk, acc_f);
                }
            }
            if (L.stats) {  // pixels evaluated split, and those evaluated again (one atomic per wave)
                const int t = __popcll(__ballot(tried)), r = __popcll(__ballot(redo));
                if ((tid & 63) == 0 && t) {
                    atomicAdd(L.stats, (unsigned long long)t);
                    if (r) atomicAdd(L.stats + 1, (unsigned long long)r);
                }
            }
        }
        done = !overflowed;
    }
    if (!done) {
        if (tid == 0) atomicOr(A.err, kErrRange);
        store(nan);
        return;
    }
    if (PATH == BSF_PATH_F64) {
        combine_halves<SPLIT>(acc_dd, bad);
    } else {
        dd t = {acc_f, 0.0};
        combine_halves<SPLIT>(t, bad);
        acc_f = t.hi;
    }
    if (!inside || half) return;
    if (!valid) {
        store(nan);
        return;
    }
    double s = (PATH == BSF_PATH_F64) ? finalize_dd<N, TK>(acc_dd, a) : finalize_f64<N, TK>(acc_f, a);
    s = ldexp(s, -sh);
    if (bad) {
        atomicOr(A.err, kErrWindow);
        s = nan;
    }
    store(s);
}

// Tier 3: the flagged 16x16 tiles of one 2x2 block of tiles (bit s of `mask`: the tile
// at (tx0 + (s & 1), ty0 + (s >> 1)), tx0, ty0 even, the block's first tile `lead`), whose
// windows exceed any workgroup's LDS, filtered from one restart window over their common
// extent, pre-integrated in S, a slice of global scratch: stage 1 runs once for up to four
// tiles (the window of the extent is little larger than one tile's, the reach dominating
// both).  The float32-output path loads the window and runs the row step of stage 1 in one
// pass (load_rows_runsum).  The mesh reads the window from LB, band_cap elements of LDS,
// in bands of rows, each band's triples spread evenly over the wave (mesh_dd_band_even,
// mesh_f64_band_even); the float64 path keeps each pixel's sums over the digit passes in
// LB's last 8 NT doubles.  Otherwise as process_tile.
template <int N, int PATH, int TK = N>
__device__ __forceinline__ void process_block(const JobDesc A, int lead, unsigned mask, const Launch L, long long* S,
                                              Shared& sh_, long long* LB, long long band_cap) {
    auto& red = sh_.red;
    auto& redi = sh_.redi;
    constexpr int SPLIT = split_of<N, PATH>(), NT = threads_of<N, PATH>(), NW = NT / 64;
    const int tid = threadIdx.x;
    const int pix = tid % kThreads, half = tid / kThreads;
    const int k2lo = SPLIT == 1 ? 0 : half * (N + 1) / 2, k2hi = SPLIT == 1 ? N : (half + 1) * (N + 1) / 2 - 1;
    __syncthreads();  // the previous item of this workgroup is done with S, LB and the scratch
    const int tx0 = lead % A.tiles_x, ty0 = lead / A.tiles_x;
    const int px = pix % kTile, py = pix / kTile;
    // the thread's pixel in sub-tile s
    struct Px {
        int m1, m2;
        bool inside, valid;
        float4 a;
    };
    auto pixel_of = [&](int s) {
        Px q;
        const int t1 = (tx0 + (s & 1)) * kTile, t2 = (ty0 + (s >> 1)) * kTile;
        q.m1 = t1 + px;
        q.m2 = t2 + py;
        q.inside = q.m1 < A.width && q.m2 < A.height;
        q.a = make_float4(0.f, 0.f, 0.f, 0.f);
        q.valid = false;
        if (q.inside) {
            q.a = *reinterpret_cast<const float4*>(A.scales + 4 * ((long long)q.m2 * A.scale_pitch + q.m1));
            const float av[4] = {q.a.x, q.a.y, q.a.z, q.a.w};
            q.valid = true;
#pragma unroll
            for (int d = 0; d < 4; ++d) q.valid = q.valid && (av[d] >= (float)kScaleMin) && (av[d] <= (float)kScaleMax);
        }
        return q;
    };
    auto store = [&](const Px& q, double v) {
        if (!q.inside || half) return;
        const long long off = (long long)q.m2 * A.out_pitch + q.m1;
        if (PATH == BSF_PATH_F64)
            ((double*)A.out)[off] = v;
        else
            ((float*)A.out)[off] = (float)v;
    };

    // 1. the scale vectors of the flagged tiles, their reach and their common extent
    double R1 = 0.0, R2 = 0.0;
    int ex0 = A.width, ey0 = A.height, ex1 = 0, ey1 = 0;
    for (int s = 0; s < 4; ++s) {
        if (!((mask >> s) & 1u)) continue;
        const int t1 = (tx0 + (s & 1)) * kTile, t2 = (ty0 + (s >> 1)) * kTile;
        ex0 = min(ex0, t1);
        ey0 = min(ey0, t2);
        ex1 = max(ex1, min(t1 + kTile, A.width));
        ey1 = max(ey1, min(t2 + kTile, A.height));
        const Px q = pixel_of(s);
        if (q.inside && !q.valid && !half) atomicOr(A.err, kErrScale);
        if (q.valid) {
            R1 = fmax(R1, reach1(N, q.a.x, q.a.y, q.a.w));
            R2 = fmax(R2, reach1(N, q.a.z, q.a.y, q.a.w));
        }
    }
    R1 = wave_max(R1);
    R2 = wave_max(R2);
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = R1;
        red[1][tid >> 6] = R2;
    }
    __syncthreads();
    R1 = red[0][0];
    R2 = red[1][0];
#pragma unroll
    for (int wv = 1; wv < NW; ++wv) {
        R1 = fmax(R1, red[0][wv]);
        R2 = fmax(R2, red[1][wv]);
    }

    // 2. the restart window of the extent
    const Window w = tile_window<N, TK>(ex0, ey0, ex1 - ex0, ey1 - ey0, R1, R2);
    const long long need = window_elems(w);
    const double nan = __builtin_nan("");
    auto store_all = [&](double v) {
        for (int s = 0; s < 4; ++s)
            if ((mask >> s) & 1u) store(pixel_of(s), v);
    };
    if (need > L.lds_cap) {
        if (tid == 0) atomicOr(A.err, kErrWindow);
        store_all(nan);
        return;
    }
    const Geo g = {w.wq, w.hq, w.wq * w.hq};
    const int ntri = (g.hq * (g.hq - 1)) / 2;
    const int cc = (ex0 + ex1) / 2 - w.x0, rc = (ey0 + ey1) / 2 - w.y0;  // centre of the extent

    // Runs body(src, nrows, row0, own0, own1) -- by every thread of the workgroup -- once per
    // band of the window: rows row0 .. row0 + nrows - 1 copied from S to LB, owning the
    // triples whose stencil starts in rows [own0, own1) (the first band also those above
    // the window, the last those below, which the taps then flag).  Consecutive bands
    // overlap by the stencil's height.  A window too wide for bands of 8 owned rows is read
    // where it lies, as one band.
    static_assert(PATH != BSF_PATH_F64 || 8 * NT <= bsf_plan::kBandTail, "the band tail holds the digit sums");
    const long long band_elems = PATH == BSF_PATH_F64 ? band_cap - 8 * NT : band_cap;
    auto over_bands = [&](auto&& body) {
        constexpr int span = stencil_hi<TK>() - stencil_lo<TK>();
        const int rows_cap = band_elems > 0 ? (int)(band_elems / g.wq) : 0;
        const int own = rows_cap - span;
        if (own < 8) {
            body((const long long*)S, g.hq, 0, INT_MIN, INT_MAX);
            return;
        }
        for (int r0 = 0;; r0 += own) {
            const bool last = r0 + own >= g.hq - span;
            const int nrows = min(rows_cap, g.hq - r0);
            __syncthreads();  // the previous band's taps are done with LB
            const long long* src = S + (long long)r0 * g.wq;
            for (int i = tid; i < nrows * g.wq; i += NT) LB[i] = src[i];
            __syncthreads();
            body((const long long*)LB, nrows, r0, r0 == 0 ? INT_MIN : r0, last ? INT_MAX : r0 + own);
            if (last) break;
        }
    };

    if constexpr (PATH == BSF_PATH_F32_TILED) {
        // float32 output (as process_tile): float64 running sums of the samples as they are
        double* Sd = reinterpret_cast<double*>(S);
        with_dtype(A.in_dtype, [&](auto dt) {
            constexpr int DT = decltype(dt)::value;
            load_rows_runsum<N, kRowRun>(Sd, g, cc, [&](int r, int c) { return sample_at<DT>(A, w.x0 + c, w.y0 + r); });
        });
        __syncthreads();
        unsigned unused = 0;
        preintegrate_window_n<N, false, 8>(Sd, g, true, cc, rc, unused, true);
        // band by band, the flagged sub-tiles in turn: each band is copied once for all four
        double msum[4] = {0.0, 0.0, 0.0, 0.0};
        unsigned bads[4] = {0u, 0u, 0u, 0u};
        over_bands([&](const long long* src, int nrows, int row0, int own0, int own1) {
#pragma unroll 1
            for (int s = 0; s < 4; ++s) {  // one copy of the mesh code
                if (!((mask >> s) & 1u)) continue;
                const Px q = pixel_of(s);
                unsigned bad = 0;
                const double part = mesh_f64_band_even<N, SRC_DBL, TK>(src, g.wq, nrows, row0, own0, own1, q.m1 - w.x0,
                                                                       q.m2 - w.y0, q.a, q.valid, k2lo, k2hi, bad);
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (s == k) {
                        msum[k] += part;
                        bads[k] |= bad;
                    }
            }
        });
        for (int s = 0; s < 4; ++s) {
            if (!((mask >> s) & 1u)) continue;
            const Px q = pixel_of(s);
            unsigned bad = bads[s];
            dd m = {msum[s], 0.0};
            combine_halves<SPLIT>(m, bad);
            if (!q.inside || half) continue;
            double v = q.valid ? finalize_f64<N, TK>(m.hi, q.a) : nan;
            if (bad) {
                atomicOr(A.err, kErrWindow);
                v = nan;
            }
            store(q, v);
        }
        return;
    }

    // 3. the exact integer grid of the window (as process_tile)
    int top = A.in_dtype == BSF_U8 ? 8 : -1100, fine = 0;
    if (A.in_dtype != BSF_U8)
        load_box<double, 1>(
            g, tid, NT,
            [&](int r, int c) {
                return A.in_dtype == BSF_F32 ? sample_at<BSF_F32>(A, w.x0 + c, w.y0 + r)
                                             : sample_at<BSF_F64>(A, w.x0 + c, w.y0 + r);
            },
            [&](int, double v) {
                int t_, f_;
                sample_grid(v, t_, f_);
                top = max(top, t_);
                fine = max(fine, f_);
            });
    top = wave_max_i(top);
    fine = wave_max_i(fine);
    __syncthreads();
    if ((tid & 63) == 0) {
        redi[0][tid >> 6] = top;
        redi[1][tid >> 6] = fine;
    }
    __syncthreads();
    top = redi[0][0];
    fine = redi[1][0];
#pragma unroll
    for (int wv = 1; wv < NW; ++wv) {
        top = max(top, redi[0][wv]);
        fine = max(fine, redi[1][wv]);
    }
    const int sh = (top + fine > 53) ? 53 - top : fine;
    const int bits = max(top + sh, 1);

    // 4. stage 1 + the tiles' meshes, on K digits when int64 would overflow; the sums of
    //    sub-tile s in acc[s][tid] (hi) and acc[s][NT + tid] (lo) of LB's tail
    double* acc = reinterpret_cast<double*>(LB + band_elems);
    unsigned badm = 0;  // bit s: a tap of sub-tile s fell outside the window
    bool done = false;
    for (int K = 1; K <= 4 && !done; ++K) {
        const int B = (bits + K - 1) / K;
        bool overflowed = false;
        for (int k = 0; k < K; ++k) {
            __syncthreads();  // the previous digit's meshes have finished reading the window
            if (A.in_dtype == BSF_U8)
                load_box<long long, 4>(
                    g, tid, NT, [&](int r, int c) { return sample_u8(A, w.x0 + c, w.y0 + r); },
                    [&](int i, long long v) { S[i] = digit(v, k, K, B); });
            else
                load_box<long long, 1>(
                    g, tid, NT,
                    [&](int r, int c) {
                        const double v = A.in_dtype == BSF_F32 ? sample_at<BSF_F32>(A, w.x0 + c, w.y0 + r)
                                                               : sample_at<BSF_F64>(A, w.x0 + c, w.y0 + r);
                        return (long long)rint(ldexp(v, sh));
                    },
                    [&](int i, long long v) { S[i] = digit(v, k, K, B); });
            for (int i = tid; i < ntri; i += NT) S[g.qn + i] = 0;
            __syncthreads();
            unsigned ovf = 0;
            preintegrate_window<N>(S, g, true, cc, rc, (K == 1 ? bits : B) + 1, ovf);
            ovf = __syncthreads_or(ovf);
            if (ovf) {
                overflowed = true;
                break;
            }
            unsigned long long mag = 0;
            for (int i = tid; i < g.qn; i += NT) {
                const long long v = S[i];
                mag |= (unsigned long long)(v < 0 ? -v : v);
            }
            constexpr int kExact = exact_bits<TK>();
            const bool fast = !__syncthreads_or((mag >> kExact) != 0ull);
            if (fast) {
                for (int i = tid; i < g.qn; i += NT) reinterpret_cast<double*>(S)[i] = (double)S[i];
                __syncthreads();
            }
            const double wk = ldexp(1.0, k * B);
            for (int s = 0; s < 4; ++s) {
                if (!((mask >> s) & 1u)) continue;
                const Px q = pixel_of(s);
                const int mx = q.m1 - w.x0, my = q.m2 - w.y0;
                const bool act = q.valid;
                unsigned bad = 0;
                bool tried = false, redo = false;
                const bool wave_split =
                    __all(!act || (double)q.a.x * q.a.y * q.a.z * q.a.w >= split_min_volume<TK>()) != 0;
                constexpr int LOW = split_low<TK>(), DEG = Tab<TK>::DEG;
                const bool try_split = LOW < DEG && K == 1 && wave_split;
                dd m = {0.0, 0.0};
                double E = 0.0;
                over_bands([&](const long long* src, int nrows, int row0, int own0, int own1) {
                    dd part;
                    if (try_split)
                        part = fast ? mesh_dd_band_even<N, SRC_DBL, LOW, TK>(src, g.wq, nrows, row0, own0, own1, mx, my,
                                                                             q.a, act, k2lo, k2hi, bad, E)
                                    : mesh_dd_band_even<N, SRC_INT, LOW, TK>(src, g.wq, nrows, row0, own0, own1, mx, my,
                                                                             q.a, act, k2lo, k2hi, bad, E);
                    else
                        part = fast ? mesh_dd_band_even<N, SRC_DBL, DEG, TK>(src, g.wq, nrows, row0, own0, own1, mx, my,
                                                                             q.a, act, k2lo, k2hi, bad, E)
                                    : mesh_dd_band_even<N, SRC_INT, DEG, TK>(src, g.wq, nrows, row0, own0, own1, mx, my,
                                                                             q.a, act, k2lo, k2hi, bad, E);
                    if (act) m = dd_add(m, part);
                });
                // the split evaluation's bound (see process_tile): too large, evaluated again compensated
                tried = act && try_split;
                redo = tried && !(E <= 8.0 * fabs(m.hi));
                if (__syncthreads_or(redo)) {
                    dd m2 = {0.0, 0.0};
                    over_bands([&](const long long* src, int nrows, int row0, int own0, int own1) {
                        const dd part =
                            fast ? mesh_dd_band_even<N, SRC_DBL, DEG, TK>(src, g.wq, nrows, row0, own0, own1, mx, my, q.a,
                                                                          redo, k2lo, k2hi, bad, E)
                                 : mesh_dd_band_even<N, SRC_INT, DEG, TK>(src, g.wq, nrows, row0, own0, own1, mx, my, q.a,
                                                                          redo, k2lo, k2hi, bad, E);
                        if (redo) m2 = dd_add(m2, part);
                    });
                    if (redo) m = m2;
                }
                badm |= bad ? (1u << s) : 0u;
                dd t = k == 0 ? dd{0.0, 0.0} : dd{acc[(2 * s) * NT + tid], acc[(2 * s + 1) * NT + tid]};
                if (act) t = dd_add(t, dd_mul_d(m, wk));
                acc[(2 * s) * NT + tid] = t.hi;
                acc[(2 * s + 1) * NT + tid] = t.lo;
                if (L.stats) {
                    const int nt_ = __popcll(__ballot(tried)), nr_ = __popcll(__ballot(redo));
                    if ((tid & 63) == 0 && nt_) {
                        atomicAdd(L.stats, (unsigned long long)nt_);
                        if (nr_) atomicAdd(L.stats + 1, (unsigned long long)nr_);
                    }
                }
            }
        }
        done = !overflowed;
    }
    if (!done) {
        if (tid == 0) atomicOr(A.err, kErrRange);
        store_all(nan);
        return;
    }
    for (int s = 0; s < 4; ++s) {
        if (!((mask >> s) & 1u)) continue;
        const Px q = pixel_of(s);
        if (!q.inside) continue;
        double v = q.valid ? ldexp(finalize_dd<N, TK>(dd{acc[(2 * s) * NT + tid], acc[(2 * s + 1) * NT + tid]}, q.a), -sh)
                           : nan;
        if ((badm >> s) & 1u) {
            atomicOr(A.err, kErrWindow);
            v = nan;
        }
        store(q, v);
    }
}

// Whether pixel `pix` of a tile lets the tile take the combined-tap mesh: outside the
// image, or valid scales with integer a1 and a3.
__device__ __forceinline__ bool lattice_pixel(const JobDesc& A, int tile, int pix) {
    const int m1 = (tile % A.tiles_x) * kTile + pix % kTile, m2 = (tile / A.tiles_x) * kTile + pix / kTile;
    if (m1 >= A.width || m2 >= A.height) return true;
    const float4 a = *reinterpret_cast<const float4*>(A.scales + 4 * ((long long)m2 * A.scale_pitch + m1));
    const float av[4] = {a.x, a.y, a.z, a.w};
    bool q = true;
#pragma unroll
    for (int d = 0; d < 4; ++d) q = q && (av[d] >= (float)kScaleMin) && (av[d] <= (float)kScaleMax);
    return q && lattice_scales(a);
}

// The window of the batch kernels, addressed through the kernel's dynamic LDS symbol.
extern __shared__ long long g_lds[];

// Tier 1 of a single job: one workgroup per tile.
template <int N, int PATH, int TK = N>
__global__ __launch_bounds__((threads_of<N, PATH>())) __attribute__((amdgpu_waves_per_eu(N < 3 ? 2 : 1))) void tile_kernel(
    JobDesc A, Launch L) {
    extern __shared__ long long S[];
    __shared__ Shared sh;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    if (__syncthreads_and(lattice_pixel(A, tile, threadIdx.x % kThreads))) return;  // lattice_tile_kernel's
    process_tile<N, PATH, TK, 0>(A, 0, tile, L, S, sh);
}

// Tier 1 of the tiles tile_kernel leaves: those whose pixels all have integer a1, a3.
// Persistent workgroups; workgroup b takes the tiles of dispatch index b, b + G, b + 2G, ...
// (G the grid, a multiple of 8, so that the XCD order of tile_kernel holds).  One load per
// thread reads the first pixel of up to a workgroup's width of its tiles at once -- a tile
// can qualify only if that pixel does -- and only those candidates are checked in full and
// filtered.  Where no tile qualifies (real scales) the launch costs one load per tile.
// all != 0 (images of at most one tile per CU): every tile, each taking the form its scales
// allow, so that such an image needs one tier-1 launch.
template <int N, int PATH, int TK = N>
__global__ __launch_bounds__((threads_of<N, PATH>())) __attribute__((amdgpu_waves_per_eu(N < 3 && PATH == BSF_PATH_F32_TILED ? 2 : 1))) void lattice_tile_kernel(
    JobDesc A, Launch L, int all) {
    extern __shared__ long long S[];
    __shared__ Shared sh;
    constexpr int NT = threads_of<N, PATH>(), NW = NT / 64;
    auto* ballots = reinterpret_cast<unsigned long long*>(sh.red[0]);  // NW words, free between tiles
    const int tiles = A.tiles_x * A.tiles_y;
    const int pix = threadIdx.x % kThreads;
    const int per = tiles > (int)blockIdx.x ? (tiles - (int)blockIdx.x + (int)gridDim.x - 1) / (int)gridDim.x : 0;
    if (all) {
        for (int k = 0; k < per; ++k)
            process_tile<N, PATH, TK, 1>(A, 0, xcd_tile((int)blockIdx.x + k * (int)gridDim.x, tiles), L, S, sh);
        return;
    }
    for (int c0 = 0; c0 < per; c0 += NT) {
        const int k = c0 + (int)threadIdx.x;
        const bool cand = k < per && lattice_pixel(A, xcd_tile((int)blockIdx.x + k * (int)gridDim.x, tiles), 0);
        const unsigned long long b = __ballot(cand);
        __syncthreads();  // the previous chunk's tiles are done with sh
        if ((threadIdx.x & 63) == 0) ballots[threadIdx.x >> 6] = b;
        __syncthreads();
        unsigned long long bw[NW];
#pragma unroll
        for (int wv = 0; wv < NW; ++wv) bw[wv] = ballots[wv];
        for (int wv = 0; wv < NW; ++wv)
            for (unsigned long long m = bw[wv]; m; m &= m - 1) {
                const int tile = xcd_tile((int)blockIdx.x + (c0 + wv * 64 + __ffsll((long long)m) - 1) * (int)gridDim.x, tiles);
                if (__syncthreads_and(lattice_pixel(A, tile, pix))) process_tile<N, PATH, TK, 1>(A, 0, tile, L, S, sh);
            }
    }
}

// Test aid: stage 1 of one tile.
template <int N, int PATH, int TK = N>
__global__ __launch_bounds__((threads_of<N, PATH>())) void debug_tile_kernel(JobDesc A, Launch L, int tile) {
    extern __shared__ long long S[];
    __shared__ Shared sh;
    process_tile<N, PATH, TK>(A, 0, tile, L, S, sh);
}

// Persistent workgroups draining a work list through an atomic cursor; every
// workgroup leaves once the cursor passes the end of the list.
__device__ __forceinline__ int next_item(unsigned* cursor, Shared& sh) {
    __syncthreads();
    if (threadIdx.x == 0) sh.item = (int)atomicAdd(cursor, 1u);
    __syncthreads();
    return sh.item;
}

// A list of (job, tile) items filled by an earlier launch, drained through a cursor.
struct ItemList {
    const unsigned* count;
    const int2* items;
    unsigned* cursor;
    int cap;
};

// Tier 2 of a single job: the tiles that did not fit tier 1's LDS (full LDS here).
template <int N, int PATH, int TK = N>
__global__ __launch_bounds__((threads_of<N, PATH>())) void overflow_kernel(JobDesc A, Launch L, ItemList in,
                                                                            unsigned* blocks) {
    extern __shared__ long long S[];
    __shared__ Shared sh;
    const int total = (int)min(*in.count, (unsigned)in.cap);
    for (;;) {
        const int i = next_item(in.cursor, sh);
        if (i >= total) break;
        process_tile<N, PATH, TK>(A, 0, in.items[i].y, L, S, sh, blocks);
    }
}

// Tier 3 of a single job: windows larger than any workgroup's LDS, each workgroup
// working in its own slice of a global scratch buffer (L2/MALL-resident).
template <int N, int PATH, int TK = N>
__global__ __launch_bounds__((threads_of<N, PATH>())) __attribute__((amdgpu_waves_per_eu(N < 3 ? 2 : 1))) void scratch_kernel(
    JobDesc A, Launch L, ItemList in, long long* scratch, long long band_cap, const unsigned* blocks) {
    extern __shared__ long long LB[];
    __shared__ Shared sh;
    long long* S = scratch + (long long)blockIdx.x * L.lds_cap;
    const int total = (int)min(*in.count, (unsigned)in.cap);
    for (;;) {
        const int i = next_item(in.cursor, sh);
        if (i >= total) break;
        const int lead = in.items[i].y;
        process_block<N, PATH, TK>(A, lead, blocks[A.item_base + lead], L, S, sh, LB, band_cap);
    }
}

// A batch of jobs: items are (job, tile) pairs numbered job by job (jobs sorted by cost
// on the host, heaviest first); tier 1 pushes tiles that need more LDS to a list.
__device__ __forceinline__ int find_job(const JobDesc* jobs, int njobs, long long item) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (jobs[mid].item_base <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// One (order, path) variant of a batch: its jobs are jobs[j0 .. j0+nj), its items
// first .. first+count-1 in the batch's numbering.  The kernels read these counts from
// device memory, so one launch sequence (a captured graph, say) serves any batch whose
// counts were uploaded before it.
struct GroupHdr {
    int j0, nj;
    long long first, count;
};

// The group's slices of the batch-wide overflow lists: items first .. first+count-1.
__device__ __forceinline__ void group_lists(const GroupHdr& h, Launch& L, ItemList* in) {
    if (L.push_cap > 0) {
        L.push_list += h.first;
        L.push_cap = (int)h.count;
    }
    if (in) {
        in->items += h.first;
        in->cap = (int)h.count;
    }
}

// Each variant runs in kernels of its own, so every variant gets the registers and LDS its
// own tiles need.
template <int N, int PATH>
__global__ __launch_bounds__((threads_of<N, PATH>())) __attribute__((amdgpu_waves_per_eu(N < 3 ? 2 : 1))) void batch_kernel(
    const JobDesc* jobs, const GroupHdr* hdr, Launch L, unsigned* cursor) {
    __shared__ Shared sh;
    const GroupHdr h = *hdr;
    group_lists(h, L, nullptr);
    for (;;) {
        const long long i = next_item(cursor, sh);
        if (i >= h.count) break;
        const int j = h.j0 + find_job(jobs + h.j0, h.nj, h.first + i);
        const JobDesc A = jobs[j];
        process_tile<N, PATH>(A, j, (int)(h.first + i - A.item_base), L, g_lds, sh);
    }
}

template <int N, int PATH>
__global__ __launch_bounds__((threads_of<N, PATH>())) void batch_overflow_kernel(const JobDesc* jobs, const GroupHdr* hdr,
                                                                                 Launch L, ItemList in, unsigned* blocks) {
    __shared__ Shared sh;
    group_lists(*hdr, L, &in);
    const int total = (int)min(*in.count, (unsigned)in.cap);
    for (;;) {
        const int i = next_item(in.cursor, sh);
        if (i >= total) break;
        const int2 it = in.items[i];
        process_tile<N, PATH>(jobs[it.x], it.x, it.y, L, g_lds, sh, blocks);
    }
}

template <int N, int PATH>
__global__ __launch_bounds__((threads_of<N, PATH>())) __attribute__((amdgpu_waves_per_eu(N < 3 ? 2 : 1))) void batch_scratch_kernel(
    const JobDesc* jobs, const GroupHdr* hdr, Launch L, ItemList in, long long* scratch, long long band_cap,
    const unsigned* blocks) {
    __shared__ Shared sh;
    long long* S = scratch + (long long)blockIdx.x * L.lds_cap;
    group_lists(*hdr, L, &in);
    const int total = (int)min(*in.count, (unsigned)in.cap);
    for (;;) {
        const int i = next_item(in.cursor, sh);
        if (i >= total) break;
        const int2 it = in.items[i];
        const JobDesc A = jobs[it.x];
        process_block<N, PATH>(A, it.y, blocks[A.item_base + it.y], L, S, sh, g_lds, band_cap);
    }
}

// Clears `n` words (a plan's per-job error words) at the start of its launch sequence.
__global__ void clear_words(unsigned* w, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) w[i] = 0u;
}

// The 64 counters at the head of a call's work area (8 per batch variant).
__global__ void reset_counters(unsigned* c) {
    if (threadIdx.x < 64) c[threadIdx.x] = 0u;
}

// ---------------------------------------------------------------------------
// Global pre-integrator (bsf_preintegrate): stage 1 (eq. RS, n folds per direction)
// over an arbitrary window held in HBM.  The workspace T has hq rows of pitch tp >= wt,
// wt = wq + hq - 1; row r holds wt - r entries (the box, then the extension triangle
// that step (4) reads).  Four passes, each reading and writing every element once:
//   rows : f -> T, one workgroup per row, the n folds fused (chunked block scan);
//   diag : T -> T along (1,1);  cols: T -> T along (0,1);  anti: T -> g along (-1,1).
// The three upward passes give each wave a strip of kStrip adjacent lines (see
// gpre_lines).  Arithmetic is modulo 2^64 (unsigned), exact wherever the true value
// fits int64.
// ---------------------------------------------------------------------------
struct GlobalArgs {
    const void* in;
    long long in_pitch;
    int width, height, in_dtype, border;
    int x0, y0, wq, hq;
    long long* T;  // workspace [hq][tp]
    long long tp;  // workspace pitch: wt rounded up to a multiple of 4 (32-byte rows)
    long long* g;
    long long g_pitch;
};

constexpr int kStrip = 4;  // lines per wave in the upward passes

using u64 = unsigned long long;


// Lines of the upward passes, by their column c0 at row 0:
//   DIR 2 (1,1):  c(r) = c0 + r, c0 in [-(hq-1), wt-1], rows max(0,-c0) .. (wt-1-c0)/2
//   DIR 3 (0,1):  c(r) = c0,     c0 in [0, wt-1],      rows 0 .. min(hq, wt-c0)-1
//   DIR 4 (-1,1): c(r) = c0 - r, c0 in [0, wt-1],      rows 0 .. min(hq-1, c0)
template <int DIR>
__device__ __forceinline__ void line_rows(int c0, int hq, int wt, int& rs, int& re) {
    if (DIR == 2) {
        rs = c0 < 0 ? -c0 : 0;
        re = min(hq, (wt - 1 - c0) / 2 + 1);
    } else if (DIR == 3) {
        rs = 0;
        re = min(hq, wt - c0);
    } else {
        rs = 0;
        re = min(hq, c0 + 1);
    }
}

// Carry state of the n-fold running sum of one line: s_f = the last value of fold f.
// Feeding m zeros into a line with state c gives the state L^m c with
//   (L^m c)_f = sum_{i <= f} c_i * binom(m - 1 + f - i, f - i).
template <int N>
__device__ __forceinline__ void propagate(const u64* c, u64 m, u64* out) {
    const u64 b1 = m, b2 = (m * (m + 1)) >> 1;  // binom(m-1+k, k), k = 1, 2
#pragma unroll
    for (int f = 0; f < N; ++f) {
        u64 v = c[f];
        if (f >= 1) v += c[f - 1] * b1;
        if (f >= 2) v += c[f - 2] * b2;
        out[f] = v;
    }
}

// Every pass is a set of independent lines, each scanned n times.  A wave owns W
// adjacent lines (W = 1 for the row pass, kStrip for the others) and walks them in
// batches of NB * kRun positions: lane (i, j), i < W, j < NB = 64 / W, owns positions
// j*kRun .. j*kRun + kRun-1 of line i.  A lane scans its positions in registers from a
// zero state, a Kogge-Stone scan over j combines the blocks' end states with the carry
// maps L, and each lane adds the closed-form contribution of its incoming state.
// Loads run kAhead batches ahead of the scan.
constexpr int kRun = 16;
constexpr int kAhead = 2;

template <int N, int W>
__device__ __forceinline__ void scan_batch(u64 (&cur)[kRun], u64 (&carry)[N], int i, int j) {
    constexpr int NB = 64 / W;
    u64 agg[N];
#pragma unroll
    for (int f = 0; f < N; ++f) {
#pragma unroll
        for (int t = 1; t < kRun; ++t) cur[t] += cur[t - 1];
        agg[f] = cur[kRun - 1];
    }
#pragma unroll
    for (int d = 1; d < NB; d <<= 1) {
        u64 prev[N], moved[N];
#pragma unroll
        for (int f = 0; f < N; ++f) prev[f] = __shfl_up(agg[f], d * W);
        propagate<N>(prev, (u64)(d * kRun), moved);
        if (j >= d) {
#pragma unroll
            for (int f = 0; f < N; ++f) agg[f] += moved[f];
        }
    }
    u64 inc[N], before[N], ex[N], last[N], through[N];
#pragma unroll
    for (int f = 0; f < N; ++f) {
        ex[f] = __shfl_up(agg[f], W);
        last[f] = __shfl(agg[f], (NB - 1) * W + i);
    }
    propagate<N>(carry, (u64)(j * kRun), before);
    propagate<N>(carry, (u64)(NB * kRun), through);
#pragma unroll
    for (int f = 0; f < N; ++f) {
        inc[f] = before[f] + (j > 0 ? ex[f] : 0ull);
        carry[f] = through[f] + last[f];
    }
#pragma unroll
    for (int t = 0; t < kRun; ++t) {
#pragma unroll
        for (int f = 1; f < N; ++f) inc[f] += inc[f - 1];
        cur[t] += inc[N - 1];
    }
}

// Exact integer of an input sample: uint8 as is, float samples on the 2^-24 grid x 2^24.
template <typename TIN>
__device__ __forceinline__ u64 sample_int(TIN v) {
    if constexpr (sizeof(TIN) == 1) return (u64)v;
    else return (u64)(long long)rint((double)v * 16777216.0);
}

// Workspace tail behind the hq x tp array: 8 zero words that positions outside a line
// read.  Selecting the address instead of the loaded value keeps every load
// unconditional straight-line code (a load under a branch would be waited for at once),
// so the loads of the next kAhead batches stay in flight while a batch is scanned.
constexpr int kZeros = 8;

__global__ void gpre_zero(GlobalArgs A) {
    u64* z = (u64*)A.T + (long long)A.hq * A.tp;
    if (threadIdx.x < kZeros) z[threadIdx.x] = 0ull;
}

// DIR 1: rows (f -> T), one wave per row.  DIR 2..4: strips of kStrip lines.
template <int N, int DIR, typename TIN>
__global__ __launch_bounds__(64) void gpre_pass(GlobalArgs A, int nwaves) {
    constexpr int W = (DIR == 1) ? 1 : kStrip;
    constexpr int NB = 64 / W;
    constexpr int span = NB * kRun;
    const int wt = A.wq + A.hq - 1, hq = A.hq;
    const long long tp = A.tp;
    const int lane = threadIdx.x, i = lane % W, j = lane / W;
    const int w = xcd_tile(blockIdx.x, gridDim.x);
    if (w >= nwaves) return;
    u64* T = (u64*)A.T;
    const u64* zeros = T + (long long)hq * tp;
    // positions along the lines: [ps, pe) for this lane's line, [sps, spe) for the wave
    int ps, pe, sps, spe, c0 = 0, r = 0;
    if (DIR == 1) {
        r = w;
        ps = sps = 0;
        pe = spe = wt - r;
    } else {
        const int first = (DIR == 2) ? -(hq - 1) : 0;
        const int s0 = first + w * kStrip;
        c0 = s0 + i;
        line_rows<DIR>(c0, hq, wt, ps, pe);
        if (c0 > wt - 1) { ps = 0; pe = 0; }
        int a, b, a2, b2;  // the strip's extent: the union over its lines
        line_rows<DIR>(min(s0 + kStrip - 1, wt - 1), hq, wt, a, b);
        line_rows<DIR>(s0, hq, wt, a2, b2);
        sps = min(a, a2);
        spe = max(b, b2);
    }
    constexpr int dc = (DIR == 2) ? 1 : (DIR == 3 ? 0 : -1);
    const long long stride = tp + dc;  // elements between consecutive positions of a line
    // positions whose values are stored: the anti-diagonal pass writes only the box
    const int qs = (DIR == 4) ? max(ps, c0 - A.wq + 1) : ps;
    // row pass: the image row and whether it lies inside the image
    const int yr = (DIR == 1) ? A.y0 + r : 0;
    const bool row_in = yr >= 0 && yr < A.height;
    const TIN* img_row = (const TIN*)A.in + (long long)clampi(yr, 0, A.height - 1) * A.in_pitch;
    const bool zero_border = A.border == BSF_BORDER_ZERO;
    auto load_batch = [&](u64 (&x)[kRun], int p0) {
        const int q0 = p0 + j * kRun;
        if (DIR == 1) {
#pragma unroll
            for (int t = 0; t < kRun; ++t) {
                const int p = q0 + t;
                const int xi = A.x0 + p;
                const bool in = p < A.wq && (!zero_border || (row_in && xi >= 0 && xi < A.width));
                const TIN* src = in ? img_row + clampi(xi, 0, A.width - 1) : (const TIN*)zeros;
                x[t] = sample_int<TIN>(*src);
            }
        } else {
            const long long base = (long long)q0 * stride + c0;
#pragma unroll
            for (int t = 0; t < kRun; ++t) {
                const int p = q0 + t;
                const bool in = p >= ps && p < pe;
                x[t] = *(in ? T + base + t * stride : zeros);
            }
        }
    };
    auto store_batch = [&](const u64 (&x)[kRun], int p0) {
        const int q0 = p0 + j * kRun;
        if (DIR == 1) {
            u64* row = T + (long long)r * tp;
            if (q0 + kRun <= pe) {  // rows are 32-byte aligned (tp % 4 == 0), q0 % 16 == 0
                ulonglong2* v = (ulonglong2*)(row + q0);
#pragma unroll
                for (int t = 0; t < kRun / 2; ++t) v[t] = make_ulonglong2(x[2 * t], x[2 * t + 1]);
            } else {
#pragma unroll
                for (int t = 0; t < kRun; ++t)
                    if (q0 + t < pe) row[q0 + t] = x[t];
            }
        } else {
            u64* dst;
            long long dstride;
            if (DIR == 4) {  // g[p][c0 - p]
                dst = (u64*)A.g + (long long)q0 * A.g_pitch + (c0 - q0);
                dstride = A.g_pitch - 1;
            } else {
                dst = T + (long long)q0 * stride + c0;
                dstride = stride;
            }
#pragma unroll
            for (int t = 0; t < kRun; ++t) {
                const int p = q0 + t;
                if (p >= qs && p < pe) dst[t * dstride] = x[t];
            }
        }
    };
    u64 carry[N];
#pragma unroll
    for (int f = 0; f < N; ++f) carry[f] = 0;
    u64 b0[kRun], b1[kRun], b2[kRun];
    static_assert(kAhead == 2, "three rotating batch buffers");
    load_batch(b0, sps);
    load_batch(b1, sps + span);
    // each step scans one batch while the loads of the next two are in flight
    auto step = [&](u64 (&proc)[kRun], u64 (&fill)[kRun], int p0) {
        load_batch(fill, p0 + kAhead * span);
        scan_batch<N, W>(proc, carry, i, j);
        store_batch(proc, p0);
    };
    for (int p0 = sps; p0 < spe; p0 += 3 * span) {
        step(b0, b2, p0);
        if (p0 + span >= spe) break;
        step(b1, b0, p0 + span);
        if (p0 + 2 * span >= spe) break;
        step(b2, b1, p0 + 2 * span);
    }
}

template <int N>
void launch_global(const GlobalArgs& A, hipStream_t st) {
    const int wt = A.wq + A.hq - 1;
    const int nd = (wt + A.hq - 1 + kStrip - 1) / kStrip;
    const int nc = (wt + kStrip - 1) / kStrip;
    hipLaunchKernelGGL(gpre_zero, dim3(1), dim3(64), 0, st, A);
    if (A.in_dtype == BSF_U8)
        hipLaunchKernelGGL((gpre_pass<N, 1, unsigned char>), dim3(A.hq), dim3(64), 0, st, A, A.hq);
    else if (A.in_dtype == BSF_F32)
        hipLaunchKernelGGL((gpre_pass<N, 1, float>), dim3(A.hq), dim3(64), 0, st, A, A.hq);
    else
        hipLaunchKernelGGL((gpre_pass<N, 1, double>), dim3(A.hq), dim3(64), 0, st, A, A.hq);
    hipLaunchKernelGGL((gpre_pass<N, 2, unsigned char>), dim3(nd), dim3(64), 0, st, A, nd);
    hipLaunchKernelGGL((gpre_pass<N, 3, unsigned char>), dim3(nc), dim3(64), 0, st, A, nc);
    hipLaunchKernelGGL((gpre_pass<N, 4, unsigned char>), dim3(nc), dim3(64), 0, st, A, nc);
}

// ---------------------------------------------------------------------------
// Scale field of elliptical windows.  The order-n box spline with scales a has the
// covariance (n/12) sum_k a_k^2 r_k r_k^T (each segment of length a_k along r_k is a
// uniform density of variance a_k^2/12; Section 4); the scales of a pixel are those whose
// covariance is closest in the Frobenius norm to the ellipse's R diag(s1^2, s2^2) R^T,
// with a_k >= kScaleMin and the least sum a_k^4 among ties (isotropic ellipses give the
// scales of Theorem 4.3).  In the units S = (12/n) Sigma and with w = a^2 the model is
//   [[w1 + t, d], [d, w3 + t]],  t = (w2 + w4)/2,  d = (w2 - w4)/2,
// so with lb = kScaleMin^2, q = |S_xy| and m <= M the two diagonal entries minus 2 lb:
// * q <= m: exact, t in [lb + q, lb + m], the least sum of squares at t = (Sxx + Syy)/4;
// * else the closest: t = lb + u, |d| = u (one of w2, w4 at the bound), u >= 0 minimising
//   max(0, u - m)^2 + max(0, u - M)^2 + 2 (u - q)^2, i.e. (m + 2q)/3 up to M, else
//   (m + M + 2q)/4; then w1 = max(lb, Sxx - t), w3 = max(lb, Syy - t).
// ---------------------------------------------------------------------------
__device__ __forceinline__ float4 ellipse_scales(float s1, float s2, float ph, int n) {
    const double v1 = (double)s1 * s1, v2 = (double)s2 * s2;
    double sn, cs;
    sincos(2.0 * (double)ph, &sn, &cs);
    const double k = 12.0 / n, hs = 0.5 * (v1 + v2), hd = 0.5 * (v1 - v2);
    const double Sxx = k * (hs + hd * cs), Syy = k * (hs - hd * cs), Sxy = k * hd * sn;
    const double lb = kScaleMin * kScaleMin;
    const double q = fabs(Sxy), A = Sxx - 2.0 * lb, B = Syy - 2.0 * lb;
    const double m = fmin(A, B), M = fmax(A, B);
    double t, d;
    if (q <= m) {
        t = fmin(fmax(0.25 * (Sxx + Syy), lb + q), lb + m);
        d = Sxy;
    } else {
        double u = (m + 2.0 * q) / 3.0;
        if (u > M) u = 0.25 * (m + M + 2.0 * q);
        u = fmax(u, 0.0);
        t = lb + u;
        d = copysign(u, Sxy);
    }
    const double w1 = fmax(lb, Sxx - t), w2 = fmax(lb, t + d), w3 = fmax(lb, Syy - t), w4 = fmax(lb, t - d);
    // a = sqrt(w) in float32, correctly rounded from the float32-rounded w: within one float32
    // ulp of the rounded float64 root (its error is below 0.75 ulp of a), at a fraction of the
    // float64 square root's cost
    return make_float4(__fsqrt_rn((float)w1), __fsqrt_rn((float)w2), __fsqrt_rn((float)w3), __fsqrt_rn((float)w4));
}

// Two adjacent pixels per thread (two independent float64 chains in flight); a block
// covers 512 consecutive pixels of one row.
__global__ __launch_bounds__(256) void ellipse_scales_kernel(const float* __restrict__ ell, long long ell_pitch, int width,
                                                             int blocks_per_row, int n, float* __restrict__ scales,
                                                             long long scale_pitch, unsigned* err) {
    const int y = blockIdx.x / blocks_per_row;
    const int x0 = (blockIdx.x - y * blocks_per_row) * 512 + 2 * threadIdx.x;
    bool bad = false;
    if (x0 < width) {
        const float* e = ell + 3 * ((long long)y * ell_pitch + x0);
        float* o = scales + 4 * ((long long)y * scale_pitch + x0);
        const bool two = x0 + 1 < width;
        float v[6];
#pragma unroll
        for (int i = 0; i < 3; ++i) v[i] = e[i];
#pragma unroll
        for (int i = 3; i < 6; ++i) v[i] = two ? e[i] : 1.0f;
        const float nan = __builtin_nanf("");
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const float s1 = v[3 * p], s2 = v[3 * p + 1], ph = v[3 * p + 2];
            const bool ok = isfinite(s1) && isfinite(s2) && isfinite(ph) && s1 > 0.f && s2 > 0.f;
            bad |= !ok;
            const float4 a = ok ? ellipse_scales(s1, s2, ph, n) : make_float4(nan, nan, nan, nan);
            if (p == 0 || two) *reinterpret_cast<float4*>(o + 4 * p) = a;
        }
    }
    const unsigned long long b = __ballot(bad);  // one flag per wave
    if (b && (int)(threadIdx.x & 63) == __ffsll((long long)b) - 1) atomicOr(err, kErrScale);
}

}  // namespace bsf

// ===========================================================================
// Host side: the C ABI.
// ===========================================================================
#include "rect.h"

// Work area of bsf_filter_noalloc: a fixed array in device memory, one copy per GPU the
// library runs on, held until the process ends.  Host code never passes this symbol to a
// kernel (on the host it names a stand-in, not device memory): it uses the device address
// hipGetSymbolAddress returns for each device, cached in noalloc_address().
constexpr size_t kNoAllocBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char noalloc_scratch[kNoAllocBytes];

struct bsf_ctx {
    int device = 0;
    int cus = 256;
    size_t ws_limit = 0;
    unsigned* d_err = nullptr;
    unsigned long long* d_stats = nullptr;  // inside the d_err allocation
    // Per-call device work areas (counters, overflow list, batch descriptors) and pinned
    // host staging, in a ring: calls on different streams may be in flight together; a
    // slot is reused only after the call that last used it has finished on the device.
    static constexpr int kRing = 8;
    struct Slot {
        void* dev = nullptr;
        size_t dev_bytes = 0;
        bsf::JobDesc* host = nullptr;
        int host_cap = 0;
        hipEvent_t done = nullptr;
    } slot[kRing];
    int slot_next = 0;
    long long lds_max_bytes = 0;   // LDS a workgroup may hold
    void* noalloc = nullptr;       // this device's copy of noalloc_scratch (null: lookup failed)
    std::string noalloc_error;     // why the lookup failed
    long long lds_static[4] = {1024, 1024, 1024, 1024};  // per order: the largest static LDS of its kernels, plus a margin
    std::string last;
    bsf_plan::Limits limits() const {
        bsf_plan::Limits L{};
        L.lds_max = lds_max_bytes;
        for (int n = 0; n < 4; ++n) L.lds_static[n] = lds_static[n];
        L.cus = cus;
        return L;
    }
};

// A captured batched launch (bsf_batch_plan_*): a fixed work area sized for its capacity,
// pinned descriptor staging, one error word per job, and the graph of the launch sequence.
struct bsf_batch_plan {
    bsf_ctx* ctx = nullptr;
    int max_jobs = 0;
    long long max_tiles = 0;
    float a_max = 0.f;
    void* dev = nullptr;            // counters | list A | list B | headers + descriptors | scratch | error words
    size_t jobs_off = 0, err_off = 0;
    bsf::JobDesc* host = nullptr;   // pinned staging: kHdrSlots header slots, then max_jobs descriptors
    unsigned* herr = nullptr;       // pinned: the per-job error words of the last run, by the caller's job index
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;      // recorded after each replay
    int last_njobs = 0;
};

namespace {

using namespace bsf;

bsf_status fail(bsf_ctx* c, bsf_status s, const std::string& msg) {
    if (c) c->last = msg;
    return s;
}

bsf_status hip_fail(bsf_ctx* c, hipError_t e, const char* what) {
    return fail(c, BSF_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Device address of noalloc_scratch on `device`, looked up once per device with that
// device current (each GPU holds its own copy of the array at its own address).
hipError_t noalloc_address(int device, void** out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    static hipError_t err[kMaxDevices] = {};
    static bool done[kMaxDevices] = {};
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!done[device]) {
        void* p = nullptr;
        err[device] = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
        addr[device] = err[device] == hipSuccess ? p : nullptr;
        done[device] = true;
    }
    *out = addr[device];
    return err[device];
}

bsf_status validate(bsf_ctx* c, const bsf_job* j, bool need_out) {
    if (!j) return fail(c, BSF_ERR_INVALID_ARG, "job is null");
    if (j->width < 1 || j->height < 1) return fail(c, BSF_ERR_INVALID_ARG, "width and height must be >= 1");
    if (j->width > (1 << 24) || j->height > (1 << 24)) return fail(c, BSF_ERR_INVALID_ARG, "image too large");
    if (!j->in) return fail(c, BSF_ERR_INVALID_ARG, "input pointer is null");
    if (j->in_pitch < j->width) return fail(c, BSF_ERR_INVALID_ARG, "in_pitch < width");
    if (j->in_dtype != BSF_U8 && j->in_dtype != BSF_F32 && j->in_dtype != BSF_F64)
        return fail(c, BSF_ERR_INVALID_ARG, "unknown input dtype");
    if (j->border != BSF_BORDER_CLAMP && j->border != BSF_BORDER_ZERO)
        return fail(c, BSF_ERR_INVALID_ARG, "unknown border rule");
    if (j->order < 1 || j->order > 3) return fail(c, BSF_ERR_UNSUPPORTED, "order must be 1, 2 or 3");
    if (!need_out) return BSF_OK;
    if (!j->scales) return fail(c, BSF_ERR_INVALID_ARG, "scales pointer is null");
    if (((uintptr_t)j->scales) % 16) return fail(c, BSF_ERR_INVALID_ARG, "scales must be 16-byte aligned");
    if (j->scale_pitch < j->width) return fail(c, BSF_ERR_INVALID_ARG, "scale_pitch < width");
    if (!j->out) return fail(c, BSF_ERR_INVALID_ARG, "output pointer is null");
    if (j->out_pitch < j->width) return fail(c, BSF_ERR_INVALID_ARG, "out_pitch < width");
    if (j->path != BSF_PATH_F64 && j->path != BSF_PATH_F32_TILED)
        return fail(c, BSF_ERR_INVALID_ARG, "unknown path");
    if (!(j->a_max == 0.0f || (j->a_max >= (float)kScaleMin && j->a_max <= (float)kScaleMax)))
        return fail(c, BSF_ERR_INVALID_ARG, "a_max must be 0 or a bound in [0.5, 1e4]");
    return BSF_OK;
}

template <int N, int K = N>
long long window_bound_elems(float a_max, int extent) {
    const double R = reach1(N, a_max, a_max, a_max);
    return window_elems(tile_window<N, K>(0, 0, extent, extent, R, R));
}

// the largest window a 16x16 tile (extent 16), or a 2x2 block of tiles in tier 3 (extent
// 32), of order n (model m: -1 = phi = delta) needs for scales up to a_max
long long window_bound(int n, float a_max, int model = -1, int extent = kTile) {
    if (model == 0) return window_bound_elems<1, table_key(1, 0)>(a_max, extent);
    if (model == 1) return window_bound_elems<1, table_key(1, 1)>(a_max, extent);
    switch (n) {
        case 1: return window_bound_elems<1>(a_max, extent);
        case 2: return window_bound_elems<2>(a_max, extent);
        default: return window_bound_elems<3>(a_max, extent);
    }
}


template <typename K>
void allow_big_lds(K* kernel) {
    // opt in to dynamic LDS beyond the default per-workgroup limit (once per kernel)
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              163840 - 1024);
    (void)hipGetLastError();
}

using bsf_plan::Plan;
using bsf_plan::WorkLayout;

Plan plan_tiers(const bsf_ctx* c, long long need, int order, long long need3 = 0) {
    return bsf_plan::plan_tiers(c->limits(), need, order, need3);
}

int per_cu(const bsf_ctx* c, long long elems, int order) { return bsf_plan::per_cu(c->limits(), elems, order); }

WorkLayout work_layout(long long items, int njobs, size_t scratch_bytes) {
    return bsf_plan::work_layout(items, njobs, sizeof(JobDesc), scratch_bytes);
}

struct Tiers {
    Launch L1, L2, L3;
    ItemList inA, inB;
    long long* scratch = nullptr;
    unsigned* blocks = nullptr;  // tier 3's block words (null without tier 3)
    int grid2 = 1, grid3 = 1, grid_lat = 1;
    int one_launch = 0;  // tiles at or below this: one tier-1 launch (one workgroup per CU)
};

// Tiers over `items` tiles whose overflow lists are la / lb (capacity items each) and
// whose counters are ctr[0..4]: [0] list A count, [1] list A cursor, [2] tier-1 cursor,
// [3] list B count, [4] list B cursor.
// blocks: tier 3's block words, one per item of the whole launch sequence (work_layout).
Tiers make_tiers_at(const bsf_ctx* c, const Plan& p, unsigned* ctr, int2* la, int2* lb, unsigned* blocks,
                    long long* scratch, long long items, int order, long long grid3 = 0) {
    Tiers t;
    t.L1 = Launch{};
    t.L1.lds_cap = p.t1;
    t.L1.stats = c->d_stats;
    t.L2 = t.L1;
    t.L2.lds_cap = p.t2;
    t.L3 = t.L1;
    t.L3.lds_cap = p.t3;
    t.grid_lat = (int)std::max<long long>(8, ((long long)c->cus * per_cu(c, p.t1, order)) & ~7ll);
    t.one_launch = c->cus;
    if (p.use2) {
        t.L1.push_count = ctr + 0;
        t.L1.push_list = la;
        t.L1.push_cap = (int)items;
        t.inA = ItemList{ctr + 0, la, ctr + 1, (int)items};
        t.grid2 = (int)std::min<long long>(items, (long long)c->cus * per_cu(c, p.t2, order));
    }
    if (p.use3) {
        t.L2.push_count = ctr + 3;
        t.L2.push_list = lb;
        t.L2.push_cap = (int)items;
        t.inB = ItemList{ctr + 3, lb, ctr + 4, (int)items};
        t.grid3 = (int)(grid3 > 0 ? grid3 : bsf_plan::grid3_of(c->limits(), items));
        t.scratch = scratch;
        t.blocks = blocks;
    }
    return t;
}

Tiers make_tiers(const bsf_ctx* c, const Plan& p, char* work, const WorkLayout& w, long long items, int order,
                 long long grid3 = 0) {
    if (!work) return make_tiers_at(c, p, nullptr, nullptr, nullptr, nullptr, nullptr, items, order);  // tier 1 only
    return make_tiers_at(c, p, (unsigned*)work, (int2*)(work + w.lists_off), (int2*)(work + w.listb_off),
                         (unsigned*)(work + w.blocks_off), (long long*)(work + w.scratch_off), items, order, grid3);
}

// Tier 3's block words start at zero in every call (a kernel: the words may sit in a
// captured graph, where memset nodes are avoided).
void clear_blocks(const Tiers& t, long long items, hipStream_t st) {
    if (t.blocks)
        hipLaunchKernelGGL(clear_words, dim3((unsigned)((items + 255) / 256)), dim3(256), 0, st, t.blocks, (int)items);
}

template <int N, int PATH, int TK = N>
hipError_t launch_single(const JobDesc& A, const Plan& p, const Tiers& t, int tiles, hipStream_t st) {
    static bool once = false;
    if (!once) {
        allow_big_lds(&tile_kernel<N, PATH, TK>);
        allow_big_lds(&lattice_tile_kernel<N, PATH, TK>);
        allow_big_lds(&overflow_kernel<N, PATH, TK>);
        allow_big_lds(&scratch_kernel<N, PATH, TK>);
        allow_big_lds(&debug_tile_kernel<N, PATH, TK>);
        once = true;
    }
    if (tiles <= t.one_launch) {  // one workgroup per CU at most: one launch, each tile in its own form
        hipLaunchKernelGGL((lattice_tile_kernel<N, PATH, TK>), dim3(tiles), dim3(threads_of<N, PATH>()), (size_t)p.t1 * 8,
                           st, A, t.L1, 1);
    } else {
        hipLaunchKernelGGL((tile_kernel<N, PATH, TK>), dim3(tiles), dim3(threads_of<N, PATH>()), (size_t)p.t1 * 8, st, A,
                           t.L1);
        hipLaunchKernelGGL((lattice_tile_kernel<N, PATH, TK>), dim3(t.grid_lat), dim3(threads_of<N, PATH>()),
                           (size_t)p.t1 * 8, st, A, t.L1, 0);
    }
    if (p.use2)
        hipLaunchKernelGGL((overflow_kernel<N, PATH, TK>), dim3(t.grid2), dim3(threads_of<N, PATH>()), (size_t)p.t2 * 8, st, A,
                           t.L2, t.inA, t.blocks);
    if (p.use3)
        hipLaunchKernelGGL((scratch_kernel<N, PATH, TK>), dim3(t.grid3), dim3(threads_of<N, PATH>()), (size_t)p.band * 8, st, A,
                           t.L3, t.inB, t.scratch, p.band, t.blocks);
    return hipGetLastError();
}

hipError_t dispatch_single(int n, int path, const JobDesc& A, const Plan& p, const Tiers& t, int tiles,
                           hipStream_t st, int model = -1) {
#define BSF_SINGLE(NN, PP) return launch_single<NN, PP>(A, p, t, tiles, st)
    if (model >= 0) {  // the continuous models (order 1)
        if (path == BSF_PATH_F64) {
            if (model == 0) return launch_single<1, BSF_PATH_F64, table_key(1, 0)>(A, p, t, tiles, st);
            return launch_single<1, BSF_PATH_F64, table_key(1, 1)>(A, p, t, tiles, st);
        }
        if (model == 0) return launch_single<1, BSF_PATH_F32_TILED, table_key(1, 0)>(A, p, t, tiles, st);
        return launch_single<1, BSF_PATH_F32_TILED, table_key(1, 1)>(A, p, t, tiles, st);
    }
    if (path == BSF_PATH_F64) {
        if (n == 1) BSF_SINGLE(1, BSF_PATH_F64);
        if (n == 2) BSF_SINGLE(2, BSF_PATH_F64);
        BSF_SINGLE(3, BSF_PATH_F64);
    }
    if (n == 1) BSF_SINGLE(1, BSF_PATH_F32_TILED);
    if (n == 2) BSF_SINGLE(2, BSF_PATH_F32_TILED);
    BSF_SINGLE(3, BSF_PATH_F32_TILED);
#undef BSF_SINGLE
}

hipError_t dispatch_debug(int n, int path, const JobDesc& A, const Launch& L, int tile, size_t lds, hipStream_t st) {
#define BSF_DBG(NN, PP)                                                                          \
    do {                                                                                         \
        allow_big_lds(&debug_tile_kernel<NN, PP>);                                               \
        hipLaunchKernelGGL((debug_tile_kernel<NN, PP>), dim3(1), dim3(threads_of<NN, PP>()), lds, st, A, L, tile); \
        return hipGetLastError();                                                                \
    } while (0)
    if (path == BSF_PATH_F64) {
        if (n == 1) BSF_DBG(1, BSF_PATH_F64);
        if (n == 2) BSF_DBG(2, BSF_PATH_F64);
        BSF_DBG(3, BSF_PATH_F64);
    }
    if (n == 1) BSF_DBG(1, BSF_PATH_F32_TILED);
    if (n == 2) BSF_DBG(2, BSF_PATH_F32_TILED);
    BSF_DBG(3, BSF_PATH_F32_TILED);
#undef BSF_DBG
}

JobDesc make_desc(const bsf_job* j, unsigned* err) {
    JobDesc a{};
    a.err = err;
    a.in = j->in;
    a.in_pitch = j->in_pitch;
    a.scales = j->scales;
    a.scale_pitch = j->scale_pitch;
    a.out = j->out;
    a.out_pitch = j->out_pitch;
    a.width = j->width;
    a.height = j->height;
    a.in_dtype = j->in_dtype;
    a.border = j->border;
    a.order = j->order;
    a.path = j->path;
    a.tiles_x = (j->width + kTile - 1) / kTile;
    a.tiles_y = (j->height + kTile - 1) / kTile;
    a.item_base = 0;
    return a;
}

// Window elements a job's tiles can need, from its a_max (0: at most the whole LDS)
long long job_window_need(const bsf_ctx* c, const bsf_job* j, int model = -1) {
    const long long full = ((long long)c->lds_max_bytes - c->lds_static[j->order]) / 8;
    if (j->a_max > 0.0f) return window_bound(j->order, j->a_max, model) + 64;
    return full;
}
// the same for the 2x2 blocks of tier 3 (0 without a_max: no tier 3)
long long job_window_need3(const bsf_job* j, int model = -1) {
    return j->a_max > 0.0f ? window_bound(j->order, j->a_max, model, 2 * kTile) + 64 : 0;
}

// Take the next ring slot, wait until its previous call has finished on the device,
// and make sure it holds `bytes` of device memory and `njobs` pinned descriptors.  The
// ring's device memory never exceeds the context's workspace limit (bsf_plan::ring_growth):
// a slot that grows takes the other slots along while the limit allows, and releases them
// when it does not.
bsf_status acquire_slot(bsf_ctx* c, size_t bytes, int njobs, int& idx) {
    idx = c->slot_next;
    size_t cur[bsf_ctx::kRing], target[bsf_ctx::kRing];
    for (int r = 0; r < bsf_ctx::kRing; ++r) cur[r] = c->slot[r].dev_bytes;
    if (!bsf_plan::ring_growth(cur, idx, bytes, c->ws_limit, target))
        return fail(c, BSF_ERR_OUT_OF_MEMORY,
                    "the call needs " + std::to_string(bytes) + " bytes of workspace, more than the context's limit of " +
                        std::to_string(c->ws_limit));
    c->slot_next = (idx + 1) % bsf_ctx::kRing;
    bsf_ctx::Slot& sl = c->slot[idx];
    hipError_t e = hipEventSynchronize(sl.done);
    if (e != hipSuccess) return hip_fail(c, e, "waiting for a work slot");
    // shrink first (so the total stays within the limit at every step), then grow
    for (int pass = 0; pass < 2; ++pass)
        for (int r = 0; r < bsf_ctx::kRing; ++r) {
            bsf_ctx::Slot& o = c->slot[r];
            const bool shrink = target[r] < o.dev_bytes, grow = target[r] > o.dev_bytes;
            if (!(pass == 0 ? shrink : grow)) continue;
            if (r != idx) {
                e = hipEventSynchronize(o.done);
                if (e != hipSuccess) return hip_fail(c, e, "waiting for a work slot");
            }
            if (o.dev) (void)hipFree(o.dev);
            o.dev = nullptr;
            o.dev_bytes = 0;
            if (target[r] > 0) {
                e = hipMalloc(&o.dev, target[r]);
                if (e != hipSuccess) return hip_fail(c, e, "work area allocation");
                o.dev_bytes = target[r];
            }
        }
    if (njobs > sl.host_cap) {
        if (sl.host) (void)hipHostFree(sl.host);
        sl.host = nullptr;
        sl.host_cap = 0;
        e = hipHostMalloc((void**)&sl.host, sizeof(JobDesc) * (size_t)njobs);
        if (e != hipSuccess) return hip_fail(c, e, "pinned staging allocation");
        sl.host_cap = njobs;
    }
    return BSF_OK;
}

template <typename K>
void static_lds(K* kernel, long long& mx) {
    hipFuncAttributes fa{};
    if (hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(kernel)) == hipSuccess)
        mx = std::max(mx, (long long)fa.sharedSizeBytes);
    (void)hipGetLastError();
}

// the largest static LDS an order's tile kernels declare (dynamic LDS + static must fit)
template <int N>
long long measure_static_lds_n() {
    long long mx = 0;
    static_lds(&tile_kernel<N, 0>, mx);
    static_lds(&tile_kernel<N, 1>, mx);
    static_lds(&lattice_tile_kernel<N, 0>, mx);
    static_lds(&lattice_tile_kernel<N, 1>, mx);
    static_lds(&overflow_kernel<N, 0>, mx);
    static_lds(&overflow_kernel<N, 1>, mx);
    static_lds(&debug_tile_kernel<N, 0>, mx);
    static_lds(&debug_tile_kernel<N, 1>, mx);
    static_lds(&batch_kernel<N, 0>, mx);
    static_lds(&batch_kernel<N, 1>, mx);
    static_lds(&batch_overflow_kernel<N, 0>, mx);
    static_lds(&batch_overflow_kernel<N, 1>, mx);
    static_lds(&batch_scratch_kernel<N, 0>, mx);
    static_lds(&batch_scratch_kernel<N, 1>, mx);
    static_lds(&scratch_kernel<N, 0>, mx);
    static_lds(&scratch_kernel<N, 1>, mx);
    if constexpr (N == 1) {  // the continuous models run at order 1
        static_lds(&tile_kernel<1, 0, table_key(1, 0)>, mx);
        static_lds(&tile_kernel<1, 1, table_key(1, 0)>, mx);
        static_lds(&tile_kernel<1, 0, table_key(1, 1)>, mx);
        static_lds(&tile_kernel<1, 1, table_key(1, 1)>, mx);
        static_lds(&lattice_tile_kernel<1, 0, table_key(1, 0)>, mx);
        static_lds(&lattice_tile_kernel<1, 1, table_key(1, 0)>, mx);
        static_lds(&lattice_tile_kernel<1, 0, table_key(1, 1)>, mx);
        static_lds(&lattice_tile_kernel<1, 1, table_key(1, 1)>, mx);
        static_lds(&overflow_kernel<1, 0, table_key(1, 1)>, mx);
        static_lds(&overflow_kernel<1, 1, table_key(1, 1)>, mx);
        static_lds(&scratch_kernel<1, 0, table_key(1, 1)>, mx);
        static_lds(&scratch_kernel<1, 1, table_key(1, 1)>, mx);
    }
    return mx;
}

template <int N, int PATH>
void opt_in_batch_kernels() {
    static bool once = false;
    if (!once) {
        allow_big_lds(&batch_kernel<N, PATH>);
        allow_big_lds(&batch_overflow_kernel<N, PATH>);
        allow_big_lds(&batch_scratch_kernel<N, PATH>);
        once = true;
    }
}

void opt_in_all_batch_kernels() {
    opt_in_batch_kernels<1, 0>();
    opt_in_batch_kernels<1, 1>();
    opt_in_batch_kernels<2, 0>();
    opt_in_batch_kernels<2, 1>();
    opt_in_batch_kernels<3, 0>();
    opt_in_batch_kernels<3, 1>();
}

// The launches of one variant; `items` (the group's items, or a plan's capacity) sizes the
// persistent grids, `hdr` holds the counts the kernels go by.
template <int N, int PATH>
hipError_t launch_batch_group(const bsf_ctx* c, const JobDesc* djobs, const GroupHdr* hdr, long long items, const Plan& p,
                              const Tiers& t, unsigned* ctr, hipStream_t st) {
    opt_in_batch_kernels<N, PATH>();
    const int grid1 = (int)std::min<long long>(items, (long long)c->cus * std::min(per_cu(c, p.t1, N), 8));
    hipLaunchKernelGGL((batch_kernel<N, PATH>), dim3(grid1), dim3(threads_of<N, PATH>()), (size_t)p.t1 * 8, st, djobs, hdr,
                       t.L1, ctr + 2);
    if (p.use2)
        hipLaunchKernelGGL((batch_overflow_kernel<N, PATH>), dim3(t.grid2), dim3(threads_of<N, PATH>()), (size_t)p.t2 * 8, st,
                           djobs, hdr, t.L2, t.inA, t.blocks);
    if (p.use3)
        hipLaunchKernelGGL((batch_scratch_kernel<N, PATH>), dim3(t.grid3), dim3(threads_of<N, PATH>()), (size_t)p.band * 8, st,
                           djobs, hdr, t.L3, t.inB, t.scratch, p.band, t.blocks);
    return hipGetLastError();
}

hipError_t dispatch_batch_group(const bsf_ctx* c, int v, const JobDesc* djobs, const GroupHdr* hdr, long long items,
                                const Plan& p, const Tiers& t, unsigned* ctr, hipStream_t st) {
    switch (v) {
        case 0: return launch_batch_group<1, 0>(c, djobs, hdr, items, p, t, ctr, st);
        case 1: return launch_batch_group<1, 1>(c, djobs, hdr, items, p, t, ctr, st);
        case 2: return launch_batch_group<2, 0>(c, djobs, hdr, items, p, t, ctr, st);
        case 3: return launch_batch_group<2, 1>(c, djobs, hdr, items, p, t, ctr, st);
        case 4: return launch_batch_group<3, 0>(c, djobs, hdr, items, p, t, ctr, st);
        default: return launch_batch_group<3, 1>(c, djobs, hdr, items, p, t, ctr, st);
    }
}

// Batch descriptors in device memory (and in their pinned staging): the six group headers
// in the first two descriptor slots, then the jobs.
constexpr int kHdrSlots = 2;
static_assert(6 * sizeof(GroupHdr) <= kHdrSlots * sizeof(JobDesc), "group headers fit their slots");

}  // namespace

namespace {

template <int N, int D, int PATH>
hipError_t launch_filter1d(const bsf::f1d::Args& A, int blocks, long long lds, hipStream_t st) {
    static bool opted = false;
    if (!opted) {
        allow_big_lds(bsf::f1d::filter1d_kernel<N, D, PATH>);
        opted = true;
    }
    hipLaunchKernelGGL((bsf::f1d::filter1d_kernel<N, D, PATH>), dim3(blocks), dim3(bsf::f1d::kThreads), (size_t)lds,
                       st, A);
    return hipGetLastError();
}

template <int PATH>
hipError_t dispatch_filter1d_path(int n, int D, const bsf::f1d::Args& A, int blocks, long long lds, hipStream_t st) {
    // D = model degree + n, model in {-1, 0, 1, 2, 3}
    switch (n * 8 + D) {
        case 1 * 8 + 0: return launch_filter1d<1, 0, PATH>(A, blocks, lds, st);
        case 1 * 8 + 1: return launch_filter1d<1, 1, PATH>(A, blocks, lds, st);
        case 1 * 8 + 2: return launch_filter1d<1, 2, PATH>(A, blocks, lds, st);
        case 1 * 8 + 3: return launch_filter1d<1, 3, PATH>(A, blocks, lds, st);
        case 1 * 8 + 4: return launch_filter1d<1, 4, PATH>(A, blocks, lds, st);
        case 2 * 8 + 1: return launch_filter1d<2, 1, PATH>(A, blocks, lds, st);
        case 2 * 8 + 2: return launch_filter1d<2, 2, PATH>(A, blocks, lds, st);
        case 2 * 8 + 3: return launch_filter1d<2, 3, PATH>(A, blocks, lds, st);
        case 2 * 8 + 4: return launch_filter1d<2, 4, PATH>(A, blocks, lds, st);
        case 2 * 8 + 5: return launch_filter1d<2, 5, PATH>(A, blocks, lds, st);
        case 3 * 8 + 2: return launch_filter1d<3, 2, PATH>(A, blocks, lds, st);
        case 3 * 8 + 3: return launch_filter1d<3, 3, PATH>(A, blocks, lds, st);
        case 3 * 8 + 4: return launch_filter1d<3, 4, PATH>(A, blocks, lds, st);
        case 3 * 8 + 5: return launch_filter1d<3, 5, PATH>(A, blocks, lds, st);
        default: return launch_filter1d<3, 6, PATH>(A, blocks, lds, st);
    }
}

hipError_t dispatch_filter1d(int n, int D, int path, const bsf::f1d::Args& A, int blocks, long long lds,
                             hipStream_t st) {
    return path == 1 ? dispatch_filter1d_path<1>(n, D, A, blocks, lds, st)
                     : dispatch_filter1d_path<0>(n, D, A, blocks, lds, st);
}

// Largest scale bound whose window fits the LDS a workgroup may hold (0 if none does).
// Both paths take the float64 path's window: it bounds the magnitudes the float32 path's plain
// mask cancels as well as the LDS of either path.
double filter1d_max_scale(const bsf_ctx* c, int n, int D) {
    const long long cap = std::min<long long>(c->lds_max_bytes, 163840 - 1024);
    double lo = 0.0, hi = 1e4;
    auto fits = [&](double a) {
        const int W = bsf::f1d::window_len(n, D, a);
        return W <= bsf::f1d::kWindowMax && bsf::f1d::lds_bytes(D, W, 0) <= cap;
    };
    if (!fits(0.5)) return 0.0;
    if (fits(hi)) return hi;
    lo = 0.5;
    for (int i = 0; i < 60; ++i) {
        const double mid = 0.5 * (lo + hi);
        (fits(mid) ? lo : hi) = mid;
    }
    return std::floor(lo * 8.0) / 8.0;
}

}  // namespace

namespace {

template <int N, int D, int SRC>
hipError_t launch_rect(const bsf::rect::Args& A, int blocks, long long lds, hipStream_t st) {
    static bool opted = false;
    if (!opted) {
        allow_big_lds(bsf::rect::rect_kernel<N, D, SRC>);
        opted = true;
    }
    hipLaunchKernelGGL((bsf::rect::rect_kernel<N, D, SRC>), dim3(blocks), dim3(bsf::rect::kThreads), (size_t)lds, st, A);
    return hipGetLastError();
}

template <int SRC>
hipError_t dispatch_rect_src(int n, int D, const bsf::rect::Args& A, int blocks, long long lds, hipStream_t st) {
    // D = model degree + n, model in -1..3
    switch (n * 8 + D) {
        case 1 * 8 + 0: return launch_rect<1, 0, SRC>(A, blocks, lds, st);
        case 1 * 8 + 1: return launch_rect<1, 1, SRC>(A, blocks, lds, st);
        case 1 * 8 + 2: return launch_rect<1, 2, SRC>(A, blocks, lds, st);
        case 1 * 8 + 3: return launch_rect<1, 3, SRC>(A, blocks, lds, st);
        case 1 * 8 + 4: return launch_rect<1, 4, SRC>(A, blocks, lds, st);
        case 2 * 8 + 1: return launch_rect<2, 1, SRC>(A, blocks, lds, st);
        case 2 * 8 + 2: return launch_rect<2, 2, SRC>(A, blocks, lds, st);
        case 2 * 8 + 3: return launch_rect<2, 3, SRC>(A, blocks, lds, st);
        case 2 * 8 + 4: return launch_rect<2, 4, SRC>(A, blocks, lds, st);
        case 2 * 8 + 5: return launch_rect<2, 5, SRC>(A, blocks, lds, st);
        case 3 * 8 + 2: return launch_rect<3, 2, SRC>(A, blocks, lds, st);
        case 3 * 8 + 3: return launch_rect<3, 3, SRC>(A, blocks, lds, st);
        case 3 * 8 + 4: return launch_rect<3, 4, SRC>(A, blocks, lds, st);
        case 3 * 8 + 5: return launch_rect<3, 5, SRC>(A, blocks, lds, st);
        default: return launch_rect<3, 6, SRC>(A, blocks, lds, st);
    }
}

// LDS a rect workgroup may hold: the device's limit less the kernels' (small) static LDS
long long rect_lds_cap(const bsf_ctx* c) { return std::min<long long>(c->lds_max_bytes, 163840) - 1024; }

// The tile side for (n, D, a_max): the largest of 32, 16, 8 whose window fits (0: none)
int rect_tile(const bsf_ctx* c, int n, int D, double a_max) {
    for (int T : {32, 16, 8})
        if (bsf::rect::lds_bytes(T, n, D, a_max) <= rect_lds_cap(c)) return T;
    return 0;
}

double rect_max_scale(const bsf_ctx* c, int n, int D) {
    auto fits = [&](double a) { return rect_tile(c, n, D, a) > 0; };
    if (!fits(0.5)) return 0.0;
    double lo = 0.5, hi = 1e4;
    if (fits(hi)) return hi;
    for (int i = 0; i < 60; ++i) {
        const double mid = 0.5 * (lo + hi);
        (fits(mid) ? lo : hi) = mid;
    }
    return std::floor(lo * 4.0) / 4.0;  // a quarter-pixel grid: exact in float32
}

}  // namespace

extern "C" {

const char* bsf_status_string(bsf_status s) {
    switch (s) {
        case BSF_OK: return "ok";
        case BSF_ERR_INVALID_ARG: return "invalid argument";
        case BSF_ERR_OUT_OF_MEMORY: return "out of memory (workspace limit)";
        case BSF_ERR_HIP: return "HIP runtime error";
        case BSF_ERR_UNSUPPORTED: return "unsupported (window exceeds on-chip memory, or order)";
        case BSF_ERR_SCALE_RANGE: return "scale out of range";
        case BSF_ERR_RANGE: return "pre-integrated value out of the exact integer range";
    }
    return "unknown status";
}

const char* bsf_last_error(const bsf_ctx* ctx) { return ctx ? ctx->last.c_str() : ""; }

bsf_status bsf_create(bsf_ctx** out, int hip_device, size_t workspace_limit_bytes) {
    if (!out) return BSF_ERR_INVALID_ARG;
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) return BSF_ERR_HIP;
    if (hip_device < 0 || hip_device >= ndev) return BSF_ERR_INVALID_ARG;
    bsf_ctx* c = new bsf_ctx();
    c->device = hip_device;
    c->ws_limit = workspace_limit_bytes ? workspace_limit_bytes : (size_t(16) << 30);
    e = hipSetDevice(hip_device);
    if (e != hipSuccess) {
        delete c;
        return BSF_ERR_HIP;
    }
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeSharedMemPerBlockOptin, hip_device) != hipSuccess || lds <= 0) {
        (void)hipGetLastError();
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, hip_device) != hipSuccess) lds = 0;
    }
    c->lds_max_bytes = lds > 0 ? lds : 65536;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, hip_device) == hipSuccess && cus > 0)
        c->cus = cus;
    // static LDS of the kernels (rounded up, plus a margin); never below 1 KiB
    const long long st_n[4] = {0, measure_static_lds_n<1>(), measure_static_lds_n<2>(), measure_static_lds_n<3>()};
    for (int n = 1; n <= 3; ++n) c->lds_static[n] = std::max(1024ll, ((st_n[n] + 255) / 256) * 256 + 256);
    (void)hipGetLastError();
    for (int r = 0; r < bsf_ctx::kRing; ++r) {
        e = hipEventCreateWithFlags(&c->slot[r].done, hipEventDisableTiming);
        if (e != hipSuccess) {
            delete c;
            return BSF_ERR_HIP;
        }
    }
    // the fixed work area of bsf_filter_noalloc (device current)
    e = noalloc_address(hip_device, &c->noalloc);
    if (e != hipSuccess) {
        c->noalloc = nullptr;
        c->noalloc_error = std::string("hipGetSymbolAddress: ") + hipGetErrorString(e);
        (void)hipGetLastError();
    }
    e = hipMalloc(&c->d_err, 64);  // the error word, then the two counters at byte 8
    if (e != hipSuccess) {
        delete c;
        return BSF_ERR_HIP;
    }
    c->d_stats = reinterpret_cast<unsigned long long*>(reinterpret_cast<char*>(c->d_err) + 8);
    e = hipMemset(c->d_err, 0, 64);
    if (e != hipSuccess) {
        (void)hipFree(c->d_err);
        delete c;
        return BSF_ERR_HIP;
    }
    *out = c;
    return BSF_OK;
}

bsf_status bsf_destroy(bsf_ctx* c) {
    if (!c) return BSF_ERR_INVALID_ARG;
    (void)hipSetDevice(c->device);
    if (c->d_err) (void)hipFree(c->d_err);
    for (int r = 0; r < bsf_ctx::kRing; ++r) {
        if (c->slot[r].dev) (void)hipFree(c->slot[r].dev);
        if (c->slot[r].host) (void)hipHostFree(c->slot[r].host);
        if (c->slot[r].done) (void)hipEventDestroy(c->slot[r].done);
    }
    delete c;
    return BSF_OK;
}

bsf_status bsf_workspace_size(const bsf_job* job, size_t* bytes) {
    if (!bytes) return BSF_ERR_INVALID_ARG;
    bsf_status s = validate(nullptr, job, true);
    if (s != BSF_OK) return s;
    // the plan bsf_filter makes, with the limits of an MI355X taken conservatively (a
    // larger static-LDS reserve moves windows to the next tier sooner, never later)
    const bsf_plan::Limits L = bsf_plan::gfx950_bound();
    const long long tiles = (long long)((job->width + kTile - 1) / kTile) * ((job->height + kTile - 1) / kTile);
    const long long need = job->a_max > 0.0f ? window_bound(job->order, job->a_max) + 64 : bsf_plan::full_cap(L, job->order);
    *bytes = bsf_plan::single_call_bytes(L, bsf_plan::plan_tiers(L, need, job->order, job_window_need3(job)), tiles);
    return BSF_OK;
}

bsf_status bsf_filter_model(bsf_ctx* c, const bsf_job* j, int model, void* stream) {
    if (!c) return BSF_ERR_INVALID_ARG;
    bsf_status s = validate(c, j, true);
    if (s != BSF_OK) return s;
    if (model < -1 || model > 1) return fail(c, BSF_ERR_UNSUPPORTED, "model degree must be -1, 0 or 1");
    if (model >= 0 && j->order != 1)
        return fail(c, BSF_ERR_UNSUPPORTED, "the continuous models are provided at order 1");
    const Plan p = plan_tiers(c, job_window_need(c, j, model), j->order, job_window_need3(j, model));
    if (!bsf_plan::plan_fits(c->limits(), p, j->order))
        return fail(c, BSF_ERR_UNSUPPORTED, "the launch's LDS exceeds the device's limit");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    const JobDesc A = make_desc(j, c->d_err);
    const int tiles = A.tiles_x * A.tiles_y;
    Tiers t;
    int slot = -1;
    if (p.use2) {
        const WorkLayout w =
            work_layout(tiles, 0, p.use3 ? (size_t)bsf_plan::grid3_of(c->limits(), tiles) * (size_t)p.t3 * 8 : 0);
        s = acquire_slot(c, w.total, 0, slot);
        if (s != BSF_OK) return s;
        t = make_tiers(c, p, (char*)c->slot[slot].dev, w, tiles, j->order);
        hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, st, (unsigned*)c->slot[slot].dev);
        clear_blocks(t, tiles, st);
    } else {
        t = make_tiers(c, p, nullptr, WorkLayout{}, tiles, j->order);
    }
    e = dispatch_single(j->order, j->path, A, p, t, tiles, st, model);
    if (e == hipSuccess && slot >= 0) e = hipEventRecord(c->slot[slot].done, st);
    if (e != hipSuccess) return hip_fail(c, e, "tile kernel launch");
    return BSF_OK;
}

bsf_status bsf_filter(bsf_ctx* c, const bsf_job* j, void* stream) { return bsf_filter_model(c, j, -1, stream); }

bsf_status bsf_filter_noalloc(bsf_ctx* c, const bsf_job* j, void* stream) {
    if (!c) return BSF_ERR_INVALID_ARG;
    bsf_status s = validate(c, j, true);
    if (s != BSF_OK) return s;
    if (!c->noalloc) return fail(c, BSF_ERR_HIP, "no fixed work area on this device (" + c->noalloc_error + ")");
    const Plan p = plan_tiers(c, job_window_need(c, j), j->order, job_window_need3(j));
    if (!bsf_plan::plan_fits(c->limits(), p, j->order))
        return fail(c, BSF_ERR_UNSUPPORTED, "the launch's LDS exceeds the device's limit");
    const JobDesc A = make_desc(j, c->d_err);
    const int tiles = A.tiles_x * A.tiles_y;
    const bsf_plan::FixedArea f = bsf_plan::fixed_area(c->limits(), p, tiles, kNoAllocBytes);
    if (!f.ok)
        return fail(c, BSF_ERR_OUT_OF_MEMORY,
                    "the call's work area (" + std::to_string(work_layout(tiles, 0, 0).total) + " bytes of tile lists" +
                        (p.use3 ? " and at least one window slice of " + std::to_string(p.t3 * 8) + " bytes" : "") +
                        ") exceeds the fixed " + std::to_string(kNoAllocBytes) + "-byte area of bsf_filter_noalloc");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    Tiers t;
    if (p.use2) {
        const WorkLayout w = work_layout(tiles, 0, f.bytes - work_layout(tiles, 0, 0).total);
        t = make_tiers(c, p, (char*)c->noalloc, w, tiles, j->order, f.grid3);
        // the counters must start at zero: a kernel clears them (the area keeps the last call's contents)
        hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, st, (unsigned*)c->noalloc);
        clear_blocks(t, tiles, st);
    } else {
        t = make_tiers(c, p, nullptr, WorkLayout{}, tiles, j->order);
    }
    e = dispatch_single(j->order, j->path, A, p, t, tiles, st);
    if (e != hipSuccess) return hip_fail(c, e, "tile kernel launch");
    return BSF_OK;
}

bsf_status bsf_filter_batched(bsf_ctx* c, const bsf_job* jobs, int njobs, void* stream) {
    if (!c) return BSF_ERR_INVALID_ARG;
    if (njobs < 0 || (njobs > 0 && !jobs)) return fail(c, BSF_ERR_INVALID_ARG, "bad batch");
    if (njobs == 0) return BSF_OK;
    constexpr int kVariants = 6;  // (order - 1) * 2 + path
    long long need[kVariants] = {}, need3[kVariants] = {};
    double vcost[kVariants] = {};
    std::vector<int> order(njobs);
    std::vector<double> cost(njobs);
    for (int i = 0; i < njobs; ++i) {
        bsf_status s = validate(c, jobs + i, true);
        if (s != BSF_OK) return fail(c, s, "job " + std::to_string(i) + ": " + c->last);
        const int n = jobs[i].order, v = (n - 1) * 2 + (int)jobs[i].path;
        need[v] = std::max(need[v], job_window_need(c, jobs + i));
        need3[v] = std::max(need3[v], job_window_need3(jobs + i));
        // per-pixel mesh work ~ (n+1)^4 taps x 7n^2 interpolation weights
        cost[i] = (double)jobs[i].width * jobs[i].height * std::pow(n + 1.0, 4) * 7.0 * n * n;
        vcost[v] += cost[i];
        order[i] = i;
    }
    // jobs grouped by variant, heaviest variant first, and heaviest jobs first within a
    // variant: their tiles are handed out first (longest-processing-time order)
    auto var = [&](int i) { return (jobs[i].order - 1) * 2 + (int)jobs[i].path; };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const int va = var(a), vb = var(b);
        if (va != vb) return vcost[va] > vcost[vb] || (vcost[va] == vcost[vb] && va < vb);
        return cost[a] > cost[b];
    });
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    long long total = 0;
    for (int k = 0; k < njobs; ++k)
        total += (long long)((jobs[order[k]].width + kTile - 1) / kTile) * ((jobs[order[k]].height + kTile - 1) / kTile);
    if (total >= (1ll << 31)) return fail(c, BSF_ERR_INVALID_ARG, "batch has too many tiles");
    // groups: contiguous runs of one variant in `order`
    struct Group {
        int v, j0, nj;
        long long first, count;
        Plan p;
    };
    std::vector<Group> groups;
    size_t scratch_bytes = 0;
    {
        long long items = 0;
        for (int k = 0; k < njobs;) {
            Group g{var(order[k]), k, 0, items, 0, Plan{}};
            while (k < njobs && var(order[k]) == g.v) {
                items += (long long)((jobs[order[k]].width + kTile - 1) / kTile) *
                         ((jobs[order[k]].height + kTile - 1) / kTile);
                ++k;
                ++g.nj;
            }
            g.count = items - g.first;
            g.p = plan_tiers(c, need[g.v], g.v / 2 + 1, need3[g.v]);
            if (!bsf_plan::plan_fits(c->limits(), g.p, g.v / 2 + 1))
                return fail(c, BSF_ERR_UNSUPPORTED, "the launch's LDS exceeds the device's limit");
            if (g.p.use3) {
                const long long grid3 = bsf_plan::grid3_of(c->limits(), g.count);
                scratch_bytes = std::max(scratch_bytes, (size_t)grid3 * (size_t)g.p.t3 * 8);
            }
            groups.push_back(g);
        }
    }
    const WorkLayout w = work_layout(total, njobs + kHdrSlots, scratch_bytes);
    int slot = -1;
    bsf_status s = acquire_slot(c, w.total, njobs + kHdrSlots, slot);
    if (s != BSF_OK) return s;
    bsf_ctx::Slot& sl = c->slot[slot];
    GroupHdr* hhdr = reinterpret_cast<GroupHdr*>(sl.host);
    for (int v = 0; v < kVariants; ++v) hhdr[v] = GroupHdr{0, 0, 0, 0};
    for (const Group& g : groups) hhdr[g.v] = GroupHdr{g.j0, g.nj, g.first, g.count};
    total = 0;
    for (int k = 0; k < njobs; ++k) {
        JobDesc d = make_desc(jobs + order[k], c->d_err);
        d.item_base = total;
        total += (long long)d.tiles_x * d.tiles_y;
        sl.host[kHdrSlots + k] = d;
    }
    char* work = (char*)sl.dev;
    const GroupHdr* dhdr = (const GroupHdr*)(work + w.jobs_off);
    const JobDesc* djobs = (const JobDesc*)(work + w.jobs_off) + kHdrSlots;
    e = hipMemcpyAsync(work + w.jobs_off, sl.host, sizeof(JobDesc) * (size_t)(njobs + kHdrSlots), hipMemcpyHostToDevice,
                       st);
    if (e != hipSuccess) return hip_fail(c, e, "uploading the batch descriptors");
    hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, st, (unsigned*)work);
    bool any3 = false;
    for (const Group& g : groups) any3 = any3 || g.p.use3;
    if (any3)  // tier 3's block words
        hipLaunchKernelGGL(clear_words, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                           (unsigned*)(work + w.blocks_off), (int)total);
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        const Group& g = groups[gi];
        unsigned* ctr = (unsigned*)work + 8 * g.v;  // each variant appears in one group
        const Tiers t = make_tiers_at(c, g.p, ctr, (int2*)(work + w.lists_off), (int2*)(work + w.listb_off),
                                      (unsigned*)(work + w.blocks_off), (long long*)(work + w.scratch_off), g.count,
                                      g.v / 2 + 1);
        e = dispatch_batch_group(c, g.v, djobs, dhdr + g.v, g.count, g.p, t, ctr, st);
        if (e != hipSuccess) return hip_fail(c, e, "batch kernel launch");
    }
    e = hipEventRecord(sl.done, st);
    if (e != hipSuccess) return hip_fail(c, e, "batch kernel launch");
    return BSF_OK;
}

bsf_status bsf_batch_plan_destroy(bsf_batch_plan* p) {
    if (!p) return BSF_ERR_INVALID_ARG;
    if (p->ctx) (void)hipSetDevice(p->ctx->device);
    if (p->done) (void)hipEventSynchronize(p->done);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->done) (void)hipEventDestroy(p->done);
    if (p->dev) (void)hipFree(p->dev);
    if (p->host) (void)hipHostFree(p->host);
    if (p->herr) (void)hipHostFree(p->herr);
    delete p;
    return BSF_OK;
}

bsf_status bsf_batch_plan_create(bsf_ctx* c, int max_jobs, long long max_tiles, float a_max, bsf_batch_plan** out) {
    if (!c || !out) return BSF_ERR_INVALID_ARG;
    *out = nullptr;
    if (max_jobs < 1 || max_jobs > (1 << 20)) return fail(c, BSF_ERR_INVALID_ARG, "max_jobs must lie in [1, 2^20]");
    if (max_tiles < 1 || max_tiles >= (1ll << 31)) return fail(c, BSF_ERR_INVALID_ARG, "max_tiles must lie in [1, 2^31)");
    if (!(a_max >= (float)kScaleMin && a_max <= (float)kScaleMax))
        return fail(c, BSF_ERR_INVALID_ARG, "a plan's a_max must lie in [0.5, 1e4]");
    constexpr int kVariants = 6;
    Plan pv[kVariants];
    size_t scratch_bytes = 0;
    for (int v = 0; v < kVariants; ++v) {
        const int n = v / 2 + 1;
        pv[v] = plan_tiers(c, window_bound(n, a_max) + 64, n, window_bound(n, a_max, -1, 2 * kTile) + 64);
        if (!bsf_plan::plan_fits(c->limits(), pv[v], n))
            return fail(c, BSF_ERR_UNSUPPORTED, "the launch's LDS exceeds the device's limit");
        if (pv[v].use3)
            scratch_bytes = std::max(scratch_bytes, (size_t)bsf_plan::grid3_of(c->limits(), max_tiles) * (size_t)pv[v].t3 * 8);
    }
    const WorkLayout w = work_layout(max_tiles, max_jobs + kHdrSlots, scratch_bytes);
    const size_t err_off = (w.total + 255) & ~(size_t)255;
    const size_t bytes = err_off + 4 * (size_t)max_jobs;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    bsf_batch_plan* p = new bsf_batch_plan();
    p->ctx = c;
    p->max_jobs = max_jobs;
    p->max_tiles = max_tiles;
    p->a_max = a_max;
    p->jobs_off = w.jobs_off;
    p->err_off = err_off;
    auto bail = [&](bsf_status st) {
        bsf_batch_plan_destroy(p);
        return st;
    };
    e = hipMalloc(&p->dev, bytes);
    if (e != hipSuccess) return bail(hip_fail(c, e, "plan work area"));
    e = hipHostMalloc((void**)&p->host, sizeof(JobDesc) * (size_t)(max_jobs + kHdrSlots));
    if (e != hipSuccess) return bail(hip_fail(c, e, "plan descriptor staging"));
    std::memset((void*)p->host, 0, sizeof(JobDesc) * (size_t)(max_jobs + kHdrSlots));
    e = hipHostMalloc((void**)&p->herr, 4 * (size_t)max_jobs);
    if (e != hipSuccess) return bail(hip_fail(c, e, "plan error staging"));
    std::memset(p->herr, 0, 4 * (size_t)max_jobs);
    e = hipEventCreateWithFlags(&p->done, hipEventDisableTiming);
    if (e != hipSuccess) return bail(hip_fail(c, e, "plan event"));
    opt_in_all_batch_kernels();  // before capture: no attribute calls inside it

    // Capture the launch sequence once on a private stream: upload the staged headers and
    // descriptors, clear the counters and error words (kernels, no memset nodes), run every
    // variant's tiers over persistent grids sized for the capacity, fetch the error words.
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return bail(hip_fail(c, e, "capture stream"));
    char* work = (char*)p->dev;
    unsigned* derr = (unsigned*)(work + err_off);
    hipGraph_t graph = nullptr;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = hipMemcpyAsync(work + w.jobs_off, p->host, sizeof(JobDesc) * (size_t)(max_jobs + kHdrSlots),
                                       hipMemcpyHostToDevice, cs);
        hipLaunchKernelGGL(reset_counters, dim3(1), dim3(64), 0, cs, (unsigned*)work);
        hipLaunchKernelGGL(clear_words, dim3((max_jobs + 255) / 256), dim3(256), 0, cs, derr, max_jobs);
        bool any3 = false;
        for (int v = 0; v < kVariants; ++v) any3 = any3 || pv[v].use3;
        if (any3)  // tier 3's block words
            hipLaunchKernelGGL(clear_words, dim3((unsigned)((max_tiles + 255) / 256)), dim3(256), 0, cs,
                               (unsigned*)(work + w.blocks_off), (int)max_tiles);
        const GroupHdr* dhdr = (const GroupHdr*)(work + w.jobs_off);
        const JobDesc* djobs = (const JobDesc*)(work + w.jobs_off) + kHdrSlots;
        for (int v = 0; v < kVariants && le == hipSuccess; ++v) {
            unsigned* ctr = (unsigned*)work + 8 * v;
            const Tiers t = make_tiers_at(c, pv[v], ctr, (int2*)(work + w.lists_off), (int2*)(work + w.listb_off),
                                          (unsigned*)(work + w.blocks_off), (long long*)(work + w.scratch_off),
                                          max_tiles, v / 2 + 1);
            le = dispatch_batch_group(c, v, djobs, dhdr + v, max_tiles, pv[v], t, ctr, cs);
        }
        if (le == hipSuccess)
            le = hipMemcpyAsync(p->herr, derr, 4 * (size_t)max_jobs, hipMemcpyDeviceToHost, cs);
        e = hipStreamEndCapture(cs, &graph);
        if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) return bail(hip_fail(c, e, "capturing the plan's launch sequence"));
    *out = p;
    return BSF_OK;
}

bsf_status bsf_batch_plan_run(bsf_batch_plan* p, const bsf_job* jobs, int njobs, void* stream) {
    if (!p) return BSF_ERR_INVALID_ARG;
    bsf_ctx* c = p->ctx;
    if (njobs < 0 || (njobs > 0 && !jobs)) return fail(c, BSF_ERR_INVALID_ARG, "bad batch");
    if (njobs > p->max_jobs) return fail(c, BSF_ERR_INVALID_ARG, "more jobs than the plan holds");
    constexpr int kVariants = 6;
    std::vector<int> order(njobs);
    std::vector<double> cost(njobs);
    double vcost[kVariants] = {};
    long long total = 0;
    for (int i = 0; i < njobs; ++i) {
        bsf_status s = validate(c, jobs + i, true);
        if (s != BSF_OK) return fail(c, s, "job " + std::to_string(i) + ": " + c->last);
        if (!(jobs[i].a_max > 0.0f && jobs[i].a_max <= p->a_max))
            return fail(c, BSF_ERR_INVALID_ARG, "job " + std::to_string(i) + ": a_max must lie in (0, the plan's a_max]");
        const int n = jobs[i].order;
        cost[i] = (double)jobs[i].width * jobs[i].height * std::pow(n + 1.0, 4) * 7.0 * n * n;
        vcost[(n - 1) * 2 + (int)jobs[i].path] += cost[i];
        total += (long long)((jobs[i].width + kTile - 1) / kTile) * ((jobs[i].height + kTile - 1) / kTile);
        order[i] = i;
    }
    if (total > p->max_tiles) return fail(c, BSF_ERR_INVALID_ARG, "the batch has more tiles than the plan holds");
    auto var = [&](int i) { return (jobs[i].order - 1) * 2 + (int)jobs[i].path; };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const int va = var(a), vb = var(b);
        if (va != vb) return vcost[va] > vcost[vb] || (vcost[va] == vcost[vb] && va < vb);
        return cost[a] > cost[b];
    });
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    // the staging is read by the previous replay's first node: wait until that replay is done
    e = hipEventSynchronize(p->done);
    if (e != hipSuccess) return hip_fail(c, e, "waiting for the plan's previous run");
    unsigned* derr = (unsigned*)((char*)p->dev + p->err_off);
    GroupHdr* hhdr = reinterpret_cast<GroupHdr*>(p->host);
    for (int v = 0; v < kVariants; ++v) hhdr[v] = GroupHdr{0, 0, 0, 0};
    long long item = 0;
    for (int k = 0; k < njobs;) {
        const int v = var(order[k]);
        GroupHdr h{k, 0, item, 0};
        while (k < njobs && var(order[k]) == v) {
            JobDesc d = make_desc(jobs + order[k], derr + order[k]);
            d.item_base = item;
            item += (long long)d.tiles_x * d.tiles_y;
            p->host[kHdrSlots + k] = d;
            ++k;
            ++h.nj;
        }
        h.count = item - h.first;
        hhdr[v] = h;
    }
    e = hipGraphLaunch(p->exec, (hipStream_t)stream);
    if (e == hipSuccess) e = hipEventRecord(p->done, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "plan replay");
    p->last_njobs = njobs;
    return BSF_OK;
}

bsf_status bsf_batch_plan_job_status(bsf_batch_plan* p, int* status, int njobs) {
    if (!p || (njobs > 0 && !status)) return BSF_ERR_INVALID_ARG;
    if (njobs < 0 || njobs > p->last_njobs) return fail(p->ctx, BSF_ERR_INVALID_ARG, "more jobs than the last run had");
    hipError_t e = hipSetDevice(p->ctx->device);
    if (e == hipSuccess) e = hipEventSynchronize(p->done);
    if (e != hipSuccess) return hip_fail(p->ctx, e, "waiting for the plan's run");
    for (int i = 0; i < njobs; ++i) {
        const unsigned h = p->herr[i];
        status[i] = (h & kErrScale) ? BSF_ERR_SCALE_RANGE
                    : (h & kErrWindow) ? BSF_ERR_UNSUPPORTED
                    : (h & kErrRange) ? BSF_ERR_RANGE
                                      : BSF_OK;
    }
    return BSF_OK;
}

bsf_status bsf_preintegrate(bsf_ctx* c, const bsf_job* j, int x0, int y0, int wq, int hq, int64_t* g,
                            ptrdiff_t g_pitch, void* stream) {
    if (!c) return BSF_ERR_INVALID_ARG;
    bsf_status s = validate(c, j, false);
    if (s != BSF_OK) return s;
    if (wq < 1 || hq < 1 || !g || g_pitch < wq) return fail(c, BSF_ERR_INVALID_ARG, "bad window");
    const size_t tp = ((size_t)(wq + hq - 1) + 3) & ~(size_t)3;
    const size_t need = (size_t)hq * tp * 8 + bsf::kZeros * 8;  // + the zero words
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    // the workspace is a slot of the context's ring: calls on different streams never share
    // one, and a slot is reused (or grown) only after its previous call has finished
    int slot = -1;
    s = acquire_slot(c, need, 0, slot);
    if (s != BSF_OK) return s;
    GlobalArgs A{};
    A.in = j->in;
    A.in_pitch = j->in_pitch;
    A.width = j->width;
    A.height = j->height;
    A.in_dtype = j->in_dtype;
    A.border = j->border;
    A.x0 = x0;
    A.y0 = y0;
    A.wq = wq;
    A.hq = hq;
    A.T = (long long*)c->slot[slot].dev;
    A.tp = (long long)tp;
    A.g = (long long*)g;
    A.g_pitch = g_pitch;
    hipStream_t st = (hipStream_t)stream;
    if (j->order == 1) bsf::launch_global<1>(A, st);
    else if (j->order == 2) bsf::launch_global<2>(A, st);
    else bsf::launch_global<3>(A, st);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(c->slot[slot].done, st);
    if (e != hipSuccess) return hip_fail(c, e, "pre-integration launch");
    return BSF_OK;
}

bsf_status bsf_get_device_error(bsf_ctx* c, void* stream) {
    if (!c) return BSF_ERR_INVALID_ARG;
    unsigned h = 0;
    hipError_t e = hipMemcpyAsync(&h, c->d_err, sizeof(unsigned), hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "reading the device error word");
    if (h) {
        e = hipMemsetAsync(c->d_err, 0, sizeof(unsigned), (hipStream_t)stream);
        if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(c, e, "clearing the device error word");
    }
    if (h & kErrScale) return fail(c, BSF_ERR_SCALE_RANGE, "a scale was not finite or outside [0.5, 1e4]");
    if (h & kErrWindow) return fail(c, BSF_ERR_UNSUPPORTED, "a restart window exceeded the on-chip memory");
    if (h & kErrRange) return fail(c, BSF_ERR_RANGE, "a pre-integrated value left the int64 range");
    return BSF_OK;
}

bsf_status bsf_get_counters(bsf_ctx* c, void* stream, unsigned long long* out, int reset) {
    if (!c || !out) return BSF_ERR_INVALID_ARG;
    hipError_t e = hipMemcpyAsync(out, c->d_stats, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                  (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e == hipSuccess && reset) {
        e = hipMemsetAsync(c->d_stats, 0, 2 * sizeof(unsigned long long), (hipStream_t)stream);
        if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    }
    if (e != hipSuccess) return hip_fail(c, e, "reading the evaluation counters");
    return BSF_OK;
}

bsf_status bsf_scales_from_ellipses(bsf_ctx* c, const float* ellipses, ptrdiff_t ellipse_pitch, int width,
                                    int height, int order, float* scales, ptrdiff_t scale_pitch, void* stream) {
    if (!c) return BSF_ERR_INVALID_ARG;
    if (!ellipses || !scales || width < 1 || height < 1 || ellipse_pitch < width || scale_pitch < width)
        return fail(c, BSF_ERR_INVALID_ARG, "bad ellipse or scale buffer");
    if (order < 1 || order > 3) return fail(c, BSF_ERR_INVALID_ARG, "order must be 1, 2 or 3");
    if ((reinterpret_cast<uintptr_t>(scales) & 15) != 0) return fail(c, BSF_ERR_INVALID_ARG, "scales must be 16-byte aligned");
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    const int bpr = (width + 511) / 512;
    if ((long long)bpr * height > 0x7fffffffll) return fail(c, BSF_ERR_INVALID_ARG, "image too large");
    hipLaunchKernelGGL(bsf::ellipse_scales_kernel, dim3(bpr * height), dim3(256), 0, (hipStream_t)stream, ellipses,
                       (long long)ellipse_pitch, width, bpr, order, scales, (long long)scale_pitch, c->d_err);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(c, e, "ellipse kernel launch");
    return BSF_OK;
}

bsf_status bsf_filter1d_max_scale(bsf_ctx* c, int order, int model, float* a_max) {
    if (!c) return BSF_ERR_INVALID_ARG;
    if (order < 1 || order > 3 || model < -1 || model > 3 || !a_max)
        return fail(c, BSF_ERR_INVALID_ARG, "order must be 1..3 and model -1..3");
    *a_max = (float)filter1d_max_scale(c, order, order + model);
    return BSF_OK;
}

bsf_status bsf_filter1d(bsf_ctx* c, const bsf_job1d* j, void* stream) {
    if (!c) return BSF_ERR_INVALID_ARG;
    if (!j) return fail(c, BSF_ERR_INVALID_ARG, "job is null");
    if (j->length < 1 || j->count < 1) return fail(c, BSF_ERR_INVALID_ARG, "length and count must be >= 1");
    if (j->length > 0x7fffffff - 2 * bsf::f1d::kWindowMax) return fail(c, BSF_ERR_INVALID_ARG, "signal too long");
    if (!j->in || !j->scales || !j->out) return fail(c, BSF_ERR_INVALID_ARG, "null buffer");
    if (j->in_pitch < j->length || j->scale_pitch < j->length || j->out_pitch < j->length)
        return fail(c, BSF_ERR_INVALID_ARG, "pitches must be >= length");
    if (j->in_dtype != BSF_U8 && j->in_dtype != BSF_F32 && j->in_dtype != BSF_F64)
        return fail(c, BSF_ERR_INVALID_ARG, "bad input dtype");
    if (j->border != BSF_BORDER_CLAMP && j->border != BSF_BORDER_ZERO) return fail(c, BSF_ERR_INVALID_ARG, "bad border");
    if (j->order < 1 || j->order > 3) return fail(c, BSF_ERR_INVALID_ARG, "order must be 1, 2 or 3");
    if (j->model < -1 || j->model > 3) return fail(c, BSF_ERR_INVALID_ARG, "model degree must lie in -1 .. 3");
    if (j->path != BSF_PATH_F64 && j->path != BSF_PATH_F32_TILED) return fail(c, BSF_ERR_INVALID_ARG, "bad path");
    const int n = j->order, D = j->order + j->model, path = (int)j->path;
    const double limit = filter1d_max_scale(c, n, D);
    double a_max = j->a_max;
    if (!(a_max == 0.0 || (a_max >= 0.5 && a_max <= 1e4)))
        return fail(c, BSF_ERR_INVALID_ARG, "a_max must be 0 or lie in [0.5, 1e4]");
    if (a_max == 0.0) a_max = limit;
    if (a_max > limit)
        return fail(c, BSF_ERR_UNSUPPORTED, "a_max " + std::to_string(a_max) + " exceeds the largest scale whose window fits on chip (" +
                                                std::to_string(limit) + ")");
    const long long tiles = (j->length + bsf::f1d::kT - 1) / bsf::f1d::kT;
    if (tiles * j->count > 0x7fffffffll) return fail(c, BSF_ERR_INVALID_ARG, "batch too large");
    bsf::f1d::Args A{};
    A.in = j->in;
    A.in_pitch = j->in_pitch;
    A.scales = j->scales;
    A.sc_pitch = j->scale_pitch;
    A.out = j->out;
    A.out_pitch = j->out_pitch;
    A.length = j->length;
    A.tiles = (int)tiles;
    A.dtype = (int)j->in_dtype;
    A.border = (int)j->border;
    A.left = bsf::f1d::window_left(n, D, a_max);
    A.W = bsf::f1d::window_len(n, D, a_max);
    A.a_max = (float)a_max;
    A.err = c->d_err;
    hipError_t e = hipSetDevice(c->device);
    if (e == hipSuccess)
        e = dispatch_filter1d(n, D, path, A, (int)(tiles * j->count), bsf::f1d::lds_bytes(D, A.W, path),
                              (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "filter1d launch");
    return BSF_OK;
}

bsf_status bsf_filter_rect_max_scale(bsf_ctx* c, int order, int model, float* a_max) {
    if (!c) return BSF_ERR_INVALID_ARG;
    if (order < 1 || order > 3 || model < -1 || model > 3 || !a_max)
        return fail(c, BSF_ERR_INVALID_ARG, "order must be 1..3 and model -1..3");
    *a_max = (float)rect_max_scale(c, order, order + model);
    return BSF_OK;
}

bsf_status bsf_filter_rect(bsf_ctx* c, const bsf_job_rect* j, void* stream) {
    if (!c) return BSF_ERR_INVALID_ARG;
    if (!j) return fail(c, BSF_ERR_INVALID_ARG, "job is null");
    if (j->width < 1 || j->height < 1) return fail(c, BSF_ERR_INVALID_ARG, "width and height must be >= 1");
    if (j->width > (1 << 24) || j->height > (1 << 24)) return fail(c, BSF_ERR_INVALID_ARG, "image too large");
    if (!j->in || !j->scales || !j->out) return fail(c, BSF_ERR_INVALID_ARG, "null buffer");
    if (((uintptr_t)j->scales) % 8) return fail(c, BSF_ERR_INVALID_ARG, "scales must be 8-byte aligned");
    if (j->in_pitch < j->width || j->scale_pitch < j->width || j->out_pitch < j->width)
        return fail(c, BSF_ERR_INVALID_ARG, "pitches must be >= width");
    if (j->in_dtype != BSF_U8 && j->in_dtype != BSF_F32 && j->in_dtype != BSF_F64)
        return fail(c, BSF_ERR_INVALID_ARG, "bad input dtype");
    if (j->border != BSF_BORDER_CLAMP && j->border != BSF_BORDER_ZERO) return fail(c, BSF_ERR_INVALID_ARG, "bad border");
    if (j->order < 1 || j->order > 3) return fail(c, BSF_ERR_INVALID_ARG, "order must be 1, 2 or 3");
    if (j->model < -1 || j->model > 3) return fail(c, BSF_ERR_INVALID_ARG, "model degree must lie in -1 .. 3");
    if (j->path != BSF_PATH_F64 && j->path != BSF_PATH_F32_TILED) return fail(c, BSF_ERR_INVALID_ARG, "bad path");
    const int n = j->order, D = j->order + j->model;
    double a_max = j->a_max;
    if (!(a_max == 0.0 || (a_max >= 0.5 && a_max <= 1e4)))
        return fail(c, BSF_ERR_INVALID_ARG, "a_max must be 0 or lie in [0.5, 1e4]");
    const double limit = rect_max_scale(c, n, D);
    if (a_max == 0.0) a_max = limit;
    if (a_max > limit)
        return fail(c, BSF_ERR_UNSUPPORTED, "a_max " + std::to_string(a_max) +
                                                " exceeds the largest scale whose window fits on chip (" +
                                                std::to_string(limit) + ")");
    bsf::rect::Args A{};
    A.in = j->in;
    A.in_pitch = j->in_pitch;
    A.dtype = (int)j->in_dtype;
    A.border = (int)j->border;
    A.scales = j->scales;
    A.sc_pitch = j->scale_pitch;
    A.out = j->out;
    A.out_pitch = j->out_pitch;
    A.width = j->width;
    A.height = j->height;
    A.path = (int)j->path;
    A.T = rect_tile(c, n, D, a_max);
    A.tiles_x = (j->width + A.T - 1) / A.T;
    A.tiles_y = (j->height + A.T - 1) / A.T;
    A.left = bsf::rect::halo_left(n, D, a_max);
    A.right = bsf::rect::halo_right(n, D, a_max);
    A.wx = A.T + A.left + A.right;
    A.pitch = bsf::rect::lds_pitch(A.wx);
    A.a_max = (float)a_max;
    A.err = c->d_err;
    const long long lds = bsf::rect::lds_bytes(A.T, n, D, a_max);
    const long long tiles = (long long)A.tiles_x * A.tiles_y;
    if (tiles > 0x7fffffffll) return fail(c, BSF_ERR_INVALID_ARG, "image too large");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(c, e, "hipSetDevice");
    if (j->model <= 1) {
        e = dispatch_rect_src<0>(n, D, A, (int)tiles, lds, st);
        if (e != hipSuccess) return hip_fail(c, e, "rect kernel launch");
        return BSF_OK;
    }
    // degree-2/3 models: c = f_ext filtered by the inverse interpolation filter, over the
    // domain every window reads, in a work slot (rows pass into h, columns pass into c)
    const int K = j->model == 2 ? bsf::f1d::Prefilter<2>::K : bsf::f1d::Prefilter<3>::K;
    bsf::rect::PrefArgs Pa{};
    Pa.in = j->in;
    Pa.in_pitch = j->in_pitch;
    Pa.dtype = (int)j->in_dtype;
    Pa.border = (int)j->border;
    Pa.width = j->width;
    Pa.height = j->height;
    Pa.org = -A.left;
    Pa.cw = A.tiles_x * A.T + A.left + A.right;
    Pa.ch = A.tiles_y * A.T + A.left + A.right;
    Pa.pitch = ((long long)Pa.cw + 31) & ~31ll;
    const size_t hbytes = (size_t)(Pa.ch + 2 * K) * Pa.pitch * 8, cbytes = (size_t)Pa.ch * Pa.pitch * 8;
    int slot = -1;
    bsf_status s = acquire_slot(c, hbytes + cbytes, 0, slot);
    if (s != BSF_OK) return s;
    Pa.h = (double*)c->slot[slot].dev;
    Pa.c = Pa.h + (size_t)(Pa.ch + 2 * K) * Pa.pitch;
    A.cbuf = Pa.c;
    A.cpitch = Pa.pitch;
    const long long hn = (long long)(Pa.ch + 2 * K) * Pa.cw, cn = (long long)Pa.ch * Pa.cw;
    const int gh = (int)std::min<long long>((hn + 255) / 256, 65536), gc = (int)std::min<long long>((cn + 255) / 256, 65536);
    if (j->model == 2) {
        hipLaunchKernelGGL(bsf::rect::rect_prefilter_rows<2>, dim3(gh), dim3(256), 0, st, Pa);
        hipLaunchKernelGGL(bsf::rect::rect_prefilter_cols<2>, dim3(gc), dim3(256), 0, st, Pa);
    } else {
        hipLaunchKernelGGL(bsf::rect::rect_prefilter_rows<3>, dim3(gh), dim3(256), 0, st, Pa);
        hipLaunchKernelGGL(bsf::rect::rect_prefilter_cols<3>, dim3(gc), dim3(256), 0, st, Pa);
    }
    e = hipGetLastError();
    if (e == hipSuccess) e = dispatch_rect_src<1>(n, D, A, (int)tiles, lds, st);
    if (e == hipSuccess) e = hipEventRecord(c->slot[slot].done, st);
    if (e != hipSuccess) return hip_fail(c, e, "rect kernel launch");
    return BSF_OK;
}

// Test aid: stage 1 of one tile, written out as the int64 box part of its window.
// geom (device int[6]): in [4] the caller puts 1 for centred anchors, 0 for the
// recursions' own zero start; out [0..3] = x0, y0, wq, hq, [5] = overflow flag.
bsf_status bsf_debug_tile_window(bsf_ctx* c, const bsf_job* j, int tile, int64_t* window, long long cap,
                                 int* geom, void* stream) {
    if (!c) return BSF_ERR_INVALID_ARG;
    bsf_status s = validate(c, j, true);
    if (s != BSF_OK) return s;
    const JobDesc A = make_desc(j, c->d_err);
    if (tile < 0 || tile >= A.tiles_x * A.tiles_y || !window || !geom)
        return fail(c, BSF_ERR_INVALID_ARG, "bad debug tile arguments");
    const long long full = (c->lds_max_bytes - c->lds_static[j->order]) / 8;
    Launch L{};
    L.lds_cap = std::min(job_window_need(c, j), full);
    if (!bsf_plan::launch_fits(c->limits(), j->order, L.lds_cap * 8))
        return fail(c, BSF_ERR_UNSUPPORTED, "the launch's LDS exceeds the device's limit");
    L.dbg_window = (long long*)window;
    L.dbg_geom = geom;
    L.dbg_cap = cap;
    hipError_t e = hipSetDevice(c->device);
    if (e == hipSuccess) e = dispatch_debug(j->order, j->path, A, L, tile, (size_t)L.lds_cap * 8, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(c, e, "debug tile launch");
    return BSF_OK;
}

}  // extern "C"
