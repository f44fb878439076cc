// Host-side launch planning of libbsf: the launch tier a restart window runs in, the LDS
// each launch asks for, the device work area of one call, the work area of a call that
// must live in a fixed buffer, and the workspace accounting of a context's slot ring.
// Plain C++ with no device code, so that the arithmetic can be compiled and checked on
// its own; the kernels never see it.
#pragma once

#include <algorithm>
#include <cstddef>

namespace bsf_plan {

// What the planner needs to know about the device.
struct Limits {
    long long lds_max;        // LDS bytes one workgroup may hold (dynamic + static)
    long long lds_static[4];  // per order n (index n): the largest static LDS of its kernels
    int cus;                  // compute units
};

// A bound for an MI355X (gfx950) when no device is at hand: 160 KiB of LDS per workgroup,
// 256 compute units, and a static-LDS reserve above what any kernel of the library declares
// (the largest is under 12 KiB), so that plans made with it never pick a smaller tier than a
// device would.
inline Limits gfx950_bound() {
    Limits L{};
    L.lds_max = 163840;
    for (int n = 0; n < 4; ++n) L.lds_static[n] = 16384;
    L.cus = 256;
    return L;
}

// Window capacities (int64 elements) of the three launch tiers: tier 1 half the LDS (two
// workgroups per CU), tier 2 the full LDS, tier 3 a per-workgroup slice of global scratch
// holding the window of a 2x2 block of tiles, whose mesh reads it from an LDS band buffer
// of `band` elements (half the LDS).
struct Plan {
    long long t1 = 0, t2 = 0, t3 = 0, band = 0;
    bool use2 = false, use3 = false;
};

inline long long full_cap(const Limits& L, int order) { return (L.lds_max - L.lds_static[order]) / 8; }
inline long long half_cap(const Limits& L, int order) { return (L.lds_max / 2 - L.lds_static[order]) / 8; }

// The tiers for tile windows of up to `need` elements (block windows of up to `need3`).
inline Plan plan_tiers(const Limits& L, long long need, int order, long long need3 = 0) {
    const long long full = full_cap(L, order), half = half_cap(L, order);
    Plan p;
    if (need <= half) {
        p.t1 = need;
    } else if (need <= full) {
        p.t1 = half;
        p.t2 = need;
        p.use2 = true;
    } else {
        p.t1 = half;
        p.t2 = full;
        p.t3 = std::max(need, need3);
        p.band = half;
        p.use2 = p.use3 = true;
    }
    return p;
}

// A launch asking for `dyn_bytes` of dynamic LDS fits next to the static LDS of the
// order's kernels.
inline bool launch_fits(const Limits& L, int order, long long dyn_bytes) {
    return dyn_bytes >= 0 && dyn_bytes + L.lds_static[order] <= L.lds_max;
}

// Elements of tier 3's band buffer that the float64 path reserves for its pixels' digit sums
// (4 tiles x 2 doubles x 256 threads); the buffer must hold more than these.
constexpr long long kBandTail = 8 * 256;

// Every LDS launch of a plan fits (tier 3's dynamic LDS is its band buffer, which must hold
// more than its tail).
inline bool plan_fits(const Limits& L, const Plan& p, int order) {
    return launch_fits(L, order, p.t1 * 8) && (!p.use2 || launch_fits(L, order, p.t2 * 8)) &&
           (!p.use3 || (launch_fits(L, order, p.band * 8) && p.band > kBandTail));
}

// Workgroups of a window size that fit one CU's LDS.
inline int per_cu(const Limits& L, long long elems, int order) {
    return (int)std::max(1ll, L.lds_max / (elems * 8 + L.lds_static[order]));
}

// Persistent workgroups of the tier-3 launch: two per CU, at most one per tile.
inline long long grid3_of(const Limits& L, long long tiles) { return std::min<long long>(tiles, (long long)L.cus * 2); }

// Device work area of one call: counters | list A | list B | tier-3 block words | job
// descriptors | scratch.
struct WorkLayout {
    size_t lists_off = 256, listb_off = 0, blocks_off = 0, jobs_off = 0, scratch_off = 0, total = 0;
};

inline WorkLayout work_layout(long long items, int njobs, size_t job_desc_bytes, size_t scratch_bytes) {
    WorkLayout w;
    w.listb_off = w.lists_off + (size_t)items * 8;  // (job, tile) pairs of two ints
    w.blocks_off = w.listb_off + (size_t)items * 8;  // one word per item
    w.jobs_off = ((w.blocks_off + (size_t)items * 4) + 63) & ~(size_t)63;
    w.scratch_off = ((w.jobs_off + (size_t)njobs * job_desc_bytes) + 255) & ~(size_t)255;
    w.total = w.scratch_off + scratch_bytes;
    return w;
}

// Bytes of the work area of one single-job call with plan p over `tiles` tiles (0 when
// only tier 1 runs: it needs no work area).
inline size_t single_call_bytes(const Limits& L, const Plan& p, long long tiles) {
    if (!p.use2) return 0;
    const size_t scratch = p.use3 ? (size_t)grid3_of(L, tiles) * (size_t)p.t3 * 8 : 0;
    return work_layout(tiles, 0, 0, scratch).total;
}

// A single-job call whose work area must live in a fixed buffer of `cap` bytes: the lists
// as usual, and as many tier-3 window slices as fit (at least one, at most grid3_of).
struct FixedArea {
    bool ok = false;
    size_t bytes = 0;  // of the buffer the call uses
    long long grid3 = 0;
};

inline FixedArea fixed_area(const Limits& L, const Plan& p, long long tiles, size_t cap) {
    FixedArea f;
    if (!p.use2) {
        f.ok = true;
        return f;
    }
    const WorkLayout w = work_layout(tiles, 0, 0, 0);
    if (w.total > cap) return f;
    if (p.use3) {
        const size_t slice = (size_t)p.t3 * 8;
        const long long fit = (long long)((cap - w.total) / slice);
        if (fit < 1) return f;
        f.grid3 = std::min<long long>(fit, grid3_of(L, tiles));
        f.bytes = w.total + (size_t)f.grid3 * slice;
    } else {
        f.bytes = w.total;
    }
    f.ok = true;
    return f;
}

// The slot ring of a context: kRing device work areas, each reused once the call that last
// used it has finished.  ring_growth decides the sizes after a call on slot `idx` asks for
// `bytes`: the slot grows to at least `bytes` (64 KiB at the least), the other slots grow
// with it while the ring's total stays within `limit` (so calls of this size do not
// allocate again), and when the slot alone would push the total past the limit the other
// slots are released first.  Returns false if `bytes` exceeds the limit itself.
constexpr int kRing = 8;

inline bool ring_growth(const size_t (&cur)[kRing], int idx, size_t bytes, size_t limit, size_t (&target)[kRing]) {
    for (int r = 0; r < kRing; ++r) target[r] = cur[r];
    if (bytes > limit) return false;
    if (cur[idx] >= bytes) return true;
    size_t cap = std::max(bytes, (size_t)1 << 16);
    if (cap > limit) cap = bytes;
    target[idx] = cap;
    auto total = [&]() {
        size_t t = 0;
        for (int r = 0; r < kRing; ++r) t += target[r];
        return t;
    };
    for (int r = 0; r < kRing && total() > limit; ++r)
        if (r != idx) target[r] = 0;
    for (int r = 0; r < kRing; ++r)
        if (r != idx && target[r] < cap && total() - target[r] + cap <= limit) target[r] = cap;
    return true;
}

}  // namespace bsf_plan
