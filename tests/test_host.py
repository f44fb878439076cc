"""Host-side logic that needs no GPU: library symbols, input recipes, admission policy."""
import collections
import ctypes
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_0908_3861_amd", "libbsf.so")
HDR = os.path.join(ROOT, "include", "bsf.h")


def declared_functions():
    src = open(HDR).read()
    return sorted(set(re.findall(r"^(?:bsf_status|const char\*)\s+(bsf_\w+)\(", src, re.M)))


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbsf.so not built")
def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 9
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if l.strip())
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    lib = ctypes.CDLL(LIB)  # loads without a GPU
    for n in names:
        assert getattr(lib, n) is not None
    lib.bsf_status_string.restype = ctypes.c_char_p
    assert lib.bsf_status_string(0) == b"ok"
    assert lib.bsf_status_string(5) == b"scale out of range"


@pytest.mark.skipif(not os.path.exists(LIB), reason="libbsf.so not built")
def test_workspace_size_is_host_only():
    from paper_0908_3861_amd import binding
    lib = ctypes.CDLL(LIB)
    lib.bsf_workspace_size.argtypes = [ctypes.POINTER(binding.Job), ctypes.POINTER(ctypes.c_size_t)]
    j = binding.Job()
    j.width, j.height, j.in_dtype, j.in_, j.in_pitch = 100, 50, 2, 16, 100
    j.scales, j.scale_pitch, j.order, j.path, j.border, j.a_max = 64, 100, 2, 0, 0, 4.0
    j.out, j.out_pitch = 32, 100
    n = ctypes.c_size_t()
    assert lib.bsf_workspace_size(ctypes.byref(j), ctypes.byref(n)) == 0
    assert n.value == 0  # every window fits half the LDS: tier 1 alone, no work area
    j.a_max = 14.0  # windows of ~100 KB: the tiles go through the overflow lists of tier 2
    assert lib.bsf_workspace_size(ctypes.byref(j), ctypes.byref(n)) == 0
    assert 2 * 7 * 4 * 8 <= n.value < 1 << 16
    j.a_max = 40.0  # beyond the LDS: tier-3 scratch slices, one per tile here (28 tiles)
    assert lib.bsf_workspace_size(ctypes.byref(j), ctypes.byref(n)) == 0
    assert n.value > 28 * 160 * 1024
    j.a_max = 0.25  # neither 0 nor an admissible bound
    assert lib.bsf_workspace_size(ctypes.byref(j), ctypes.byref(n)) == 1
    j.a_max = 4.0
    j.order = 7
    assert lib.bsf_workspace_size(ctypes.byref(j), ctypes.byref(n)) == 4  # unsupported order
    j.order, j.scales = 2, 66  # misaligned scale field
    assert lib.bsf_workspace_size(ctypes.byref(j), ctypes.byref(n)) == 1


def test_input_recipes():
    from paper_0908_3861_amd import synth
    rng = np.random.default_rng(0)
    img = synth.unit_grid_image(rng, 64, 32, np.float32)
    assert img.dtype == np.float32 and np.all(img * 2 ** 24 == np.round(img * 2 ** 24))
    u8 = synth.blurred_u8_image(rng, 128, 96, 3.0)
    assert u8.dtype == np.uint8 and u8.min() == 0 and u8.max() == 255
    sc = synth.smooth_scales(rng, 128, 96, 1.0, 16.0, 32.0)
    assert sc.dtype == np.float32 and sc.min() >= 1.0 and sc.max() <= 16.0
    for d in range(4):
        assert abs(sc[..., d].min() - 1.0) < 1e-4 and abs(sc[..., d].max() - 16.0) < 1e-4
    ii = synth.integer_scales(rng, 10, 10, 1, 8)
    assert set(np.unique(ii)) <= set(range(1, 9))
    jobs = synth.batch_jobs(count=6, seed=1, side_hi=512)
    assert all(j.image.shape[0] % 64 == 0 and j.order in (1, 2, 3) for j in jobs)
    reqs = synth.serving_requests(2.0, 5.0, seed=3, side_hi=256)
    assert all(0 <= t < 2.0 for t, _ in reqs)
    assert all(128 <= r.image.shape[0] <= 256 for _, r in reqs)


def test_admission_is_fifo_by_footprint_and_slots():
    from paper_0908_3861_amd.serve import Admission
    adm = Admission(budget_bytes=100, slots=3)
    pend = collections.deque([40, 50, 30, 5])
    g = adm.admit(pend, max_group=8, footprint=lambda r: r)
    assert g == [40, 50] and list(pend) == [30, 5]  # 30 does not fit; 5 may not overtake it
    adm.release(40)
    g = adm.admit(pend, max_group=8, footprint=lambda r: r)
    assert g == [30, 5] and not pend and adm.busy == 3 and adm.used == 85
    pend.append(1)
    assert adm.admit(pend, max_group=8, footprint=lambda r: r) == []  # all three slots busy
    adm2 = Admission(budget_bytes=10 ** 9, slots=2)
    pend = collections.deque([1, 1, 1])
    assert len(adm2.admit(pend, 8, footprint=lambda r: r)) == 2  # slot limit
    # the tiles one launch holds: a group stops before the request that would overflow it
    adm3 = Admission(budget_bytes=10 ** 9, slots=8)
    pend = collections.deque([300, 500, 300, 100])
    g = adm3.admit(pend, 8, footprint=lambda r: 1, max_tiles=1000, tiles=lambda r: r)
    assert g == [300, 500] and list(pend) == [300, 100]
    assert adm3.admit(pend, 8, footprint=lambda r: 1, max_tiles=1000, tiles=lambda r: r) == [300, 100]


def test_rep3_groups_header_is_current(tmp_path):
    """rep3_groups.h is what gen_rep_groups.py writes from the committed order-3 table."""
    csrc = os.path.join(ROOT, "paper_0908_3861_amd", "csrc")
    out = tmp_path / "rep3_groups.h"
    subprocess.run([sys.executable, os.path.join(csrc, "gen_rep_groups.py"), "--out", str(out)], check=True,
                   capture_output=True)
    assert out.read_text() == open(os.path.join(csrc, "rep3_groups.h")).read()


def test_model_tables_header_is_current(tmp_path):
    """model_tables.h is what gen_tables.py writes for the continuous models (degrees 0, 1)."""
    csrc = os.path.join(ROOT, "paper_0908_3861_amd", "csrc")
    out = tmp_path / "model_tables.h"
    subprocess.run([sys.executable, os.path.join(csrc, "gen_tables.py"), "--orders", "", "--models-out", str(out)],
                   check=True, capture_output=True)
    assert out.read_text() == open(os.path.join(csrc, "model_tables.h")).read()


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes job structures have the C layout of include/bsf.h (field offsets and size),
    checked by compiling the header with gcc."""
    from paper_0908_3861_amd import binding
    structs = {"bsf_job": binding.Job, "bsf_job1d": binding.Job1d, "bsf_job_rect": binding.JobRect}
    rename = {"in_": "in"}
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HDR}"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            c = rename.get(fname, fname)
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {c}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-o", str(exe), str(src)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


PLAN_DRIVER = r'''
#include <cstdio>
#include <cstdlib>
#include "plan.h"
using namespace bsf_plan;
static int fails = 0;
#define CHECK(c) do { if (!(c)) { std::printf("FAIL line %d: %s\n", __LINE__, #c); ++fails; } } while (0)
int main() {
    // every plan's LDS launches fit, for any static reserve the kernels may declare
    for (long long st : {0ll, 1024ll, 5376ll, 12288ll, 40000ll})
        for (int order = 1; order <= 3; ++order) {
            Limits L{163840, {st, st, st, st}, 256};
            const long long full = full_cap(L, order), half = half_cap(L, order);
            CHECK(launch_fits(L, order, full * 8) && !launch_fits(L, order, full * 8 + 8));
            for (long long need : {1ll, half - 1, half, half + 1, full - 1, full, full + 1, 10 * full}) {
                const Plan p = plan_tiers(L, need, order);
                CHECK(plan_fits(L, p, order));
                CHECK(p.t1 <= half);                                  // two workgroups per CU
                CHECK((need <= half) == !p.use2);
                CHECK((need > full) == p.use3);
                CHECK(!p.use3 || p.t3 == need);                      // tier 3 holds any window
                const Plan p3 = plan_tiers(L, need, order, 2 * need);  // and any 2x2 block's window
                CHECK(!p3.use3 || p3.t3 == 2 * need);
                CHECK(p.use3 == (p.band > 0) && p.band <= half);      // tier 3's LDS band buffer
                CHECK(p.use3 || (p.use2 ? p.t2 : p.t1) >= need);      // the last LDS tier holds it
                // the bound used without a device never plans a smaller work area
                const Limits B = gfx950_bound();
                if (st <= B.lds_static[order])
                    for (long long tiles : {1ll, 7ll, 4096ll})
                        CHECK(single_call_bytes(B, plan_tiers(B, need, order), tiles) >=
                              single_call_bytes(L, p, tiles));
            }
        }
    // a static reserve the planner does not know about is caught before the launch
    {
        Limits L{163840, {0, 1024, 1024, 1024}, 256};
        const Plan p = plan_tiers(L, full_cap(L, 2), 2);
        Limits M = L;
        M.lds_static[2] = 4096;
        CHECK(plan_fits(L, p, 2) && !plan_fits(M, p, 2));
        // tier 3's band buffer is checked as well
        Plan q = plan_tiers(L, 10 * full_cap(L, 2), 2);
        CHECK(q.use3 && plan_fits(L, q, 2));
        q.band = full_cap(L, 2) + 1;
        CHECK(!plan_fits(L, q, 2));
        q.band = kBandTail;  // no room beside the float64 path's digit sums
        CHECK(!plan_fits(L, q, 2));
    }
    // work area of a fixed buffer: lists, then at least one tier-3 slice
    {
        const Limits L{163840, {0, 2048, 2048, 6144}, 256};
        const Plan p = plan_tiers(L, 50000, 2);
        CHECK(p.use3);
        const FixedArea a = fixed_area(L, p, 1000, (size_t)32 << 20);
        CHECK(a.ok && a.grid3 >= 1 && a.grid3 <= grid3_of(L, 1000) && a.bytes <= ((size_t)32 << 20));
        CHECK(!fixed_area(L, plan_tiers(L, 5000000, 2), 1000, (size_t)32 << 20).ok);  // one slice too large
        CHECK(!fixed_area(L, p, 5000000, (size_t)32 << 20).ok);                      // lists too large
        CHECK(fixed_area(L, plan_tiers(L, 100, 2), 5000000, 0).ok);                   // tier 1: no area
    }
    // the slot ring never holds more than the workspace limit
    {
        srand(7);
        for (int trial = 0; trial < 20000; ++trial) {
            size_t cur[kRing], tgt[kRing];
            const size_t limit = (size_t)(rand() % 4096 + 1) << (rand() % 12);
            size_t tot = 0;
            for (int r = 0; r < kRing; ++r) {
                cur[r] = (rand() & 1) ? (size_t)(rand() % 2048) << (rand() % 10) : 0;
                if (tot + cur[r] > limit) cur[r] = 0;
                tot += cur[r];
            }
            const int idx = rand() % kRing;
            const size_t bytes = (size_t)(rand() % 4096) << (rand() % 12);
            const bool ok = ring_growth(cur, idx, bytes, limit, tgt);
            size_t after = 0;
            for (int r = 0; r < kRing; ++r) after += tgt[r];
            CHECK(ok == (bytes <= limit));
            if (ok) {
                CHECK(tgt[idx] >= bytes);
                CHECK(after <= limit || after == tot);  // within the limit (or untouched)
                for (int r = 0; r < kRing; ++r) CHECK(r == idx || tgt[r] <= cur[r] || tgt[r] == tgt[idx]);
            }
        }
        size_t cur[kRing] = {0}, tgt[kRing];
        CHECK(ring_growth(cur, 3, 1000, (size_t)1 << 30, tgt));
        for (int r = 0; r < kRing; ++r) CHECK(tgt[r] == ((size_t)1 << 16));  // every slot grows at once
    }
    std::printf("fails %d\n", fails);
    return fails != 0;
}
'''


def test_launch_plan_arithmetic(tmp_path):
    """The host planner (csrc/plan.h): every launch's dynamic + static LDS fits the device,
    tiers hold their windows, the device-free workspace bound never undercuts a device's
    plan, a fixed buffer is carved into lists and tier-3 slices, and the slot ring stays
    within the workspace limit.  Compiled on its own with g++ (plain C++, no device code)."""
    src = tmp_path / "plan_driver.cpp"
    src.write_text(PLAN_DRIVER)
    exe = tmp_path / "plan_driver"
    csrc = os.path.join(ROOT, "paper_0908_3861_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-I", csrc, "-o", str(exe), str(src)], check=True,
                   capture_output=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True)
    assert res.returncode == 0, res.stdout
    assert "fails 0" in res.stdout
