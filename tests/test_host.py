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
    assert n.value >= 7 * 4 * 8  # room for every tile in the overflow list
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


def test_rep3_groups_header_is_current(tmp_path):
    """rep3_groups.h is what gen_rep_groups.py writes from the committed order-3 table."""
    csrc = os.path.join(ROOT, "paper_0908_3861_amd", "csrc")
    out = tmp_path / "rep3_groups.h"
    subprocess.run([sys.executable, os.path.join(csrc, "gen_rep_groups.py"), "--out", str(out)], check=True,
                   capture_output=True)
    assert out.read_text() == open(os.path.join(csrc, "rep3_groups.h")).read()


def test_binding_structs_match_the_header(tmp_path):
    """The ctypes job structures have the C layout of include/bsf.h (field offsets and size),
    checked by compiling the header with gcc."""
    from paper_0908_3861_amd import binding
    structs = {"bsf_job": binding.Job, "bsf_job1d": binding.Job1d}
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
