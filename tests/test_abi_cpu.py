"""The C ABI library loads, exports every function include/mm.h declares, and
rejects bad arguments before touching the device (no GPU needed)."""

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mm_[a-z_A-Z0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def mm():
    import paper_1309_7473_amd as mm
    return mm


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("mm_create_scan", "mm_apply_A", "mm_rhs", "mm_build_precon",
              "mm_apply_precon_binned", "mm_apply_precon_circulant", "mm_pcg_solve",
              "mm_last_error", "mm_scan_workspace_bytes", "mm_destroy_scan"):
        assert n in names


def test_library_exports_every_declared_symbol(mm):
    lib = C.CDLL(mm.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding wraps each of them under the same name
    for n in declared_functions():
        assert hasattr(mm, n), n


def _desc(mm, **kw):
    d = mm.mm_scan_desc()
    d.ncomp, d.ny, d.nx, d.ndet, d.tod_dtype, d.nsamp = 3, 64, 64, 4, mm.MM_F32, 1 << 16
    for k, v in kw.items():
        setattr(d, k, v)
    return d


def test_workspace_query_and_plan(mm):
    d = _desc(mm)
    nb = mm.mm_scan_workspace_bytes(d)
    assert nb > 0 and nb % 256 == 0
    # grows with detector-group size (timestream scratch) for a four-step plan
    d2 = _desc(mm, det_group=1, scatter=mm.MM_SCATTER_ATOMIC)
    d3 = _desc(mm, det_group=4, scatter=mm.MM_SCATTER_ATOMIC)
    assert mm.mm_scan_workspace_bytes(d3) - mm.mm_scan_workspace_bytes(d2) == 3 * (1 << 15) * 8


def test_pixel_index_workspace(mm):
    # the run-length index is sized for one 4 B run a sample (the worst case);
    # I,Q,U adds 4 B of time-major angles and 4 B of pixel-major angles a
    # sample (with a per-pixel offset table).  The per-sample index costs 12 B
    # a sample for I,Q,U (index and float32 weight pairs, or index and
    # angles) plus the 4 B of time-major angles, and 4 B for I
    a = mm.mm_scan_workspace_bytes(_desc(mm, scatter=mm.MM_SCATTER_ATOMIC))
    b = mm.mm_scan_workspace_bytes(_desc(mm, pointing_code=mm.MM_PTC_OFF))
    c = mm.mm_scan_workspace_bytes(_desc(mm, scatter=mm.MM_SCATTER_SAMPLES,
                                         pointing_code=mm.MM_PTC_OFF))
    S = 4 * (1 << 16)
    tail = 2 * 4 * (64 * 64 + 1) + 4 * 256
    assert 12 * S <= b - a <= 12 * S + tail + 4 * (64 * 64 + 1) + 256
    assert 16 * S <= c - a <= 16 * S + tail
    a1 = mm.mm_scan_workspace_bytes(_desc(mm, ncomp=1, scatter=mm.MM_SCATTER_ATOMIC))
    b1 = mm.mm_scan_workspace_bytes(_desc(mm, ncomp=1))
    c1 = mm.mm_scan_workspace_bytes(_desc(mm, ncomp=1, scatter=mm.MM_SCATTER_SAMPLES))
    assert 4 * S <= b1 - a1 <= 4 * S + 2 * 4 * (64 * 64 + 1) + 3 * 256
    assert c1 == b1


def test_chunk_coded_pointing_workspace(mm):
    # pass 1's chunk-coded pointing: 4 B a sample and 16 B per 64-sample chunk
    # for I,Q,U stored pointing on the float32 and bfloat16 four-step paths,
    # nothing for I only, float64 or pointing_code = MM_PTC_OFF
    S = 4 * (1 << 16)
    for kw in ({}, {"scatter": mm.MM_SCATTER_SAMPLES}, {"tod_dtype": mm.MM_BF16}):
        on = mm.mm_scan_workspace_bytes(_desc(mm, **kw))
        off = mm.mm_scan_workspace_bytes(_desc(mm, pointing_code=mm.MM_PTC_OFF, **kw))
        want = 4 * S + 16 * (S // 64)
        assert want <= on - off <= want + 2 * 256, kw
    for kw in ({"ncomp": 1}, {"tod_dtype": mm.MM_F64}, {"scatter": mm.MM_SCATTER_ATOMIC},
               {"nsamp": 1 << 12}):
        on = mm.mm_scan_workspace_bytes(_desc(mm, **kw))
        off = mm.mm_scan_workspace_bytes(_desc(mm, pointing_code=mm.MM_PTC_OFF, **kw))
        assert on == off > 0, kw


def test_bf16_pass_buffer_is_half_of_f32(mm):
    # bfloat16 storage: 4 B per packed complex in the pass buffer instead of 8
    a = mm.mm_scan_workspace_bytes(_desc(mm, det_group=4, scatter=mm.MM_SCATTER_ATOMIC))
    b = mm.mm_scan_workspace_bytes(_desc(mm, det_group=4, scatter=mm.MM_SCATTER_ATOMIC,
                                         tod_dtype=mm.MM_BF16))
    assert a - b == 4 * (1 << 15) * 4


def test_compensated_accumulation_takes_the_gather_on_one_kernel_plans(mm):
    # nsamp = 2^12 is a one-kernel plan: the gather index (4 B/sample of runs,
    # 4 B of pixel-major and 4 B of time-major angles) and a pass buffer
    # (4 B/sample) appear only under MM_ACC_F32X2
    a = mm.mm_scan_workspace_bytes(_desc(mm, nsamp=1 << 12))
    b = mm.mm_scan_workspace_bytes(_desc(mm, nsamp=1 << 12, acc=mm.MM_ACC_F32X2))
    S = 4 * (1 << 12)
    assert 16 * S <= b - a <= 16 * S + 3 * 4 * (64 * 64 + 1) + 6 * 256


@pytest.mark.parametrize("field,value", [
    ("ncomp", 2), ("ny", 48), ("nx", 2), ("ndet", 0), ("nsamp", 1022), ("nsamp", 1001), ("nsamp", 8),
    ("nsamp", 2 * 3**9 * 2**4), ("nsamp", 7 * 2**8),
    ("nsamp", 1 << 23), ("tod_dtype", 7), ("fft_m1", 3), ("det_group", -1), ("scatter", 5),
    ("scatter", 3),
    ("acc", 2), ("pointing_code", 2), ("pointing_code", -1),
])
def test_invalid_descriptions_rejected(mm, field, value):
    d = _desc(mm, **{field: value})
    assert mm.mm_scan_workspace_bytes(d) == 0
    assert mm.mm_last_error()
    h = C.c_void_p()
    st = mm.lib.mm_create_scan(C.byref(d), None, C.byref(h))
    assert st == mm.MM_EINVAL and not h.value


def test_correlated_noise_descriptions(mm):
    import numpy as np
    n = 1 << 16
    edges = np.array([0, 10, 100, n // 2 + 1], np.int32)
    ok = _desc(mm, corr_rank=2, corr_nbins=3, corr_edges=edges.ctypes.data)
    assert mm.mm_scan_workspace_bytes(ok) > 0
    bad = [dict(corr_rank=17, corr_nbins=3, corr_edges=edges.ctypes.data),
           dict(corr_rank=2, corr_nbins=0, corr_edges=edges.ctypes.data),
           dict(corr_rank=2, corr_nbins=3, corr_edges=None)]
    short = np.array([0, 10, 100, n // 2], np.int32)          # does not reach n/2 + 1
    flat = np.array([0, 10, 10, n // 2 + 1], np.int32)       # not increasing
    bad += [dict(corr_rank=2, corr_nbins=3, corr_edges=short.ctypes.data),
            dict(corr_rank=2, corr_nbins=3, corr_edges=flat.ctypes.data)]
    tiny = np.array([0, 10, (1 << 12) // 2 + 1], np.int32)    # nsamp below 2^13
    bad += [dict(corr_rank=2, corr_nbins=2, corr_edges=tiny.ctypes.data, nsamp=1 << 12)]
    for kw in bad:
        assert mm.mm_scan_workspace_bytes(_desc(mm, **kw)) == 0, kw
        assert mm.mm_last_error()


def test_compensated_accumulation_needs_the_gather(mm):
    d = _desc(mm, acc=mm.MM_ACC_F32X2, scatter=mm.MM_SCATTER_ATOMIC)
    assert mm.mm_scan_workspace_bytes(d) == 0
    assert "MM_ACC_F32X2" in mm.mm_last_error()


def test_create_requires_pointers_and_workspace(mm):
    h = C.c_void_p()
    assert mm.lib.mm_create_scan(None, None, C.byref(h)) == mm.MM_EINVAL
    d = _desc(mm)
    assert mm.lib.mm_create_scan(C.byref(d), None, C.byref(h)) == mm.MM_EINVAL
    assert "inv_noise" in mm.mm_last_error()
    d.inv_noise = 0x2000
    assert mm.lib.mm_create_scan(C.byref(d), None, C.byref(h)) == mm.MM_EINVAL
    assert "pix" in mm.mm_last_error()
    d.pix, d.inv_noise, d.cos2psi, d.sin2psi = 0x1000, 0x2000, 0x3000, 0x4000
    assert mm.lib.mm_create_scan(C.byref(d), None, C.byref(h)) == mm.MM_EINVAL
    assert "workspace" in mm.mm_last_error()
    d.workspace = 0x100010  # misaligned
    d.workspace_bytes = 1 << 40
    assert mm.lib.mm_create_scan(C.byref(d), None, C.byref(h)) == mm.MM_EINVAL
    d.workspace = 0x100000
    d.workspace_bytes = 16
    assert mm.lib.mm_create_scan(C.byref(d), None, C.byref(h)) == mm.MM_ENOMEM
    d1 = _desc(mm, ncomp=1)
    d1.pix, d1.inv_noise, d1.cos2psi = 0x1000, 0x2000, 0x3000
    assert mm.lib.mm_create_scan(C.byref(d1), None, C.byref(h)) == mm.MM_EINVAL


def test_calls_on_invalid_handle(mm):
    bogus = C.c_void_p(0)
    assert mm.lib.mm_apply_A(bogus, None, None, None) == mm.MM_EINVAL
    assert mm.lib.mm_rhs(bogus, None, None, None) == mm.MM_EINVAL
    assert mm.lib.mm_build_precon(bogus, 3, None, None) == mm.MM_EINVAL
    assert mm.lib.mm_apply_precon_circulant(bogus, None, None, None) == mm.MM_EINVAL
    assert mm.lib.mm_pcg_solve(bogus, 2, None, None, None, None, None) == mm.MM_EINVAL
    info = mm.mm_scan_info()
    assert mm.lib.mm_get_info(bogus, C.byref(info)) == mm.MM_EINVAL
    mm.lib.mm_destroy_scan(bogus)  # no-op


def test_last_error_is_thread_local(mm):
    import threading
    mm.lib.mm_apply_A(C.c_void_p(0), None, None, None)
    mine = mm.mm_last_error()
    other = []
    t = threading.Thread(target=lambda: other.append(mm.lib.mm_last_error()))
    t.start()
    t.join()
    assert mine and other == [b""]


def test_boresight_pointing_descriptor(mm):
    """Validation of the boresight pointing mode (no device work: every
    rejection happens before the first HIP call)."""
    h = C.c_void_p()
    # boresight pointing keeps the per-sample index: compare with stored
    # pointing on the per-sample index too
    d = _desc(mm, nsamp=2**16, scatter=mm.MM_SCATTER_SAMPLES, pointing_code=mm.MM_PTC_OFF)
    stored = mm.mm_scan_workspace_bytes(d)
    d.pointing = 2
    assert mm.mm_scan_workspace_bytes(d) == 0 and "pointing" in mm.mm_last_error()
    d.pointing = mm.MM_POINT_BORESIGHT
    # float32 weights kept beside the index; no time-major angles (pass 1
    # computes the weights from the model) but 20 B per time sample of
    # float32 boresight copies and 12 B per detector
    diff = mm.mm_scan_workspace_bytes(d) - stored
    assert 0 <= diff - (20 * d.nsamp + 12 * d.ndet - 4 * d.ndet * d.nsamp) <= 5 * 256
    d.tod_dtype = mm.MM_F64
    d.pointing = mm.MM_POINT_STORED
    stored = mm.mm_scan_workspace_bytes(d)
    d.pointing = mm.MM_POINT_BORESIGHT
    otf = mm.mm_scan_workspace_bytes(d)
    # float64 path: the index holds no weights, 8 B per sample less
    assert stored - otf >= 8 * d.ndet * d.nsamp - 4096
    d.tod_dtype = mm.MM_F32
    d.scatter = mm.MM_SCATTER_ATOMIC
    assert mm.mm_scan_workspace_bytes(d) == 0 and "SCATTER_AUTO" in mm.mm_last_error()
    d.scatter = mm.MM_SCATTER_AUTO
    d.inv_noise = 0x2000
    d.pix = 0x1000
    assert mm.lib.mm_create_scan(C.byref(d), None, C.byref(h)) == mm.MM_EINVAL
    assert "must be NULL" in mm.mm_last_error()
    d.pix = None
    assert mm.lib.mm_create_scan(C.byref(d), None, C.byref(h)) == mm.MM_EINVAL
    assert "required" in mm.mm_last_error()
    d.bore, d.det_off = 0x10008, 0x20000
    assert mm.lib.mm_create_scan(C.byref(d), None, C.byref(h)) == mm.MM_EINVAL
    assert "aligned" in mm.mm_last_error()
    d.bore = 0x10000
    assert mm.lib.mm_create_scan(C.byref(d), None, C.byref(h)) == mm.MM_EINVAL
    assert "workspace" in mm.mm_last_error()


def test_mixed_radix_lengths(mm):
    """n = 2^a 3^b 5^c: n/2 <= 8192 plans the one-kernel filter; longer ones
    the four-step with rows of 2^l (32..4096) and every factor 3 and 5 in the
    columns (at most 8192 long); correlated noise and boresight pointing
    need a power of two."""
    for n in (30, 1000, 3 * 2**11, 15 * 2**9, 2 * 3**8, 2 * 5**5, 2**4 * 3 * 5**3,
              3 * 2**14, 3 * 2**20, 15 * 2**18, 2 * 3**5 * 2**12, 2 * 5**4 * 2**10):
        d = _desc(mm, nsamp=n)
        assert mm.mm_scan_workspace_bytes(d) > 0, n
    for n in (2 * 3**9 * 2**4, 2 * 5**6 * 2**6):   # no four-step split
        d = _desc(mm, nsamp=n)
        assert mm.mm_scan_workspace_bytes(d) == 0 and "split" in mm.mm_last_error()
    d = _desc(mm, nsamp=1000, pointing=mm.MM_POINT_BORESIGHT)
    assert mm.mm_scan_workspace_bytes(d) == 0 and "power of two" in mm.mm_last_error()
    import numpy as np
    edges = np.array([0, 100, 501], np.int32)
    d = _desc(mm, nsamp=1000, corr_rank=1, corr_nbins=2, corr_edges=edges.ctypes.data)
    assert mm.mm_scan_workspace_bytes(d) == 0 and "power of two" in mm.mm_last_error()


STRUCTS = ["mm_scan_desc", "mm_precon_opts", "mm_pcg_opts", "mm_pcg_result", "mm_scan_info",
           "mm_train_opts", "mm_profile"]


def test_struct_layouts_match_the_header(mm, tmp_path):
    """Every struct the binding declares has the header's size and field
    offsets (compiled with the system C compiler from include/mm.h)."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mm.h"', "int main(void) {"]
    for s in STRUCTS:
        cls = getattr(mm, s)
        lines.append(f'printf("{s} size %zu\\n", sizeof({s}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{s} {f} %zu\\n", offsetof({s}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            s, f, v = ln.split()
            got[(s, f)] = int(v)
    for s in STRUCTS:
        cls = getattr(mm, s)
        assert C.sizeof(cls) == got[(s, "size")], s
        for f, _ in cls._fields_:
            assert getattr(cls, f).offset == got[(s, f)], (s, f)
