"""CPU tests of the C ABI library: it builds for gfx950, loads, exports every
function include/rw.h declares, and its host-side argument validation rejects
bad calls before anything reaches a device (validation-only context, no GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2606_27604_amd import rw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rw.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(rw.LIB_PATH):
        from paper_2606_27604_amd import build
        build.build()
    return rw.load_library()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rw_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("rw_forward", "rw_adjoint", "rw_batch_forward", "rw_batch_adjoint", "rw_finalize",
              "rw_create", "rw_destroy", "rw_check", "rw_debug_trace"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", rw.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (rw_[a-z_0-9]+)$", out, flags=re.M))
    for n in declared_functions():
        assert n in exported, f"{n} declared in rw.h but not exported"
        assert hasattr(lib, n)
    assert set(rw.EXPORTS) <= exported


def test_library_is_built_for_gfx950_only(lib):
    blob = open(rw.LIB_PATH, "rb").read()
    targets = set(re.findall(rb"amdgcn-amd-amdhsa-+(gfx[0-9a-f]+)", blob))
    assert targets == {b"gfx950"}, targets


def test_status_strings_and_version(lib):
    assert lib.rw_status_string(0) == b"RW_OK"
    assert lib.rw_status_string(5) == b"RW_E_DEVICE_FLAG"
    assert lib.rw_version().startswith(b"rwmc-gfx950")


def _args():
    g = rw.Geometry(n_media=3).c()
    m = rw.RwMediaC(0x1000, 0x2000, 0x3000, 0x4000, 0, 1, 81, None, 0)
    t = rw.RwTallyC(0x5000, 0x6000, 0x7000, 0x8000)
    return g, m, t


def test_validation_rejects_bad_arguments_without_a_device(lib):
    ctx = rw.Context(-1)
    g, m, t = _args()
    call = lambda: lib.rw_forward(ctx.h, ctypes.byref(m), ctypes.byref(g), 1024, 0,  # noqa: E731
                                  ctypes.byref(t), None)
    # well-formed call: passes validation, then reports that there is no device
    assert call() == rw.RW_E_UNSUPPORTED
    cases = [
        ("n_bins", 0), ("n_bins", 5000), ("n_media", 0), ("n_rel", 0.0), ("r_min_mm", 0.0),
        ("r_max_mm", 1e-4), ("max_vertices", 0), ("rr_survive", 0.0), ("n_rel", float("nan")),
    ]
    for field, val in cases:
        g2 = rw.Geometry(n_media=3).c()
        setattr(g2, field, val)
        st = lib.rw_forward(ctx.h, ctypes.byref(m), ctypes.byref(g2), 1024, 0, ctypes.byref(t), None)
        assert st == rw.RW_E_INVALID, (field, val, st)
        assert ctx.last_error()
    g5 = rw.Geometry(n_media=5).c()
    assert lib.rw_forward(ctx.h, ctypes.byref(m), ctypes.byref(g5), 1024, 0, ctypes.byref(t),
                          None) == rw.RW_E_UNSUPPORTED
    assert lib.rw_forward(ctx.h, ctypes.byref(m), ctypes.byref(g), -1, 0, ctypes.byref(t),
                          None) == rw.RW_E_INVALID
    assert lib.rw_forward(ctx.h, None, ctypes.byref(g), 16, 0, ctypes.byref(t), None) == rw.RW_E_INVALID
    bad_m = rw.RwMediaC(0, 0x2000, 0x3000, 0x4000, 0, 1, 81, None, 0)
    assert lib.rw_forward(ctx.h, ctypes.byref(bad_m), ctypes.byref(g), 16, 0, ctypes.byref(t),
                          None) == rw.RW_E_INVALID
    bad_t = rw.RwTallyC(0x5000, 0, 0x7000, 0x8000)
    assert lib.rw_forward(ctx.h, ctypes.byref(m), ctypes.byref(g), 16, 0, ctypes.byref(bad_t),
                          None) == rw.RW_E_INVALID
    small_stride = rw.RwMediaC(0x1000, 0x2000, 0x3000, 0x4000, 0, 1, 81, None, 10)
    assert lib.rw_forward(ctx.h, ctypes.byref(small_stride), ctypes.byref(g), 16, 0,
                          ctypes.byref(t), None) == rw.RW_E_INVALID
    assert lib.rw_forward(None, ctypes.byref(m), ctypes.byref(g), 16, 0, ctypes.byref(t),
                          None) == rw.RW_E_INVALID


def test_batch_and_adjoint_validation(lib):
    ctx = rw.Context(-1)
    g, m, t = _args()
    opts = rw.RwBatchOptsC(1, 0, 10, 5)  # window end before begin
    assert lib.rw_batch_forward(ctx.h, ctypes.byref(m), ctypes.byref(g), None, 64, 0,
                                ctypes.byref(t), ctypes.byref(opts), None) == rw.RW_E_INVALID
    opts = rw.RwBatchOptsC(1, 0, 0, 0)
    # a per-unit path array needs the largest count in paths_uniform
    assert lib.rw_batch_forward(ctx.h, ctypes.byref(m), ctypes.byref(g), 0x9000, 0, 0,
                                ctypes.byref(t), ctypes.byref(opts), None) == rw.RW_E_INVALID
    assert lib.rw_batch_forward(ctx.h, ctypes.byref(m), ctypes.byref(g), 0x9000, 128, 0,
                                ctypes.byref(t), ctypes.byref(opts), None) == rw.RW_E_UNSUPPORTED
    # adjoint: grad and flags are required
    assert lib.rw_adjoint(ctx.h, ctypes.byref(m), ctypes.byref(g), 64, 0, None, None, None, None,
                          None, 0x8000, None) == rw.RW_E_INVALID
    assert lib.rw_adjoint(ctx.h, ctypes.byref(m), ctypes.byref(g), 64, 0, None, None, 0x9000,
                          None, None, None, None) == rw.RW_E_INVALID
    ok_opts = rw.RwBatchOptsC(0, 0, 0, 0)
    assert lib.rw_batch_adjoint(ctx.h, ctypes.byref(m), ctypes.byref(g), None, 64, 0, None, None,
                                0x9000, None, None, 0x8000, ctypes.byref(ok_opts),
                                None) == rw.RW_E_UNSUPPORTED
    # trace takes one unit only
    assert lib.rw_debug_trace(ctx.h, ctypes.byref(m), ctypes.byref(g), None, 4, 4, 0, 0, 0x1,
                              0x2, None, None) == rw.RW_E_INVALID


def test_create_without_gpu_fails_cleanly(lib):
    h = ctypes.c_void_p(1234)
    st = lib.rw_create(ctypes.byref(h), 0)
    if st == rw.RW_OK:
        lib.rw_destroy(h)
        pytest.skip("a GPU is present")
    assert st == rw.RW_E_HIP and not h.value
    assert lib.rw_destroy(None) == rw.RW_OK


def test_product_path_has_no_cpu_fallback(tmp_path):
    # the binding raises when the library is missing instead of computing on the CPU
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2606_27604_amd import rw\n"
            "try:\n    rw.load_library(%r)\nexcept ImportError as e:\n    print('raised')\n"
            % (ROOT, str(tmp_path / "missing.so")))
    out = subprocess.run(["python", "-c", code], capture_output=True, text=True)
    assert "raised" in out.stdout
    src = open(os.path.join(ROOT, "paper_2606_27604_amd", "rw.py")).read()
    src += open(os.path.join(ROOT, "paper_2606_27604_amd", "api.py")).read()
    assert "oracle" not in src


def test_noalloc_forward_checks_its_scratch_bound_on_the_host(lib):
    """rw_forward_noalloc rejects a call whose slot sums cannot fit its fixed
    scratch array before anything reaches a device; a call that fits passes the
    check and then reports the missing device."""
    ctx = rw.Context(-1)
    m = rw.RwMediaC(0x1000, 0x2000, 0x3000, 0x4000, 0, 2048, 1, None, 0)
    t = rw.RwTallyC(0x5000, 0x6000, 0x7000, 0x8000)
    g = rw.Geometry(n_media=1, n_bins=4096).c()
    st = lib.rw_forward_noalloc(ctx.h, ctypes.byref(m), ctypes.byref(g), 1 << 17, 0,
                                ctypes.byref(t), None)
    assert st == rw.RW_E_UNSUPPORTED and "scratch" in ctx.last_error()
    g256 = rw.Geometry(n_media=1).c()
    st = lib.rw_forward_noalloc(ctx.h, ctypes.byref(m), ctypes.byref(g256), 1 << 17, 0,
                                ctypes.byref(t), None)
    assert st == rw.RW_E_UNSUPPORTED and "validation-only" in ctx.last_error()
    bad_t = rw.RwTallyC(0x5000, 0, 0x7000, 0x8000)
    assert lib.rw_forward_noalloc(ctx.h, ctypes.byref(m), ctypes.byref(g256), 16, 0,
                                  ctypes.byref(bad_t), None) == rw.RW_E_INVALID


def test_hero_walk_argument_checks(lib):
    """rw_layered_hero_forward rejects unsupported group sizes, unit counts
    that are not a multiple of the group and path counts that are not a
    multiple of it, before anything reaches a device."""
    ctx = rw.Context(-1)
    g = rw.Geometry(n_media=2).c()
    t = rw.RwTallyC(0x5000, 0x6000, 0x7000, 0x8000)
    L = rw.RwLayersC(0x1000, 0x2000, 0x3000, 0x4000, 1.4, 36, 0, 0)
    call = lambda C, n: lib.rw_layered_hero_forward(ctx.h, ctypes.byref(L), ctypes.byref(g), C,  # noqa: E731
                                                    n, 0, ctypes.byref(t), None)
    assert call(5, 1000) == rw.RW_E_UNSUPPORTED
    assert call(8, 800) == rw.RW_E_INVALID        # 36 units are not groups of 8
    assert call(3, 1000) == rw.RW_E_INVALID       # 1000 paths are not a multiple of 3
    assert call(9, 900) == rw.RW_E_UNSUPPORTED and "validation-only" in ctx.last_error()
    g3 = rw.Geometry(n_media=3).c()
    assert lib.rw_layered_hero_forward(ctx.h, ctypes.byref(L), ctypes.byref(g3), 3, 300, 0,
                                       ctypes.byref(t), None) == rw.RW_E_INVALID


def test_dwivedi_walk_argument_checks(lib):
    """rw_dwivedi_forward rejects technique probabilities outside (0, 1],
    cosine incidence and bad path counts before anything reaches a device."""
    ctx = rw.Context(-1)
    g = rw.Geometry(n_media=3).c()
    gc = rw.Geometry(n_media=3, incidence=1).c()
    t = rw.RwTallyC(0x5000, 0x6000, 0x7000, 0x8000)
    m = rw.RwMediaC(0x1000, 0x2000, 0x3000, 0x4000, 0, 1, 4, None, 0)
    call = lambda geo, n, q: lib.rw_dwivedi_forward(ctx.h, ctypes.byref(m), ctypes.byref(geo),  # noqa: E731
                                                    n, 0, q, ctypes.byref(t), None)
    assert call(g, 1000, 0.0) == rw.RW_E_INVALID
    assert call(g, 1000, 1.5) == rw.RW_E_INVALID
    assert call(g, 1000, float("nan")) == rw.RW_E_INVALID
    assert call(gc, 1000, 0.5) == rw.RW_E_UNSUPPORTED
    assert call(g, -1, 0.5) == rw.RW_E_INVALID
    assert call(g, 1000, 1.0) == rw.RW_E_UNSUPPORTED and "validation-only" in ctx.last_error()
