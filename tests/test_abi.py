"""C-ABI checks that need no GPU: the library loads, exports every function
include/maxtimes.h declares, and rejects bad arguments synchronously (before
anything touches the device).  No compute call is made here."""

import ctypes
import os
import re

import pytest

import paper_1511_05690_amd as mt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "maxtimes.h")

pytestmark = pytest.mark.skipif(not os.path.exists(mt.library_path()),
                                reason="libmaxtimes.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "defined")))


def test_every_declared_symbol_is_exported():
    lib = mt.load_library()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings_and_version():
    lib = mt.load_library()
    for code in range(6):
        assert lib.maxtimes_status_string(code)
    assert lib.maxtimes_version().startswith(b"maxtimes")


def _ws(P, path="bf16", b=1, m=64, k=64, n=64, **kw):
    return mt.workspace_size(b, m, k, n, P, path=path, **kw)


def test_workspace_sizes_scale_with_family_and_path():
    small = _ws([1, 2])
    big = _ws(mt.pfamily(128))
    assert 0 < small < big
    # BF16: 11 planes of 256x64 (padded) per operand for {1..128} with split p <= 4
    planes = 11 * 256 * 64 * 2
    assert big >= 2 * planes
    f64 = _ws(mt.pfamily(128), path="fp64")
    assert f64 > 0
    assert mt.apsp_workspace_size(100, mt.pfamily(64), path="fp64") > 0


@pytest.mark.parametrize("P,err", [([], 1), ([2, 1], 1), ([0, 1], 1), ([1, 5000], 1),
                                   ([1, 1], 1), (list(range(1, 40)), 1)])
def test_bad_family_rejected(P, err):
    with pytest.raises(mt.MaxTimesError) as e:
        _ws(P)
    assert e.value.status == err


def test_bad_path_flags_and_sizes_rejected():
    with pytest.raises(mt.MaxTimesError) as e:
        _ws([1, 2], path=7)
    assert e.value.status == 1
    with pytest.raises(mt.MaxTimesError) as e:
        _ws([1, 2], flags=64)
    assert e.value.status == 1
    with pytest.raises(mt.MaxTimesError) as e:
        _ws([1, 2], m=-1)
    assert e.value.status == 1
    with pytest.raises(mt.MaxTimesError) as e:
        _ws([1, 2], n=1 << 25)
    assert e.value.status == 5


def _opts(P, path=1, flags=0):
    return mt._options(P, path, None, None, flags)


def test_null_pointers_and_small_workspace_rejected_before_launch():
    lib = mt.load_library()
    o = _opts([1, 2, 4])
    fake = ctypes.c_void_p(0x100000)  # never dereferenced: every call fails validation first
    null = ctypes.c_void_p(0)
    st = lib.maxtimes_estimate(fake, fake, 0, 1, 8, 8, 8, None, fake, null, fake, 1 << 30, null)
    assert st == 1
    st = lib.maxtimes_estimate(fake, fake, 0, 1, 8, 8, 8, ctypes.byref(o), null, null, fake, 1 << 30, null)
    assert st == 1 and b"C is NULL" in lib.maxtimes_last_error()
    st = lib.maxtimes_estimate(null, fake, 0, 1, 8, 8, 8, ctypes.byref(o), fake, null, fake, 1 << 30, null)
    assert st == 1
    st = lib.maxtimes_estimate(fake, fake, 9, 1, 8, 8, 8, ctypes.byref(o), fake, null, fake, 1 << 30, null)
    assert st == 1
    st = lib.maxtimes_estimate(fake, fake, 0, 1, 8, 8, 8, ctypes.byref(o), fake, null, fake, 16, null)
    assert st == 3 and b"workspace" in lib.maxtimes_last_error()
    st = lib.maxtimes_estimate(fake, fake, 0, 1, 8, 8, 8, ctypes.byref(o), fake, null, null, 1 << 30, null)
    assert st == 1
    misaligned = ctypes.c_void_p(0x100004)
    st = lib.maxtimes_estimate(fake, fake, 0, 1, 8, 8, 8, ctypes.byref(o), fake, null, misaligned, 1 << 30, null)
    assert st == 1
    # empty output: nothing to do, nothing touched
    st = lib.maxtimes_estimate(null, null, 0, 1, 0, 8, 8, ctypes.byref(o), null, null, null, 0, null)
    assert st == 0
    # raw output is an APSP-only flag
    o2 = _opts([1, 2], flags=8)
    st = lib.maxtimes_estimate(fake, fake, 0, 1, 8, 8, 8, ctypes.byref(o2), fake, null, fake, 1 << 30, null)
    assert st == 1


def test_noalloc_rejects_before_launch():
    """maxtimes_estimate_noalloc checks its arguments, and that the product's
    workspace fits the static scratch, before any device call."""
    lib = mt.load_library()
    o = _opts([1, 2, 4, 8, 16, 32, 64, 128])
    fake = ctypes.c_void_p(0x100000)
    null = ctypes.c_void_p(0)
    st = lib.maxtimes_estimate_noalloc(fake, fake, 0, 1, 8, 8, 8, ctypes.byref(o), null, null, null)
    assert st == 1 and b"C is NULL" in lib.maxtimes_last_error()
    st = lib.maxtimes_estimate_noalloc(fake, fake, 0, 1, 4096, 4096, 4096, ctypes.byref(o), fake, null, null)
    assert st == 3 and b"static scratch" in lib.maxtimes_last_error()
    need = mt.workspace_size(1, 4096, 4096, 4096, [1, 2, 4, 8, 16, 32, 64, 128])
    assert need > mt.NOALLOC_SCRATCH_BYTES
    st = lib.maxtimes_estimate_noalloc(null, null, 0, 1, 0, 8, 8, ctypes.byref(o), null, null, null)
    assert st == 0


def test_balance_flag_workspace_and_scope():
    """MT_FLAG_BALANCE adds 4 b k FP64 values (column maxima of A, row maxima
    of B, d, 1 / d) to the product workspace and is refused by APSP."""
    lib = mt.load_library()
    P = [1, 2, 4, 8]
    w0 = mt.workspace_size(3, 100, 777, 90, P)
    w1 = mt.workspace_size(3, 100, 777, 90, P, flags=mt.FLAG_BALANCE)
    assert w1 - w0 == 4 * ((3 * 777 * 8 + 255) // 256 * 256)
    o = _opts(P, flags=mt.FLAG_BALANCE)
    out = ctypes.c_size_t(0)
    assert lib.apsp_workspace_size(64, ctypes.byref(o), ctypes.byref(out)) == 1
    assert b"MT_FLAG_BALANCE" in lib.maxtimes_last_error()


def test_apsp_argument_errors():
    lib = mt.load_library()
    o = _opts([1, 2, 4], path=0)
    fake = ctypes.c_void_p(0x100000)
    null = ctypes.c_void_p(0)
    assert lib.apsp_estimate(fake, 8, 0.0, -1, ctypes.byref(o), fake, 0, null, fake, 1 << 30, null) == 1
    assert lib.apsp_estimate(fake, 8, float("inf"), -1, ctypes.byref(o), fake, 0, null, fake, 1 << 30, null) == 1
    assert lib.apsp_estimate(null, 8, 1.0, -1, ctypes.byref(o), fake, 0, null, fake, 1 << 30, null) == 1
    assert lib.apsp_estimate(fake, 8, 1.0, -1, ctypes.byref(o), fake, 0, null, fake, 8, null) == 3
    assert lib.apsp_estimate(fake, 8, 1.0, 100, ctypes.byref(o), fake, 0, null, fake, 1 << 30, null) == 1
    o2 = _opts([1, 2], path=0, flags=2)
    assert lib.apsp_estimate(fake, 8, 1.0, -1, ctypes.byref(o2), fake, 0, null, fake, 1 << 30, null) == 5
    assert lib.apsp_estimate(null, 0, 1.0, -1, ctypes.byref(o), null, 0, null, null, 0, null) == 0


def test_timing_read_without_launches():
    mt.timing_reset()
    assert mt.timing_read("mt_") == (0.0, 0)


def test_projection_flag_validation():
    """MT_FLAG_PROJECT_R1: not with the norm correction; the FP64 path needs
    one more FP64 buffer of the output's size; the backward rejects it."""
    R1 = mt.FLAG_PROJECT_R1
    with pytest.raises(mt.MaxTimesError) as e:
        _ws([1, 2], flags=R1 | mt.FLAG_NORM_CORRECT)
    assert e.value.status == 1
    m = n = 64
    plain = _ws([1, 2, 4], path="fp64", m=m, n=n)
    r1 = _ws([1, 2, 4], path="fp64", m=m, n=n, flags=R1)
    assert r1 - plain == m * n * 8
    assert _ws([1, 2, 4], path="bf16", flags=R1) == _ws([1, 2, 4], path="bf16")
    lib = mt.load_library()
    fake = ctypes.c_void_p(0x100000)
    null = ctypes.c_void_p(0)
    o = _opts([1, 2, 4], flags=R1)
    st = lib.maxtimes_estimate_backward(fake, fake, fake, fake, fake, 0, 1, 8, 8, 8, ctypes.byref(o),
                                        fake, fake, fake, 1 << 30, null)
    assert st == 5 and b"projection" in lib.maxtimes_last_error()
    with pytest.raises(ValueError):
        mt._projection_flag("r3")


def test_search_start_validation():
    """The forward search start is a plan index in 0 .. MT_MAX_P - 1, or -1
    (the default: a pilot chooses)."""
    assert mt.search_start() == -1
    old = mt.search_start()
    try:
        for bad in (-2, mt.MAX_P):
            with pytest.raises(mt.MaxTimesError) as e:
                mt.set_search_start(bad)
            assert e.value.status == 1
        mt.set_search_start(3)
        assert mt.search_start() == 3
    finally:
        mt.set_search_start(old)


def test_small_product_limit_validation():
    """Products with b m k n up to the limit (default 2^25) take the
    one-kernel FP64 path; 0 turns it off, a negative limit is rejected."""
    assert mt.small_product_limit() == 1 << 25
    old = mt.small_product_limit()
    try:
        with pytest.raises(mt.MaxTimesError) as e:
            mt.set_small_product_limit(-1)
        assert e.value.status == 1
        mt.set_small_product_limit(0)
        assert mt.small_product_limit() == 0
        mt.set_small_product_limit(1 << 40)
        assert mt.small_product_limit() == 1 << 40
    finally:
        mt.set_small_product_limit(old)


def test_bf16_inner_dimension_limit():
    """The BF16 path contracts at most 2^23 terms per entry; the FP64 path
    keeps the general 2^24 limit."""
    assert _ws([1, 2], path="bf16", k=1 << 23) > 0
    with pytest.raises(mt.MaxTimesError) as e:
        _ws([1, 2], path="bf16", k=(1 << 23) + 1)
    assert e.value.status == 5
    assert _ws([1, 2], path="fp64", k=(1 << 23) + 1) > 0


def test_affine_and_exact_rows_validation():
    """Argument checks of the exact-rows and affine entry points (no GPU)."""
    lib = mt.load_library()
    nb = ctypes.c_size_t(0)
    assert lib.apsp_exact_rows_workspace_size(100, 4, ctypes.byref(nb)) == 0
    assert nb.value >= 100 * 4 * 8
    assert lib.apsp_exact_rows_workspace_size(-1, 4, ctypes.byref(nb)) == 1
    assert lib.apsp_affine_workspace_size(ctypes.byref(nb)) == 0 and nb.value > 0
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(0x100000)
    st = lib.apsp_exact_rows(null, 10, fake, 2, fake, None, fake, 1 << 20, null)
    assert st == 1 and b"NULL" in lib.maxtimes_last_error()
    st = lib.apsp_affine_correct(fake, 7, 10, fake, 2, fake, fake, 1, fake, 1 << 20, null)
    assert st == 1 and b"dtype" in lib.maxtimes_last_error()
    st = lib.apsp_affine_correct(fake, 0, 10, fake, 2, fake, null, 1, fake, 1 << 20, null)
    assert st == 1 and b"ab" in lib.maxtimes_last_error()
    st = lib.apsp_affine_correct(fake, 0, 10, fake, 2, fake, fake, 1, fake, 1, null)
    assert st == 3


def test_r2_flag_validation():
    """MT_FLAG_PROJECT_R2: FP64 path only, not with R1 or the norm
    correction, and the added norms 3p/4 enlarge the FP64 workspace by one
    output-sized stack plane per power (no GPU needed)."""
    R2 = mt.FLAG_PROJECT_R2
    with pytest.raises(mt.MaxTimesError) as e:
        _ws([1, 2, 4], path="bf16", flags=R2)
    assert e.value.status == 5
    for bad in (R2 | mt.FLAG_PROJECT_R1, R2 | mt.FLAG_NORM_CORRECT):
        with pytest.raises(mt.MaxTimesError) as e:
            _ws([1, 2, 4], path="fp64", flags=bad)
        assert e.value.status == 1
    m = n = 64
    # {1, 2, 4, 8}: added norms 3 and 6 -> 6 stack planes of 64 x 64 doubles
    r2 = _ws([1, 2, 4, 8], path="fp64", m=m, n=n, flags=R2)
    assert r2 >= 6 * m * n * 8
    # 32 powers at most, family and added norms together
    with pytest.raises(mt.MaxTimesError) as e:
        _ws([2 ** i for i in range(13)] + [3 * 2 ** i for i in range(12, 19)], path="fp64", flags=R2)


def test_maxconv_validation():
    """Argument checks of the max-convolution entry points (no GPU): FP64
    path only, no flags, n + m - 1 <= 16384 (a workspace above 4096),
    non-NULL pointers; empty sizes return at once."""
    lib = mt.load_library()
    fake = ctypes.c_void_p(0x100000)
    null = ctypes.c_void_p(0)
    big = ctypes.c_size_t(1 << 40)
    o = _opts([1, 2, 4], path=0)
    nb = ctypes.c_size_t(7)
    assert lib.maxconv_workspace_size(2, 2048, 2049, ctypes.byref(o), ctypes.byref(nb)) == 0 and nb.value == 0
    assert lib.maxconv_workspace_size(2, 2048, 2050, ctypes.byref(o), ctypes.byref(nb)) == 0
    assert nb.value >= 2 * 2 * 8192 * 16
    assert lib.maxconv_workspace_size(2, 8192, 8193, ctypes.byref(o), ctypes.byref(nb)) == 0
    assert lib.maxconv_workspace_size(2, 8192, 8194, ctypes.byref(o), ctypes.byref(nb)) == 5
    st = lib.maxconv_estimate(fake, fake, 0, 2, 2048, 2049, ctypes.byref(o), null, null, null, 0, null)
    assert st == 1 and b"NULL" in lib.maxtimes_last_error()
    st = lib.maxconv_estimate(fake, fake, 0, 2, 8192, 8194, ctypes.byref(o), fake, null, fake, big, null)
    assert st == 5 and b"16384" in lib.maxtimes_last_error()
    # a long pair needs its workspace
    st = lib.maxconv_estimate(fake, fake, 0, 2, 2048, 2050, ctypes.byref(o), fake, null, fake, 16, null)
    assert st == 3
    st = lib.maxconv_estimate(fake, fake, 0, 2, 8, 8, ctypes.byref(_opts([1, 2], path=1)), fake, null, null, 0, null)
    assert st == 5
    st = lib.maxconv_estimate(fake, fake, 0, 2, 8, 8, ctypes.byref(_opts([1, 2], path=0, flags=4)), fake, null, null,
                              0, null)
    assert st == 5
    assert lib.maxconv_estimate(fake, fake, 3, 2, 8, 8, ctypes.byref(o), fake, null, null, 0, null) == 1
    assert lib.maxconv_estimate(fake, fake, 0, -1, 8, 8, ctypes.byref(o), fake, null, null, 0, null) == 1
    assert lib.maxconv_estimate(fake, fake, 0, 1 << 31, 8, 8, ctypes.byref(o), fake, null, null, 0, null) == 5
    assert lib.maxconv_estimate(fake, fake, 0, 2, 8, 8, None, fake, null, null, 0, null) == 1
    assert lib.maxconv_estimate(null, null, 0, 0, 8, 8, ctypes.byref(o), null, null, null, 0, null) == 0
    assert lib.maxconv_estimate(null, null, 0, 4, 0, 8, ctypes.byref(o), null, null, null, 0, null) == 0
    assert lib.maxconv_exact(null, fake, 0, 2, 8, 8, fake, null) == 1
    assert lib.maxconv_exact(fake, fake, 0, 2, (1 << 24) + 1, 8, fake, null) == 5
    assert lib.maxconv_exact(null, null, 1, 0, 8, 8, null, null) == 0


def test_xy_topk_validation():
    """Argument checks of the x + y top-k entry points (no GPU): FP64 path
    only, no flag but the paired one (k <= 4096 with it), 2n - 1 <= 16384,
    k >= 0, workspace size, NULL pointers."""
    lib = mt.load_library()
    o = _opts(list(mt.XY_FAMILY), path=0)
    nb = ctypes.c_size_t(0)
    assert lib.xy_topk_workspace_size(1024, 256, ctypes.byref(o), ctypes.byref(nb)) == 0
    assert nb.value >= 2 * 24 * 2047 * 8 + 256 * 16
    assert lib.xy_topk_workspace_size(8193, 4, ctypes.byref(o), ctypes.byref(nb)) == 5
    assert lib.xy_topk_workspace_size(8192, 4, ctypes.byref(o), ctypes.byref(nb)) == 0
    assert lib.xy_topk_workspace_size(0, 4, ctypes.byref(o), ctypes.byref(nb)) == 1
    assert lib.xy_topk_workspace_size(8, -1, ctypes.byref(o), ctypes.byref(nb)) == 1
    assert lib.xy_topk_workspace_size(8, 4, ctypes.byref(_opts([1, 2], path=1)), ctypes.byref(nb)) == 5
    assert lib.xy_topk_workspace_size(8, 4, ctypes.byref(_opts([1, 2], path=0, flags=1)), ctypes.byref(nb)) == 5
    # k <= 4096: room for 2 min(k, 2n - 1) candidates with their columns
    # (plain and paired alike); the paired flag takes k <= 4096 and is for
    # this entry point only
    paired = _opts(list(mt.XY_FAMILY), path=0, flags=mt.FLAG_XY_PAIRED)
    plain_nb = ctypes.c_size_t(0)
    assert lib.xy_topk_workspace_size(1024, 256, ctypes.byref(paired), ctypes.byref(nb)) == 0
    assert lib.xy_topk_workspace_size(1024, 256, ctypes.byref(o), ctypes.byref(plain_nb)) == 0
    assert nb.value == plain_nb.value >= 2 * 24 * 2047 * 8 + 2 * 256 * (12 + 24 * 8)
    assert lib.xy_topk_workspace_size(1024, 5000, ctypes.byref(o), ctypes.byref(plain_nb)) == 0
    assert lib.xy_topk_workspace_size(8192, 4096, ctypes.byref(paired), ctypes.byref(nb)) == 0
    assert lib.xy_topk_workspace_size(8192, 4097, ctypes.byref(paired), ctypes.byref(nb)) == 5
    assert "k <= 4096" in lib.maxtimes_last_error().decode()
    assert lib.maxconv_workspace_size(1, 8, 8, ctypes.byref(paired), ctypes.byref(nb)) == 1
    fake = ctypes.c_void_p(0x100000)
    null = ctypes.c_void_p(0)
    assert lib.xy_topk_estimate(null, fake, 0, 8, 4, ctypes.byref(o), fake, null, null, null, fake, 1 << 30,
                                null) == 1
    assert lib.xy_topk_estimate(fake, fake, 0, 8, 4, ctypes.byref(o), null, null, null, null, fake, 1 << 30,
                                null) == 1
    assert lib.xy_topk_estimate(fake, fake, 0, 8, 4, ctypes.byref(o), fake, null, null, null, fake, 64, null) == 3
    assert lib.xy_topk_estimate(fake, fake, 5, 8, 4, ctypes.byref(o), fake, null, null, null, fake, 1 << 30,
                                null) == 1


def test_workspace_map():
    """The inspection map of the product's workspace (no GPU): ordered,
    inside the workspace, planes of the plane spec."""
    for path, P in (("bf16", [1, 2, 4, 8, 16]), ("fp64", [1, 2, 4, 8])):
        m = mt.workspace_map(2, 100, 70, 50, P, path=path)
        size = _ws(P, path=path, b=2, m=100, k=70, n=50)
        assert m["r"] < m["c"] < m["a_planes"] < m["b_planes"] < size
        esz = m["elem_bytes"]
        assert m["b_planes"] + 2 * m["n_planes"] * m["n_pad"] * m["k_pad"] * esz <= size
        assert m["power"] == P
        assert m["m_pad"] >= 100 and m["n_pad"] >= 50 and m["k_pad"] >= 70
        if path == "bf16":
            assert esz == 2 and m["split"] == [True, True, True, False, False]
            assert m["first_plane"] == [0, 2, 4, 6, 7] and m["n_planes"] == 8
        else:
            assert esz == 8 and m["n_planes"] == 4 and not any(m["split"])
    with pytest.raises(mt.MaxTimesError):
        mt.workspace_map(1, 8, 8, 8, [2, 1])
