"""C-ABI checks that need no GPU: the library loads, exports every symbol the
public header declares, and rejects bad arguments before any device work."""
import ctypes
import os
import re

import pytest

import paper_1709_07175_amd as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in os.listdir(os.path.join(ROOT, "include"))
           if h.endswith(".h")]


def _declared():
    names = []
    for h in HEADERS:
        txt = open(h).read()
        names += re.findall(r"^LSPCA_API\s+[\w\s\*]*?\b(\w+)\s*\(", txt, flags=re.M)
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_1709_07175_amd import build
        build.build()
    return L.load()


def test_every_declared_symbol_is_exported(lib):
    declared = _declared()
    assert len(declared) >= 10
    raw = ctypes.CDLL(L.LIB_PATH)
    missing = [n for n in declared if not hasattr(raw, n)]
    assert not missing, missing
    assert sorted(set(declared)) == sorted(set(L.EXPORTS))


def test_version_and_strerror(lib):
    assert L.version().startswith("lspca")
    for code, name in L.STATUS.items():
        assert lib.lspca_strerror(code)
    assert lib.lspca_strerror(12345) == b"unknown status"


def _fit_args(**over):
    a = dict(X=1 << 20, dt=L.F32, m=100, n=50, ldx=50, k=5, kind=L.GAUSSIAN, seed=1,
             opts=None, V=1 << 21, s=1 << 22, sx=None)
    a.update(over)
    return a


@pytest.mark.parametrize("over,needle", [
    (dict(X=None), "X is NULL"),
    (dict(k=0), "k must"),
    (dict(k=51), "k must"),
    (dict(m=0), "m and n"),
    (dict(ldx=49), "ldx"),
    (dict(kind=7), "omega kind"),
    (dict(dt=9), "dtype"),
    (dict(V=None), "must not be NULL"),
])
def test_fit_rejects_bad_arguments_before_device_work(lib, over, needle):
    a = _fit_args(**over)
    st = lib.lspca_fit(a["X"], a["dt"], a["m"], a["n"], a["ldx"], a["k"], a["kind"], a["seed"],
                       a["opts"], a["V"], a["s"], a["sx"])
    assert st == -1
    assert needle in lib.lspca_last_error().decode()


def test_k_above_m_is_rejected(lib):
    # Corollary 1 needs l <= min{m, n}
    st = lib.lspca_fit(1 << 20, L.F32, 4, 50, 50, 5, L.GAUSSIAN, 1, None, 1 << 21, 1 << 22, None)
    assert st == -1 and "min(m, n)" in lib.lspca_last_error().decode()


def test_sparse_p_must_be_power_of_two(lib):
    o = L.lspca_opts()
    o.struct_size = ctypes.sizeof(o)
    o.sparse_p = 48
    st = lib.lspca_fit(1 << 20, L.F32, 100, 50, 50, 5, L.VERY_SPARSE, 1, ctypes.byref(o),
                       1 << 21, 1 << 22, None)
    assert st == -1 and "power of two" in lib.lspca_last_error().decode()
    st = lib.lspca_omega(10, 4, L.VERY_SPARSE, 1, 3, L.F32, 1 << 20, None)
    assert st == -1


def test_small_route_and_stripe_rows_are_checked(lib):
    o = L.lspca_opts()
    o.struct_size = ctypes.sizeof(o)
    o.small_route = 2
    st = lib.lspca_fit(1 << 20, L.F32, 100, 50, 50, 5, L.GAUSSIAN, 1, ctypes.byref(o), 1 << 21, 1 << 22, None)
    assert st == -1 and "small_route" in lib.lspca_last_error().decode()
    o.small_route = 1
    o.stripe_rows = -5
    st = lib.lspca_fit(1 << 20, L.F32, 100, 50, 50, 5, L.GAUSSIAN, 1, ctypes.byref(o), 1 << 21, 1 << 22, None)
    assert st == -1 and "stripe_rows" in lib.lspca_last_error().decode()


def test_factor_and_transform_argument_checks(lib):
    assert lib.lspca_factor(None, None, 3, 10, None, 1, 1, None) == -1
    assert lib.lspca_factor(1 << 20, None, 3, 10, None, 1 << 21, 1 << 22, 1 << 23) == -1  # sigma_x needs G
    assert lib.lspca_factor(1 << 20, None, 11, 10, None, 1 << 21, 1 << 22, None) == -1    # k > n
    assert lib.lspca_transform(1 << 20, L.F32, 5, 10, 9, 1 << 21, 3, 1 << 22, None) == -1  # ldx < n
    assert lib.lspca_transform(None, L.F32, 0, 10, 10, None, 3, None, None) == 0          # r = 0: no work
    assert lib.lspca_accumulate(1 << 20, L.F32, 10, 10, 10, 3, L.GAUSSIAN, 1, None, None, None) == -1


def test_small_opts_struct_is_accepted(lib):
    # a caller built against an older, shorter lspca_opts: only the size is read
    class Old(ctypes.Structure):
        _fields_ = [("struct_size", ctypes.c_uint32), ("sparse_p", ctypes.c_uint32)]
    o = Old(8, 3)
    po = ctypes.cast(ctypes.pointer(o), ctypes.POINTER(L.lspca_opts))
    st = lib.lspca_fit(1 << 20, L.F32, 100, 50, 50, 5, L.VERY_SPARSE, 1, po,
                       1 << 21, 1 << 22, None)
    assert st == -1 and "power of two" in lib.lspca_last_error().decode()


def test_server_argument_checks(lib):
    h = ctypes.c_void_p()
    assert lib.lspca_server_create(None, 64, 8, L.BF16, 0, 4, ctypes.byref(h)) == -1   # V NULL
    assert lib.lspca_server_create(1 << 20, 0, 8, L.BF16, 0, 4, ctypes.byref(h)) == -1  # n < 1
    assert lib.lspca_server_create(1 << 20, 64, 8, 7, 0, 4, ctypes.byref(h)) == -1      # dtype
    assert lib.lspca_server_create(1 << 20, 64, 8, L.BF16, 0, 0, ctypes.byref(h)) == -1  # max_inflight
    assert "max_inflight" in lib.lspca_last_error().decode()
    t = ctypes.c_uint64()
    assert lib.lspca_server_submit(None, 1 << 20, 4, 1 << 21, ctypes.byref(t)) == -1
    assert lib.lspca_server_wait(None, 1, 0, None) == -1
    assert lib.lspca_server_pause(None, 1) == -1
    st = L.lspca_server_stats()
    st.struct_size = ctypes.sizeof(st)
    assert lib.lspca_server_get_stats(None, ctypes.byref(st)) == -1
    assert lib.lspca_server_destroy(None) == 0


def test_host_stream_argument_checks(lib):
    # NULL X, NULL F, negative stripe: refused before any device work
    assert lib.lspca_accumulate_host(None, L.F32, 10, 10, 10, 3, L.GAUSSIAN, 1, None, 0, 1 << 20, None) == -1
    assert lib.lspca_accumulate_host(1 << 20, L.F32, 10, 10, 10, 3, L.GAUSSIAN, 1, None, 0, None, None) == -1
    assert lib.lspca_accumulate_host(1 << 20, L.F32, 10, 10, 10, 3, L.GAUSSIAN, 1, None, -5, 1 << 21, None) == -1
    assert "stripe_rows" in lib.lspca_last_error().decode()
    assert lib.lspca_fit_host(1 << 20, L.F32, 10, 10, 10, 11, L.GAUSSIAN, 1, None, 0, 1 << 21, 1 << 22, None) == -1


def test_spca_fit_stream_argument_checks(lib):
    assert lib.spca_fit_stream(None, L.F32, 100, 50, 50, 5, L.GAUSSIAN, 1, None, 1 << 20, 1 << 21) == -1
    assert lib.spca_fit_stream(1 << 20, L.F32, 4, 50, 50, 5, L.GAUSSIAN, 1, None, 1 << 21, 1 << 22) == -1  # k > m
    assert lib.spca_fit_stream(1 << 20, L.F32, 100, 50, 50, 5, L.GAUSSIAN, 1, None, None, 1 << 22) == -1


def test_csr_argument_checks(lib):
    # refused before any device work: NULL arrays, unsupported value type,
    # bad sizes, k above min(m, n)
    P, F, G = 1 << 20, 1 << 21, 1 << 22
    acc = lib.lspca_accumulate_csr
    assert acc(None, P, P, L.F32, 10, 10, 5, 3, L.GAUSSIAN, 1, None, F, None) == -1
    assert "rowptr" in lib.lspca_last_error().decode()
    assert acc(P, None, P, L.F32, 10, 10, 5, 3, L.GAUSSIAN, 1, None, F, None) == -1
    assert acc(P, P, P, L.BF16, 10, 10, 5, 3, L.GAUSSIAN, 1, None, F, None) == -7
    assert acc(P, P, P, 9, 10, 10, 5, 3, L.GAUSSIAN, 1, None, F, None) == -1
    assert acc(P, P, P, L.F32, 0, 10, 5, 3, L.GAUSSIAN, 1, None, F, None) == -1
    assert acc(P, P, P, L.F32, 10, 10, -1, 3, L.GAUSSIAN, 1, None, F, None) == -1
    assert acc(P, P, P, L.F32, 10, 10, 5, 11, L.GAUSSIAN, 1, None, F, None) == -1
    assert acc(P, P, P, L.F32, 10, 10, 5, 3, 7, 1, None, F, None) == -1
    assert acc(P, P, P, L.F32, 10, 10, 5, 3, L.GAUSSIAN, 1, None, None, G) == -1
    fit = lib.lspca_fit_csr
    assert fit(P, P, P, L.F64, 4, 10, 5, 5, L.GAUSSIAN, 1, None, F, G, None) == -1      # k > m
    assert "min(m, n)" in lib.lspca_last_error().decode()
    assert fit(P, P, P, L.F64, 10, 10, 5, 3, L.GAUSSIAN, 1, None, None, G, None) == -1
    sp = lib.spca_fit_csr
    assert sp(P, P, P, L.F32, 1000, 1000, 5, 257, L.GAUSSIAN, 1, None, F, G) == -7           # QR block height
    assert sp(P, P, P, L.F64, 1000, 1000, 5, 129, L.GAUSSIAN, 1, None, F, G) == -7
    assert sp(P, P, P, L.F32, 10, 100, 5, 11, L.GAUSSIAN, 1, None, F, G) == -1              # k > m
    assert sp(P, P, P, L.F32, 100, 100, 5, 10, L.GAUSSIAN, 1, None, None, G) == -1
    tr = lib.lspca_transform_csr
    assert tr(None, None, None, L.F32, 0, 10, 0, None, 3, None, None) == 0               # r = 0: no work
    assert tr(P, P, P, L.F32, 5, 10, 5, None, 3, F, None) == -1                          # V NULL
    assert tr(P, P, P, L.F32, -1, 10, 5, F, 3, G, None) == -1


def test_transform_noalloc_argument_checks(lib):
    tr = lib.lspca_transform_noalloc
    assert tr(1 << 20, L.F32, 5, 10, 9, 1 << 21, 3, 1 << 22, None) == -1    # ldx < n
    assert tr(None, L.F32, 0, 10, 10, None, 3, None, None) == 0             # r = 0: no work
    assert tr(None, L.F32, 5, 10, 10, 1 << 21, 3, 1 << 22, None) == -1      # X NULL
    assert tr(1 << 20, 9, 5, 10, 10, 1 << 21, 3, 1 << 22, None) == -1       # dtype
    # V^T beyond the fixed scratch: refused before any device work
    cap = L.NOALLOC_SCRATCH_BYTES
    for dt, es, parts in ((L.F64, 8, 1), (L.F32, 4, 1), (L.BF16, 2, 2), (L.F16, 2, 2)):
        nk = cap // (es * parts)
        assert tr(1 << 20, dt, 5, nk // 256 + 1, nk // 256 + 1, 1 << 21, 256, 1 << 22, None) == -5
        assert "scratch" in lib.lspca_last_error().decode()
    assert tr(1 << 20, L.F32, 5, 1 << 40, 1 << 40, 1 << 21, 1 << 30, 1 << 22, None) == -5  # no overflow
