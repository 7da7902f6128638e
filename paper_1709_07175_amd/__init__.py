"""Python binding of liblspca.so (MI355X Lazy SPCA), by ctypes.

The functions here only marshal arguments: device tensors are passed as raw
pointers, the current torch stream as the HIP stream. Every computation runs
in the library's HIP kernels. There is no fallback: if the library is not
built, or no GPU is present, calls raise.

Names mirror the C ABI of include/lspca.h: omega, accumulate, factor, fit,
spca_fit, transform, plus the projection server.
"""
import ctypes
import os

__all__ = [
    "load", "LspcaError", "F64", "F32", "BF16", "F16", "GAUSSIAN", "VERY_SPARSE",
    "version", "omega", "accumulate", "factor", "fit", "spca_fit", "transform",
    "accumulate_host", "fit_host", "spca_fit_stream",
    "last_timings", "exported_symbols", "LIB_PATH", "Server",
]

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblspca.so")

F64, F32, BF16, F16 = 0, 1, 2, 3
GAUSSIAN, VERY_SPARSE = 0, 1
KIND = {"gaussian": GAUSSIAN, "sparse": VERY_SPARSE, GAUSSIAN: GAUSSIAN, VERY_SPARSE: VERY_SPARSE}

STATUS = {0: "LSPCA_OK", -1: "LSPCA_EINVAL", -2: "LSPCA_ENOMEM", -3: "LSPCA_EHIP",
          -4: "LSPCA_ERANK", -5: "LSPCA_E2BIG", -6: "LSPCA_EAGAIN", -7: "LSPCA_ENOTSUP",
          -8: "LSPCA_ETIMEDOUT", -9: "LSPCA_ENOTFOUND", -10: "LSPCA_ENOCONV"}

# Every symbol include/lspca.h declares.
EXPORTS = ["lspca_version", "lspca_strerror", "lspca_last_error", "lspca_last_timings",
           "lspca_omega", "lspca_accumulate", "lspca_factor", "lspca_fit", "spca_fit",
           "lspca_transform", "lspca_transform_noalloc", "lspca_accumulate_host", "lspca_fit_host", "spca_fit_stream",
           "lspca_accumulate_csr", "lspca_fit_csr", "lspca_transform_csr", "spca_fit_csr",
           "lspca_server_create", "lspca_server_submit", "lspca_server_wait",
           "lspca_server_pause", "lspca_server_get_stats", "lspca_server_destroy"]


class LspcaError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class lspca_opts(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("sparse_p", ctypes.c_uint32),
                ("refine", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("small_route", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("stripe_rows", ctypes.c_int64)]


class lspca_timings(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("omega_ms", "sketch_ms", "factor_ms", "reduce_ms", "small_ms", "qr_ms",
                 "pass2_ms", "transform_ms", "total_ms", "layout_ms")]


class lspca_server_stats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("max_requests_per_launch", ctypes.c_uint32),
                ("max_concurrent_launches", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("launches", ctypes.c_uint64), ("rows_completed", ctypes.c_uint64),
                ("arena_peak_bytes", ctypes.c_uint64), ("queue_ns", ctypes.c_uint64),
                ("enqueue_ns", ctypes.c_uint64), ("device_ns", ctypes.c_uint64)]


_lib = None
_P, _I64, _I32, _U64, _U32 = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                              ctypes.c_uint64, ctypes.c_uint32)
_SIGS = {
    "lspca_version": ([], ctypes.c_char_p),
    "lspca_strerror": ([ctypes.c_int], ctypes.c_char_p),
    "lspca_last_error": ([], ctypes.c_char_p),
    "lspca_last_timings": ([ctypes.POINTER(lspca_timings)], ctypes.c_int),
    "lspca_omega": ([_I64, _I32, ctypes.c_int, _U64, _U32, ctypes.c_int, _P, _P], ctypes.c_int),
    "lspca_accumulate": ([_P, ctypes.c_int, _I64, _I64, _I64, _I32, ctypes.c_int, _U64,
                          ctypes.POINTER(lspca_opts), _P, _P], ctypes.c_int),
    "lspca_factor": ([_P, _P, _I32, _I64, ctypes.POINTER(lspca_opts), _P, _P, _P], ctypes.c_int),
    "lspca_fit": ([_P, ctypes.c_int, _I64, _I64, _I64, _I32, ctypes.c_int, _U64,
                   ctypes.POINTER(lspca_opts), _P, _P, _P], ctypes.c_int),
    "spca_fit": ([_P, ctypes.c_int, _I64, _I64, _I64, _I32, ctypes.c_int, _U64,
                  ctypes.POINTER(lspca_opts), _P, _P], ctypes.c_int),
    "lspca_transform": ([_P, ctypes.c_int, _I64, _I64, _I64, _P, _I32, _P,
                         ctypes.POINTER(lspca_opts)], ctypes.c_int),
    "lspca_transform_noalloc": ([_P, ctypes.c_int, _I64, _I64, _I64, _P, _I32, _P,
                                 ctypes.POINTER(lspca_opts)], ctypes.c_int),
    "spca_fit_stream": ([_P, ctypes.c_int, _I64, _I64, _I64, _I32, ctypes.c_int, _U64,
                         ctypes.POINTER(lspca_opts), _P, _P], ctypes.c_int),
    "lspca_accumulate_host": ([_P, ctypes.c_int, _I64, _I64, _I64, _I32, ctypes.c_int, _U64,
                               ctypes.POINTER(lspca_opts), _I64, _P, _P], ctypes.c_int),
    "lspca_fit_host": ([_P, ctypes.c_int, _I64, _I64, _I64, _I32, ctypes.c_int, _U64,
                        ctypes.POINTER(lspca_opts), _I64, _P, _P, _P], ctypes.c_int),
    "lspca_accumulate_csr": ([_P, _P, _P, ctypes.c_int, _I64, _I64, _I64, _I32, ctypes.c_int, _U64,
                              ctypes.POINTER(lspca_opts), _P, _P], ctypes.c_int),
    "lspca_fit_csr": ([_P, _P, _P, ctypes.c_int, _I64, _I64, _I64, _I32, ctypes.c_int, _U64,
                       ctypes.POINTER(lspca_opts), _P, _P, _P], ctypes.c_int),
    "lspca_transform_csr": ([_P, _P, _P, ctypes.c_int, _I64, _I64, _I64, _P, _I32, _P,
                             ctypes.POINTER(lspca_opts)], ctypes.c_int),
    "spca_fit_csr": ([_P, _P, _P, ctypes.c_int, _I64, _I64, _I64, _I32, ctypes.c_int, _U64,
                      ctypes.POINTER(lspca_opts), _P, _P], ctypes.c_int),
    "lspca_server_create": ([_P, _I64, _I32, ctypes.c_int, ctypes.c_size_t, _I32,
                             ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "lspca_server_submit": ([_P, _P, _I64, _P, ctypes.POINTER(_U64)], ctypes.c_int),
    "lspca_server_wait": ([_P, _U64, _I64, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "lspca_server_pause": ([_P, ctypes.c_int], ctypes.c_int),
    "lspca_server_get_stats": ([_P, ctypes.POINTER(lspca_server_stats)], ctypes.c_int),
    "lspca_server_destroy": ([_P], ctypes.c_int),
}


def load(path=LIB_PATH):
    """Load the built library (no build is attempted here)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run __graft_entry__.build() or "
                           "python paper_1709_07175_amd/build.py")
    lib = ctypes.CDLL(path)
    for name, (args, res) in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def exported_symbols(path=LIB_PATH):
    lib = ctypes.CDLL(path)
    return [n for n in EXPORTS if hasattr(lib, n)]


def version():
    return load().lspca_version().decode()


def _check(status):
    if status != 0:
        msg = load().lspca_last_error().decode(errors="replace")
        raise LspcaError(status, msg)


# ------------------------------------------------------------ torch glue --
def _torch():
    import torch
    return torch


_DT = None


def _dtype_code(t):
    torch = _torch()
    global _DT
    if _DT is None:
        _DT = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16, torch.float16: F16}
    if t.dtype not in _DT:
        raise TypeError(f"unsupported dtype {t.dtype}")
    return _DT[t.dtype]


def _dev(t, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    return t


def _rowmajor(X, name="X"):
    _dev(X, name)
    if X.dim() != 2 or X.stride(1) != 1:
        raise ValueError(f"{name} must be 2-D with unit column stride")
    return X.stride(0)


SMALL_ROUTE = {"qr": 0, "eig": 1}


def _opts(stream=None, sparse_p=0, refine=-1, timing=False, small_route="qr", stripe_rows=0):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    o = lspca_opts()
    o.struct_size = ctypes.sizeof(lspca_opts)
    o.sparse_p = sparse_p
    o.refine = refine
    o.timing = 1 if timing else 0
    o.stream = ctypes.c_void_p(stream.cuda_stream)
    o.small_route = SMALL_ROUTE[small_route] if isinstance(small_route, str) else int(small_route)
    o.stripe_rows = stripe_rows
    return o


def _f64_out(shape, device):
    torch = _torch()
    return torch.empty(shape, dtype=torch.float64, device=device)


def omega(n, k, kind, seed, dtype, p=0, device="cuda"):
    """Omega (n x k) as the fit uses it (lspca_omega)."""
    torch = _torch()
    tdt = {F64: torch.float64, F32: torch.float32, BF16: torch.bfloat16, F16: torch.float16}[dtype]
    out = torch.empty((n, k), dtype=tdt, device=device)
    _check(load().lspca_omega(n, k, KIND[kind], seed, p, dtype, out.data_ptr(),
                              torch.cuda.current_stream().cuda_stream))
    return out


def accumulate(X, k, kind, seed, F, G=None, **kw):
    """Algorithm 4 step 2 for the slice X: F += U^T X, G += U^T U (in place)."""
    ldx = _rowmajor(X)
    o = _opts(**kw)
    _check(load().lspca_accumulate(X.data_ptr(), _dtype_code(X), X.shape[0], X.shape[1], ldx, k,
                                   KIND[kind], seed, ctypes.byref(o), _dev(F, "F").data_ptr(),
                                   _dev(G, "G").data_ptr() if G is not None else None))
    return F, G


def factor(F, G=None, want_sigma_x=False, **kw):
    """Truncated SVD of F (k x n): returns V (n x k), D (k) and, if asked,
    Sigma^s (k) from G."""
    k, n = F.shape
    V = _f64_out((n, k), F.device)
    s = _f64_out((k,), F.device)
    sx = _f64_out((k,), F.device) if want_sigma_x else None
    o = _opts(**kw)
    _check(load().lspca_factor(_dev(F, "F").data_ptr(), G.data_ptr() if G is not None else None,
                               k, n, ctypes.byref(o), V.data_ptr(), s.data_ptr(),
                               sx.data_ptr() if sx is not None else None))
    return (V, s, sx) if want_sigma_x else (V, s)


def fit(X, k, kind="gaussian", seed=0, want_sigma_x=False, **kw):
    """Lazy SPCA (Algorithm 2): returns V (n x k), D (k) [, Sigma^s (k)]."""
    ldx = _rowmajor(X)
    m, n = X.shape
    V = _f64_out((n, k), X.device)
    s = _f64_out((k,), X.device)
    sx = _f64_out((k,), X.device) if want_sigma_x else None
    o = _opts(**kw)
    _check(load().lspca_fit(X.data_ptr(), _dtype_code(X), m, n, ldx, k, KIND[kind], seed,
                            ctypes.byref(o), V.data_ptr(), s.data_ptr(),
                            sx.data_ptr() if sx is not None else None))
    return (V, s, sx) if want_sigma_x else (V, s)


def spca_fit(X, k, kind="gaussian", seed=0, **kw):
    """SPCA (Algorithm 1) with a tall-skinny Householder QR: V^s, Sigma^s."""
    ldx = _rowmajor(X)
    m, n = X.shape
    V = _f64_out((n, k), X.device)
    s = _f64_out((k,), X.device)
    o = _opts(**kw)
    _check(load().spca_fit(X.data_ptr(), _dtype_code(X), m, n, ldx, k, KIND[kind], seed,
                           ctypes.byref(o), V.data_ptr(), s.data_ptr()))
    return V, s


def spca_fit_stream(X, k, kind="gaussian", seed=0, **kw):
    """Streaming SPCA (Algorithm 3), one pass over X: V^s, Sigma^s."""
    ldx = _rowmajor(X)
    m, n = X.shape
    V = _f64_out((n, k), X.device)
    s = _f64_out((k,), X.device)
    o = _opts(**kw)
    _check(load().spca_fit_stream(X.data_ptr(), _dtype_code(X), m, n, ldx, k, KIND[kind], seed,
                                  ctypes.byref(o), V.data_ptr(), s.data_ptr()))
    return V, s


def transform(X, V, Z=None, **kw):
    """Z = X V (FP64 for FP64 X, FP32 otherwise)."""
    torch = _torch()
    ldx = _rowmajor(X)
    r, n = X.shape
    k = V.shape[1]
    if V.dtype != torch.float64 or not V.is_contiguous():
        raise ValueError("V must be a contiguous FP64 device tensor")
    zdt = torch.float64 if X.dtype == torch.float64 else torch.float32
    if Z is None:
        Z = torch.empty((r, k), dtype=zdt, device=X.device)
    o = _opts(**kw)
    _check(load().lspca_transform(X.data_ptr(), _dtype_code(X), r, n, ldx, _dev(V, "V").data_ptr(),
                                  k, Z.data_ptr(), ctypes.byref(o)))
    return Z


# Size of the fixed device array lspca_transform_noalloc uses (the header's
# LSPCA_NOALLOC_SCRATCH_BYTES).
NOALLOC_SCRATCH_BYTES = 16 << 20


def transform_noalloc(X, V, Z, **kw):
    """Z = X V like transform(), through lspca_transform_noalloc: the library
    allocates nothing (V^T goes to its fixed per-device array), so Z must be
    given. Calls that overlap on one device race on that array."""
    torch = _torch()
    ldx = _rowmajor(X)
    r, n = X.shape
    k = V.shape[1]
    if V.dtype != torch.float64 or not V.is_contiguous():
        raise ValueError("V must be a contiguous FP64 device tensor")
    zdt = torch.float64 if X.dtype == torch.float64 else torch.float32
    if Z.dtype != zdt or tuple(Z.shape) != (r, k) or not Z.is_contiguous():
        raise ValueError(f"Z must be a contiguous {zdt} tensor of shape ({r}, {k})")
    o = _opts(**kw)
    _check(load().lspca_transform_noalloc(X.data_ptr(), _dtype_code(X), r, n, ldx,
                                          _dev(V, "V").data_ptr(), k, _dev(Z, "Z").data_ptr(),
                                          ctypes.byref(o)))
    return Z


class CSR:
    """A CSR matrix on the device: rowptr (m + 1, int64), colidx (int32) and
    values (FP32 or FP64), n columns. rowptr may be a row slice of a larger
    matrix (rowptr[0] > 0) sharing colidx and values."""

    def __init__(self, rowptr, colidx, values, n):
        torch = _torch()
        for t, name in ((rowptr, "rowptr"), (colidx, "colidx"), (values, "values")):
            _dev(t, name)
            if t.dim() != 1 or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous 1-D device tensor")
        if rowptr.dtype != torch.int64 or colidx.dtype != torch.int32:
            raise TypeError("rowptr must be int64 and colidx int32")
        if values.dtype not in (torch.float32, torch.float64):
            raise TypeError("values must be float32 or float64")
        if rowptr.numel() < 1:
            raise ValueError("rowptr needs m + 1 >= 1 entries")
        self.rowptr, self.colidx, self.values, self.n = rowptr, colidx, values, int(n)
        self.m = rowptr.numel() - 1
        self.nnz = int(rowptr[-1].item())              # end position of the last row
        if self.nnz > min(colidx.numel(), values.numel()):
            raise ValueError("rowptr[-1] exceeds the entries of colidx / values")

    def rows(self, r0, r1):
        """The row slice [r0, r1) (no copy)."""
        return CSR(self.rowptr[r0:r1 + 1], self.colidx, self.values, self.n)

    def _args(self):
        return (self.rowptr.data_ptr(), self.colidx.data_ptr(), self.values.data_ptr(),
                _dtype_code(self.values))


def accumulate_csr(X, k, kind, seed, F, G=None, **kw):
    """Algorithm 4 step 2 for a CSR slice X: F += U^T X, G += U^T U."""
    o = _opts(**kw)
    _check(load().lspca_accumulate_csr(*X._args(), X.m, X.n, X.nnz, k, KIND[kind], seed,
                                       ctypes.byref(o), _dev(F, "F").data_ptr(),
                                       _dev(G, "G").data_ptr() if G is not None else None))
    return F, G


def fit_csr(X, k, kind="gaussian", seed=0, want_sigma_x=False, **kw):
    """Lazy SPCA (Algorithm 2) of a CSR X: V (n x k), D (k) [, Sigma^s (k)]."""
    dev = X.values.device
    V = _f64_out((X.n, k), dev)
    s = _f64_out((k,), dev)
    sx = _f64_out((k,), dev) if want_sigma_x else None
    o = _opts(**kw)
    _check(load().lspca_fit_csr(*X._args(), X.m, X.n, X.nnz, k, KIND[kind], seed, ctypes.byref(o),
                                V.data_ptr(), s.data_ptr(), sx.data_ptr() if sx is not None else None))
    return (V, s, sx) if want_sigma_x else (V, s)


def spca_fit_csr(X, k, kind="gaussian", seed=0, **kw):
    """SPCA (Algorithm 1) of a CSR X with the GPU tall-skinny QR: V^s, Sigma^s."""
    dev = X.values.device
    V = _f64_out((X.n, k), dev)
    s = _f64_out((k,), dev)
    o = _opts(**kw)
    _check(load().spca_fit_csr(*X._args(), X.m, X.n, X.nnz, k, KIND[kind], seed, ctypes.byref(o),
                               V.data_ptr(), s.data_ptr()))
    return V, s


def transform_csr(X, V, Z=None, **kw):
    """Z = X V for a CSR X (Z of the value type)."""
    torch = _torch()
    k = V.shape[1]
    if V.dtype != torch.float64 or not V.is_contiguous() or V.shape[0] != X.n:
        raise ValueError("V must be a contiguous n x k FP64 device tensor")
    if Z is None:
        Z = torch.empty((X.m, k), dtype=X.values.dtype, device=X.values.device)
    o = _opts(**kw)
    _check(load().lspca_transform_csr(*X._args(), X.m, X.n, X.nnz, _dev(V, "V").data_ptr(), k,
                                      Z.data_ptr(), ctypes.byref(o)))
    return Z


def _host_rowmajor(X):
    if X.is_cuda:
        raise ValueError("X must be a host tensor (pinned for full copy rate)")
    if X.dim() != 2 or X.stride(1) != 1:
        raise ValueError("X must be 2-D with unit column stride")
    return X.stride(0)


def accumulate_host(X, k, kind, seed, F, G=None, stripe_rows=0, **kw):
    """Algorithm 4 over a host tensor X (streamed through the device):
    F += U^T X, G += U^T U on the device accumulators (in place)."""
    ldx = _host_rowmajor(X)
    o = _opts(**kw)
    _check(load().lspca_accumulate_host(X.data_ptr(), _dtype_code(X), X.shape[0], X.shape[1], ldx, k,
                                        KIND[kind], seed, ctypes.byref(o), stripe_rows,
                                        _dev(F, "F").data_ptr(),
                                        _dev(G, "G").data_ptr() if G is not None else None))
    return F, G


def fit_host(X, k, kind="gaussian", seed=0, want_sigma_x=False, stripe_rows=0, device="cuda", **kw):
    """Lazy SPCA (Algorithm 4) of a host tensor X: V (n x k), D (k)
    [, Sigma^s (k)] on the device."""
    ldx = _host_rowmajor(X)
    m, n = X.shape
    V = _f64_out((n, k), device)
    s = _f64_out((k,), device)
    sx = _f64_out((k,), device) if want_sigma_x else None
    o = _opts(**kw)
    _check(load().lspca_fit_host(X.data_ptr(), _dtype_code(X), m, n, ldx, k, KIND[kind], seed,
                                 ctypes.byref(o), stripe_rows, V.data_ptr(), s.data_ptr(),
                                 sx.data_ptr() if sx is not None else None))
    return (V, s, sx) if want_sigma_x else (V, s)


def last_timings():
    t = lspca_timings()
    _check(load().lspca_last_timings(ctypes.byref(t)))
    return {n: getattr(t, n) for n, _ in lspca_timings._fields_}


class Server:
    """Projection server (lspca_server_*): continuous batching of Z = X V.

    V (n x k FP64, device) is copied at creation. submit() takes X (r x n,
    rows contiguous, the server's dtype) and Z (r x k, FP32; FP64 for an F64
    server), both device tensors or both host tensors (pinned for
    asynchronous copies), and returns a ticket; wait() returns the latency
    in ms measured by the server. The tensors must stay alive and untouched
    until the request completes.
    """

    def __init__(self, V, dtype, arena_bytes=0, max_inflight=32):
        torch = _torch()
        if V.dtype != torch.float64 or not V.is_cuda or not V.is_contiguous():
            raise ValueError("V must be a contiguous FP64 device tensor")
        self.n, self.k = V.shape
        self.dtype = dtype
        h = ctypes.c_void_p()
        _check(load().lspca_server_create(V.data_ptr(), self.n, self.k, dtype, arena_bytes,
                                          max_inflight, ctypes.byref(h)))
        self._h = h

    def submit(self, X, Z):
        if X.dim() != 2 or X.shape[1] != self.n or not X.is_contiguous():
            raise ValueError("X must be a contiguous r x n tensor")
        if _dtype_code(X) != self.dtype:
            raise TypeError("X dtype differs from the server's")
        if Z.shape != (X.shape[0], self.k) or not Z.is_contiguous():
            raise ValueError("Z must be a contiguous r x k tensor")
        t = _U64()
        _check(load().lspca_server_submit(self._h, X.data_ptr(), X.shape[0], Z.data_ptr(),
                                          ctypes.byref(t)))
        return t.value

    def submit_ptr(self, x_ptr, rows, z_ptr):
        """Submit by raw addresses (rows contiguous, as submit)."""
        t = _U64()
        _check(load().lspca_server_submit(self._h, x_ptr, rows, z_ptr, ctypes.byref(t)))
        return t.value

    def wait(self, ticket, timeout_us=-1):
        lat = ctypes.c_double()
        _check(load().lspca_server_wait(self._h, ticket, timeout_us, ctypes.byref(lat)))
        return lat.value

    def pause(self, paused=True):
        _check(load().lspca_server_pause(self._h, 1 if paused else 0))

    def stats(self):
        st = lspca_server_stats()
        st.struct_size = ctypes.sizeof(lspca_server_stats)
        _check(load().lspca_server_get_stats(self._h, ctypes.byref(st)))
        return {n: getattr(st, n) for n, _ in lspca_server_stats._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().lspca_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
