"""Low-rank-plus-noise data matrices, seeded, in every storage type.

Storage types are named "f64", "f32", "bf16", "f16". numpy has no bfloat16,
so BF16 data live in numpy as uint16 bit patterns; `storage_to_f64` decodes
any storage array exactly into float64. Down-conversion is round to nearest
even (FP64 -> FP32 -> BF16/FP16 in two steps, the same convention as the
library's Omega specification).
"""
import math

import numpy as np

# Workload presets: the shapes, spectra and noise levels of the five
# configurations (dense stand-ins for the paper's sparse datasets).
CONFIGS = {
    1: dict(name="lazy-vs-spca-f64", m=20_000, n=1_000, r=50, spectrum="inv",
            s=0.01, k=50, kind="gaussian", dtype="f64"),
    2: dict(name="lazy-vs-spca-f32", m=1_000_000, n=4_096, r=256, spectrum="invsqrt",
            s=0.05, k=256, kind="gaussian", dtype="f32"),
    3: dict(name="precision-bf16-sparse", m=1_000_000, n=4_096, r=256, spectrum="invsqrt",
            s=0.05, k=256, kind="sparse", dtype="bf16", p=64),
    4: dict(name="large-f16", m=4_600_000, n=2_048, r=128, spectrum="inv",
            s=0.02, k=128, kind="gaussian", dtype="f16"),
    5: dict(name="serving-bf16", m=65_536, n=4_096, r=256, spectrum="invsqrt",
            s=0.05, k=256, kind="gaussian", dtype="bf16"),
}


def config(i, **over):
    c = dict(CONFIGS[i])
    c.update(over)
    c.setdefault("p", 64)
    c["data_seed"] = 17090700 + i
    c["omega_seed"] = 7175 + i
    return c


def sigmas(spectrum, r, scale=1.0):
    i = np.arange(1, r + 1, dtype=np.float64)
    if spectrum == "inv":
        s = 1.0 / i
    elif spectrum == "invsqrt":
        s = i ** -0.5
    elif spectrum == "flat":
        s = np.ones(r)
    else:
        raise ValueError(spectrum)
    return scale * s


def random_orthonormal_np(rows, cols, rng):
    """Gaussian rows x cols matrix with orthonormal columns (via QR)."""
    q, r = np.linalg.qr(rng.standard_normal((rows, cols)))
    return q * np.sign(np.diag(r))


def _bf16_bits(f32):
    u = np.ascontiguousarray(f32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)
    return (u & np.uint64(0xFFFF)).astype(np.uint16)


def to_storage_np(X64, dtype):
    """FP64 array -> storage array (uint16 bit patterns for BF16)."""
    X64 = np.asarray(X64, dtype=np.float64)
    if dtype == "f64":
        return np.ascontiguousarray(X64)
    f32 = X64.astype(np.float32)
    if dtype == "f32":
        return f32
    if dtype == "f16":
        return f32.astype(np.float16)
    if dtype == "bf16":
        return _bf16_bits(f32)
    raise ValueError(dtype)


def storage_to_f64(Xs, dtype):
    """Storage array -> exact FP64 values."""
    if dtype == "bf16":
        u = np.asarray(Xs, dtype=np.uint16).astype(np.uint32) << np.uint32(16)
        return u.view(np.float32).astype(np.float64)
    return np.asarray(Xs).astype(np.float64)


def lowrank_np(m, n, r, spectrum="inv", s=0.01, seed=0, dtype="f64", scale=1.0):
    """X = A diag(sigma) B^T + E (m x n) in the storage type, from numpy's
    PCG64 stream seeded with `seed`."""
    rng = np.random.default_rng(seed)
    r = min(r, m, n)
    A = random_orthonormal_np(m, r, rng)
    B = random_orthonormal_np(n, r, rng)
    X = (A * sigmas(spectrum, r, scale)) @ B.T
    if s:
        X += s * rng.standard_normal((m, n))
    return to_storage_np(X, dtype)


_TORCH_DT = {"f64": "float64", "f32": "float32", "bf16": "bfloat16", "f16": "float16"}


def _orthonormal_torch(rows, cols, g, device):
    """Gaussian rows x cols matrix with orthonormal columns, by one Cholesky
    QR pass in FP64 on the device (the cols x cols factor on the host)."""
    import torch
    A = torch.randn(rows, cols, generator=g, device=device, dtype=torch.float64)
    Gm = (A.t() @ A).cpu().numpy()
    Linv = np.linalg.inv(np.linalg.cholesky(Gm))
    return A @ torch.from_numpy(Linv.T.copy()).to(device)


def lowrank_torch(m, n, r, spectrum="inv", s=0.01, seed=0, dtype="f32",
                  device="cuda", scale=1.0, chunk_rows=65_536, out=None):
    """The same model, drawn with torch's generator on `device`, written
    chunk by chunk (for matrices too large to draw on the host). Returns a
    contiguous (m, n) tensor of the storage type."""
    import torch
    tdt = getattr(torch, _TORCH_DT[dtype])
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    r = min(r, m, n)
    A = _orthonormal_torch(m, r, g, device).to(torch.float32)
    Bm = _orthonormal_torch(n, r, g, device)
    sig = torch.as_tensor(sigmas(spectrum, r, scale), device=device, dtype=torch.float64)
    Bs = (Bm * sig).t().contiguous().to(torch.float32)        # r x n
    X = out if out is not None else torch.empty(m, n, device=device, dtype=tdt)
    for r0 in range(0, m, chunk_rows):
        r1 = min(m, r0 + chunk_rows)
        blk = A[r0:r1] @ Bs
        if s:
            blk += s * torch.randn(r1 - r0, n, generator=g, device=device,
                                   dtype=torch.float32)
        X[r0:r1] = blk.to(tdt)
    del A, Bm, Bs
    return X


def request_sizes(count, seed, max_rows=65_536):
    """Request row counts r = floor(exp(u ln(max_rows + 1))), u ~ U[0, 1):
    log-uniform on [1, max_rows]."""
    rng = np.random.default_rng(seed)
    u = rng.random(count)
    r = np.floor(np.exp(u * math.log(max_rows + 1))).astype(np.int64)
    return np.clip(r, 1, max_rows)
