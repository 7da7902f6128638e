"""lspca_transform_noalloc, the projection for callers that cannot allocate
device memory: called through the C ABI, its Z must be bitwise the one
lspca_transform gives on the same inputs (the same kernels; only where V^T
lives differs), on two calls in a row with the second one smaller, for every
type of X, at the largest V the fixed scratch holds, and interleaved with
lspca_transform on other streams (their buffers are separate)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _tdt(dtype):
    import torch
    return {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16,
            "f16": torch.float16}[dtype]


def _inputs(r, n, k, dtype, seed, ldx=None):
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    ldx = ldx or n
    Xfull = torch.randn(r, ldx, generator=g, device="cuda", dtype=torch.float64).to(_tdt(dtype))
    X = Xfull[:, :n]                                   # leading dimension ldx >= n
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, k)))
    V = torch.from_numpy(np.ascontiguousarray(q)).cuda()
    return X, V


def _zeros_like_out(X, k):
    import torch
    zdt = torch.float64 if X.dtype == torch.float64 else torch.float32
    return torch.full((X.shape[0], k), float("nan"), dtype=zdt, device="cuda")


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
def test_noalloc_matches_transform_two_calls(gpu_lib, dtype):
    import torch
    # first call: several row tiles and a ragged tail; second: smaller in
    # every dimension and with a leading dimension above n
    for (r, n, k, ldx, seed) in ((5003, 1100, 96, None, 1), (777, 300, 40, 320, 2)):
        X, V = _inputs(r, n, k, dtype, seed, ldx)
        Z_ref = gpu_lib.transform(X, V)
        Z = _zeros_like_out(X, k)
        gpu_lib.transform_noalloc(X, V, Z)
        torch.cuda.synchronize()
        assert torch.equal(Z, Z_ref), (dtype, r, n, k)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
def test_noalloc_at_the_scratch_limit(gpu_lib, dtype):
    import torch
    es = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}[dtype]
    parts = 2 if dtype in ("bf16", "f16") else 1
    k = 256
    n = gpu_lib.NOALLOC_SCRATCH_BYTES // (es * parts * k)   # V^T fills the array exactly
    X, V = _inputs(300, n, k, dtype, 3)
    Z_ref = gpu_lib.transform(X, V)
    Z = _zeros_like_out(X, k)
    gpu_lib.transform_noalloc(X, V, Z)
    torch.cuda.synchronize()
    assert torch.equal(Z, Z_ref)
    # one more row of V does not fit
    X2, V2 = _inputs(8, n + 1, k, dtype, 4)
    with pytest.raises(gpu_lib.LspcaError) as e:
        gpu_lib.transform_noalloc(X2, V2, _zeros_like_out(X2, k))
    assert e.value.name == "LSPCA_E2BIG"


def test_noalloc_interleaved_with_transform_on_other_streams(gpu_lib):
    import torch
    X, V = _inputs(65_536, 4096, 256, "bf16", 5)
    Xs, Vs = _inputs(1000, 512, 32, "bf16", 6)
    Z_ref = gpu_lib.transform(X, V)
    Zs_ref = gpu_lib.transform(Xs, Vs)
    torch.cuda.synchronize()
    sA, sB = torch.cuda.Stream(), torch.cuda.Stream()
    for it in range(3):
        Z = _zeros_like_out(X, 256)
        Zs = _zeros_like_out(Xs, 32)
        Zw = _zeros_like_out(Xs, 32)
        torch.cuda.synchronize()
        gpu_lib.transform_noalloc(X, V, Z, stream=sA)    # queued, not waited
        gpu_lib.transform(Xs, Vs, Z=Zw, stream=sB)       # the library's workspace
        sA.synchronize()
        gpu_lib.transform_noalloc(Xs, Vs, Zs, stream=sA)
        torch.cuda.synchronize()
        assert torch.equal(Z, Z_ref), it
        assert torch.equal(Zs, Zs_ref), it
        assert torch.equal(Zw, Zs_ref), it
