"""Calls queued on different streams share the library's per-device
workspace (the converted V of a projection, F and G of a fit, ...). The
library orders them on the device: each call's stream waits for the previous
call's last use of the workspace. Here a large projection is queued on one
stream and, at once, fits run on another; every result must be bitwise the
one each call gives alone."""
import numpy as np
import pytest

from synth import lowrank_np

pytestmark = pytest.mark.gpu


def _orth(n, k, seed):
    import torch
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, k)))
    return torch.from_numpy(np.ascontiguousarray(q)).cuda()


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_projection_and_fit_on_two_streams(gpu_lib, dtype):
    import torch
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16}[dtype]
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    # the projection: 262,144 x 4,096 rows (a few ms of device work)
    X = torch.randn(262_144, 4096, generator=g, device="cuda", dtype=torch.float32).to(tdt)
    V = _orth(4096, 256, 1)
    # the fits: a small FP32 matrix, two different k
    Xs = torch.from_numpy(lowrank_np(6000, 512, 32, "invsqrt", 0.05, 3, "f32")).cuda()
    torch.cuda.synchronize()
    Z_ref = gpu_lib.transform(X, V)
    fits_ref = [gpu_lib.fit(Xs, kk, "gaussian", 11) for kk in (32, 48)]
    torch.cuda.synchronize()
    sA, sB = torch.cuda.Stream(), torch.cuda.Stream()
    for it in range(3):
        Z = torch.full_like(Z_ref, float("nan"))
        torch.cuda.synchronize()
        gpu_lib.transform(X, V, Z=Z, stream=sA)          # queued, not waited
        fits = [gpu_lib.fit(Xs, kk, "gaussian", 11, stream=sB) for kk in (32, 48)]
        torch.cuda.synchronize()
        assert torch.equal(Z, Z_ref), f"projection differs on iteration {it}"
        for (V1, s1), (V0, s0) in zip(fits, fits_ref):
            assert torch.equal(V1, V0) and torch.equal(s1, s0), f"fit differs on iteration {it}"
    # the other order: a fit's pass on one stream, then a projection on another
    F = torch.zeros((64, 512), dtype=torch.float64, device="cuda")
    F_ref = F.clone()
    gpu_lib.accumulate(Xs, 64, "gaussian", 3, F_ref)
    torch.cuda.synchronize()
    gpu_lib.accumulate(Xs, 64, "gaussian", 3, F, stream=sB)
    Z = torch.full_like(Z_ref, float("nan"))
    gpu_lib.transform(X, V, Z=Z, stream=sA)
    torch.cuda.synchronize()
    assert torch.equal(F, F_ref)
    assert torch.equal(Z, Z_ref)
