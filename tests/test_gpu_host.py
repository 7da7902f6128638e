"""GPU tests of Algorithm 4 over X in host memory (lspca_accumulate_host,
lspca_fit_host): the streamed F and G against the FP64 oracle within the
pass bound, resuming from a saved (F, G), and the fit against the
device-resident fit."""
import numpy as np
import pytest

from oracle import lspca_oracle as O
from oracle import philox as P
from synth import lowrank_np, storage_to_f64
from tests.helpers import pass_bound, to_device

pytestmark = pytest.mark.gpu


def _host(Xs, dtype, pin=True):
    t = to_device(Xs, dtype, device="cpu")
    return t.pin_memory() if pin else t.contiguous()


@pytest.mark.parametrize("m,n,k,dtype,stripe", [(5000, 300, 20, "f64", 1024), (4999, 203, 17, "f32", 512),
                                                (6000, 512, 64, "bf16", 1024), (3001, 256, 32, "f16", 768)])
def test_streamed_pass_matches_oracle(gpu_lib, m, n, k, dtype, stripe):
    import torch
    Xs = lowrank_np(m, n, k, "invsqrt", 0.05, 41, dtype)
    X64 = storage_to_f64(Xs, dtype)
    om = P.omega(n, k, "gaussian", 9, dtype=dtype)
    F = torch.zeros((k, n), dtype=torch.float64, device="cuda")
    G = torch.zeros((k, k), dtype=torch.float64, device="cuda")
    gpu_lib.accumulate_host(_host(Xs, dtype), k, "gaussian", 9, F, G, stripe_rows=stripe)
    ref = O.streaming_lazy_fit(X64, om, k)
    bF, bG = pass_bound(X64, om, dtype)
    assert np.all(np.abs(F.cpu().numpy() - ref["F"]) <= bF)
    assert np.all(np.abs(G.cpu().numpy() - ref["G"]) <= bG)


def test_resume_from_saved_state(gpu_lib):
    """Save (F, G) to the host after the first rows, restore it into fresh
    buffers, stream the remaining rows: the result equals one uninterrupted
    stream within the pass bound (Algorithm 4 is a sum over slices)."""
    import torch
    m, n, k, m1 = 6000, 384, 24, 2500
    Xs = lowrank_np(m, n, k, "invsqrt", 0.05, 42, "f32")
    X64 = storage_to_f64(Xs, "f32")
    Xh = _host(Xs, "f32")
    F = torch.zeros((k, n), dtype=torch.float64, device="cuda")
    G = torch.zeros((k, k), dtype=torch.float64, device="cuda")
    gpu_lib.accumulate_host(Xh[:m1], k, "gaussian", 5, F, G, stripe_rows=1024)
    saved = (F.cpu().numpy().copy(), G.cpu().numpy().copy())
    del F, G
    F2 = torch.from_numpy(saved[0]).cuda()
    G2 = torch.from_numpy(saved[1]).cuda()
    gpu_lib.accumulate_host(Xh[m1:], k, "gaussian", 5, F2, G2, stripe_rows=1024)
    om = P.omega(n, k, "gaussian", 5, dtype="f32")
    ref = O.streaming_lazy_fit(X64, om, k)
    bF, bG = pass_bound(X64, om, "f32")
    assert np.all(np.abs(F2.cpu().numpy() - ref["F"]) <= bF)
    assert np.all(np.abs(G2.cpu().numpy() - ref["G"]) <= bG)


@pytest.mark.parametrize("pin", [True, False])
def test_fit_host_matches_device_fit(gpu_lib, pin):
    m, n, k = 9000, 250, 20
    Xs = lowrank_np(m, n, k, "invsqrt", 0.05, 43, "f64")
    Vh, sh, sxh = gpu_lib.fit_host(_host(Xs, "f64", pin), k, "gaussian", 3, want_sigma_x=True,
                                   stripe_rows=2048)
    Vd, sd, sxd = gpu_lib.fit(to_device(Xs, "f64"), k, "gaussian", 3, want_sigma_x=True)
    assert O.principal_sines(Vd.cpu().numpy(), Vh.cpu().numpy()).max() < 1e-10
    assert np.max(np.abs(sh.cpu().numpy() - sd.cpu().numpy()) / sd.cpu().numpy()) < 1e-11
    assert np.max(np.abs(sxh.cpu().numpy() - sxd.cpu().numpy()) / sxd.cpu().numpy()) < 1e-11


def test_device_x_is_refused(gpu_lib):
    import torch
    Xd = torch.zeros((100, 20), dtype=torch.float32, device="cuda")
    F = torch.zeros((4, 20), dtype=torch.float64, device="cuda")
    st = gpu_lib.load().lspca_accumulate_host(Xd.data_ptr(), gpu_lib.F32, 100, 20, 20, 4, gpu_lib.GAUSSIAN, 1,
                                              None, 0, F.data_ptr(), None)
    assert st == -1 and "device memory" in gpu_lib.load().lspca_last_error().decode()
