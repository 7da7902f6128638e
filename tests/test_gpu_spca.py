"""GPU-vs-oracle parity for spca_fit (Algorithm 1 with the tall-skinny
Householder QR), and Proposition 2 across the two GPU fits."""
import numpy as np
import pytest

from oracle import lspca_oracle as O
from oracle import philox as P
from synth import lowrank_np, storage_to_f64
from tests.helpers import U32, gamma, subspace_tol, to_device

pytestmark = pytest.mark.gpu


def _data(m, n, k, dtype, seed=5):
    Xs = lowrank_np(m, n, k, "invsqrt", 0.05, seed, dtype)
    return Xs, storage_to_f64(Xs, dtype)


def _f_bound(X64, Q, k, dtype):
    """Error of F = Q^T X from an FP32 Householder Q: the QR's backward error
    (orthogonality loss of Q and ||U - QR||, each about c k u in relative
    terms; c = 20 here) moves F by at most that times ||X||_2, and the FP32
    accumulation of Q^T X adds gamma_m |Q|^T |X|. 16-bit data: Q enters as
    Q_hi + Q_lo, with u16^2 |Q| left over."""
    m = X64.shape[0]
    normX = np.linalg.norm(X64, 2)
    b = 20 * k * U32 * normX * np.ones((k, X64.shape[1])) / np.sqrt(X64.shape[1])
    b = b + gamma(m, U32) * (np.abs(Q).T @ np.abs(X64))
    if dtype in ("bf16", "f16"):
        u16 = 2.0 ** -8 if dtype == "bf16" else 2.0 ** -11
        b = b + 1.01 * u16 ** 2 * (np.abs(Q).T @ np.abs(X64))
    return b


@pytest.mark.parametrize("m,n,k", [(1037, 203, 17), (128, 60, 7), (129, 60, 7), (300, 80, 50),
                                   (3 * 128 + 5, 40, 20)])
def test_spca_fit_f64_matches_oracle(gpu_lib, m, n, k):
    """FP64: leaves of 128 rows; ragged last leaf, one leaf, odd trees."""
    Xs, X64 = _data(m, n, k, "f64")
    V, s = gpu_lib.spca_fit(to_device(Xs, "f64"), k, "gaussian", 3)
    ref = O.spca_fit(X64, P.omega(n, k, "gaussian", 3), k)
    V = V.cpu().numpy()
    assert O.principal_sines(ref["V"], V).max() < 1e-10
    assert np.max(np.abs(s.cpu().numpy() - ref["sigma"]) / ref["sigma"]) < 1e-10


def test_spca_fit_full_first_config_f64(gpu_lib):
    from synth import config
    c = config(1)
    Xs = lowrank_np(c["m"], c["n"], c["r"], c["spectrum"], c["s"], c["data_seed"], "f64")
    V, s = gpu_lib.spca_fit(to_device(Xs, "f64"), c["k"], "gaussian", c["omega_seed"])
    ref = O.spca_fit(Xs, P.omega(c["n"], c["k"], "gaussian", c["omega_seed"]), c["k"])
    assert O.principal_sines(ref["V"], V.cpu().numpy()).max() < 1e-10
    assert np.max(np.abs(s.cpu().numpy() - ref["sigma"]) / ref["sigma"]) < 1e-10


@pytest.mark.parametrize("m,n,k,dtype", [(1037, 203, 17, "f32"), (2600, 512, 256, "f32"),
                                         (1037, 203, 17, "bf16"), (2049, 300, 64, "f16")])
def test_spca_fit_lower_precision_within_bound(gpu_lib, m, n, k, dtype):
    Xs, X64 = _data(m, n, k, dtype)
    V, s = gpu_lib.spca_fit(to_device(Xs, dtype), k, "gaussian", 11)
    om = P.omega(n, k, "gaussian", 11, dtype=dtype)
    ref = O.spca_fit(X64, om, k)
    err = np.linalg.norm(_f_bound(X64, ref["Q"], k, dtype))
    s = s.cpu().numpy()
    assert np.max(np.abs(s - ref["sigma"]) / ref["sigma"]) <= err / ref["sigma"][-1] + 1e-12
    assert O.principal_sines(ref["V"], V.cpu().numpy()).max() <= subspace_tol(ref["sigma"][-1], err) + 1e-12


def test_proposition_2_across_gpu_fits(gpu_lib):
    """Prop. 2: the GPU SPCA and GPU Lazy SPCA bases span the same subspace;
    Prop. 3: identical pairwise distances after projection."""
    import torch
    m, n, k = 4000, 300, 24
    Xs, X64 = _data(m, n, k, "f64")
    X = to_device(Xs, "f64")
    Vs, _ = gpu_lib.spca_fit(X, k, "gaussian", 8)
    Vl, _ = gpu_lib.fit(X, k, "gaussian", 8)
    assert O.principal_sines(Vs.cpu().numpy(), Vl.cpu().numpy()).max() < 1e-10
    Zs = gpu_lib.transform(X, Vs).cpu().numpy()
    Zl = gpu_lib.transform(X, Vl).cpu().numpy()
    pairs = np.random.default_rng(0).integers(0, m, size=(3000, 2))
    ds, dl = O.pairwise_distances(Zs, pairs), O.pairwise_distances(Zl, pairs)
    assert np.max(np.abs(ds - dl)) <= 1e-10 * np.max(ds)
    torch.cuda.synchronize()


def test_spca_fit_k_above_block_height_is_refused(gpu_lib):
    Xs, _ = _data(400, 300, 10, "f64")
    with pytest.raises(gpu_lib.LspcaError) as e:
        gpu_lib.spca_fit(to_device(Xs, "f64"), 129, "gaussian", 1)
    assert e.value.name == "LSPCA_ENOTSUP"


# ------------------------------------------------- Algorithm 3 (streaming) --

@pytest.fixture
def small_stripes(monkeypatch):
    """Per-stripe sketch budget of 256 KiB: several stripes (and R merges)
    even for small inputs. The library reads it at every call."""
    monkeypatch.setenv("LSPCA_STRIPE_BYTES", str(256 * 1024))
    yield


@pytest.mark.parametrize("m,n,k", [(1037, 203, 17), (3000, 80, 50), (129, 60, 7)])
def test_spca_fit_stream_f64_matches_oracle(gpu_lib, m, n, k):
    Xs, X64 = _data(m, n, k, "f64")
    V, s = gpu_lib.spca_fit_stream(to_device(Xs, "f64"), k, "gaussian", 3)
    ref = O.streaming_spca_fit(X64, P.omega(n, k, "gaussian", 3), k, S=3)
    assert O.principal_sines(ref["V"], V.cpu().numpy()).max() < 1e-10
    assert np.max(np.abs(s.cpu().numpy() - ref["sigma"]) / ref["sigma"]) < 1e-10


@pytest.mark.parametrize("m,n,k,dtype", [(9000, 120, 24, "f64"), (9000, 200, 24, "f32"),
                                         (9000, 256, 32, "bf16")])
def test_spca_fit_stream_many_stripes(gpu_lib, small_stripes, m, n, k, dtype):
    """Several stripes: the running R is merged with every stripe's R."""
    Xs, X64 = _data(m, n, k, dtype)
    V, s = gpu_lib.spca_fit_stream(to_device(Xs, dtype), k, "gaussian", 4)
    om = P.omega(n, k, "gaussian", 4, dtype=dtype)
    ref = O.spca_fit(X64, om, k)
    if dtype == "f64":
        assert O.principal_sines(ref["V"], V.cpu().numpy()).max() < 1e-10
        assert np.max(np.abs(s.cpu().numpy() - ref["sigma"]) / ref["sigma"]) < 1e-10
    else:
        err = np.linalg.norm(_f_bound(X64, ref["Q"], k, dtype))
        s = s.cpu().numpy()
        assert np.max(np.abs(s - ref["sigma"]) / ref["sigma"]) <= err / ref["sigma"][-1] + 1e-12
        assert O.principal_sines(ref["V"], V.cpu().numpy()).max() <= subspace_tol(ref["sigma"][-1], err) + 1e-12


def test_streaming_and_two_pass_spca_agree(gpu_lib):
    """Algorithm 3 and Algorithm 1 compute the same V^s and Sigma^s."""
    m, n, k = 6000, 300, 30
    Xs, _ = _data(m, n, k, "f64")
    X = to_device(Xs, "f64")
    V1, s1 = gpu_lib.spca_fit(X, k, "gaussian", 6)
    V3, s3 = gpu_lib.spca_fit_stream(X, k, "gaussian", 6)
    assert O.principal_sines(V1.cpu().numpy(), V3.cpu().numpy()).max() < 1e-10
    assert np.max(np.abs(s1.cpu().numpy() - s3.cpu().numpy()) / s1.cpu().numpy()) < 1e-11


def test_lazy_fit_many_stripes_matches_one_stripe(gpu_lib, monkeypatch):
    """The fit's own stripe loop (Algorithm 4 over device-resident X)."""
    m, n, k = 9000, 200, 20
    Xs, X64 = _data(m, n, k, "f64")
    X = to_device(Xs, "f64")
    V1, s1 = gpu_lib.fit(X, k, "gaussian", 2)
    monkeypatch.setenv("LSPCA_STRIPE_BYTES", str(128 * 1024))
    V2, s2 = gpu_lib.fit(X, k, "gaussian", 2)
    assert O.principal_sines(V1.cpu().numpy(), V2.cpu().numpy()).max() < 1e-10
    assert np.max(np.abs(s1.cpu().numpy() - s2.cpu().numpy()) / s1.cpu().numpy()) < 1e-11
