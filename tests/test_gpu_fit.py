"""GPU-vs-oracle parity for Omega, the pass (F, G), the small stage, the
Lazy SPCA fit and the projection, through the C ABI (Python binding)."""
import numpy as np
import pytest

from oracle import lspca_oracle as O
from oracle import philox as P
from synth import lowrank_np, random_orthonormal_np, storage_to_f64
from tests.helpers import U32, U64, pass_bound, subspace_tol, to_device

pytestmark = pytest.mark.gpu

TORCH_DT = {"f64": "float64", "f32": "float32", "bf16": "bfloat16", "f16": "float16"}
CODE = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3}

# (m, n, k, dtype): ragged sizes that span several tiles, with odd n (scalar
# load path) and n a multiple of 4 (vector load path)
PASS_CASES = [
    (1037, 203, 17, "f64"),
    (2000, 256, 32, "f64"),
    (1037, 203, 17, "f32"),
    (3001, 516, 64, "f32"),
    (1037, 203, 17, "bf16"),
    (3001, 520, 136, "bf16"),
    (1037, 203, 17, "f16"),
    (2999, 512, 64, "f16"),
    # m and n multiples of 8: the 16-bit vector-load paths, split-row chunk tails
    (4000, 512, 64, "bf16"),
    (3008, 520, 136, "f16"),
    (6000, 256, 256, "bf16"),
    # FP32 with m >= 4096 and n a multiple of 32: the streamed sketch kernel
    # (128 x 128 tiles for k <= 128, 128 x 256 above), ragged last row tile
    (5003, 512, 100, "f32"),
    (4500, 256, 200, "f32"),
]


def _data(m, n, k, dtype, seed=11, spectrum="invsqrt", s=0.05):
    Xs = lowrank_np(m, n, k, spectrum, s, seed, dtype)
    return Xs, storage_to_f64(Xs, dtype)


# ------------------------------------------------------------------ Omega --

@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
@pytest.mark.parametrize("kind", ["gaussian", "sparse"])
def test_omega_matches_specification(gpu_lib, dtype, kind):
    import torch
    n, k, seed = 333, 70, (1 << 33) + 77
    dev = gpu_lib.omega(n, k, kind, seed, CODE[dtype], p=16)
    got = dev.to(torch.float64).cpu().numpy()
    want = P.omega(n, k, kind, seed, p=16, dtype=dtype)
    if kind == "sparse":
        assert np.array_equal(got, want)                     # integer work: exact
    elif dtype == "f64":
        # both sides evaluate log/sqrt/cos/sin in FP64 (device vs host libm)
        assert np.max(np.abs(got - want) / np.maximum(1, np.abs(want))) < 8 * U64
    else:
        # rounding the FP64 value to FP32/16-bit: identical unless the two FP64
        # values straddle a rounding boundary (probability ~1e-8 per entry)
        mism = np.count_nonzero(got != want)
        assert mism <= 2
        ulp = {"f32": 2.0 ** -23, "bf16": 2.0 ** -7, "f16": 2.0 ** -10}[dtype]
        assert np.all(np.abs(got - want) <= ulp * np.maximum(np.abs(want), 2.0 ** -14) + 1e-300)


# ------------------------------------------------------------------- pass --

@pytest.mark.parametrize("m,n,k,dtype", PASS_CASES)
def test_accumulate_matches_oracle_within_bound(gpu_lib, m, n, k, dtype):
    import torch
    Xs, X64 = _data(m, n, k, dtype)
    om = P.omega(n, k, "gaussian", 99, dtype=dtype)
    X = to_device(Xs, dtype)
    F = torch.zeros((k, n), dtype=torch.float64, device="cuda")
    G = torch.zeros((k, k), dtype=torch.float64, device="cuda")
    gpu_lib.accumulate(X, k, "gaussian", 99, F, G)
    torch.cuda.synchronize()
    ref = O.streaming_lazy_fit(X64, om, k)
    bF, bG = pass_bound(X64, om, dtype)
    eF = np.abs(F.cpu().numpy() - ref["F"])
    eG = np.abs(G.cpu().numpy() - ref["G"])
    assert np.all(eF <= bF), float(np.max(eF / bF))
    assert np.all(eG <= bG), float(np.max(eG / bG))


def test_accumulate_over_slices_equals_one_pass(gpu_lib):
    """Algorithm 4: any horizontal slicing accumulates the same F."""
    import torch
    m, n, k, dtype = 2999, 260, 24, "f32"
    Xs, X64 = _data(m, n, k, dtype)
    X = to_device(Xs, dtype)
    F1 = torch.zeros((k, n), dtype=torch.float64, device="cuda")
    gpu_lib.accumulate(X, k, "gaussian", 5, F1)
    F3 = torch.zeros((k, n), dtype=torch.float64, device="cuda")
    for r0, r1 in [(0, 1000), (1000, 1001), (1001, m)]:
        gpu_lib.accumulate(X[r0:r1], k, "gaussian", 5, F3)
    torch.cuda.synchronize()
    om = P.omega(n, k, "gaussian", 5, dtype=dtype)
    bF, _ = pass_bound(X64, om, dtype)
    assert np.all(np.abs(F1.cpu().numpy() - F3.cpu().numpy()) <= 2 * bF)


def test_strided_rows(gpu_lib):
    """ldx > n: X is a column slice of a wider matrix."""
    import torch
    m, n, k = 700, 130, 12
    Xs, X64 = _data(m, n + 7, k, "f64")
    X = to_device(Xs, "f64")[:, :n]
    assert X.stride(0) == n + 7
    V, s = gpu_lib.fit(X, k, "gaussian", 3)
    ref = O.lazy_fit(X64[:, :n], P.omega(n, k, "gaussian", 3), k)
    assert O.principal_sines(ref["V"], V.cpu().numpy()).max() < 1e-10
    assert np.allclose(s.cpu().numpy(), ref["sigma"], rtol=1e-10)


# --------------------------------------------------------------------- fit --

@pytest.mark.parametrize("m,n,k,dtype", PASS_CASES)
def test_fit_matches_oracle(gpu_lib, m, n, k, dtype):
    Xs, X64 = _data(m, n, k, dtype)
    om = P.omega(n, k, "gaussian", 21, dtype=dtype)
    V, s, sx = gpu_lib.fit(to_device(Xs, dtype), k, "gaussian", 21, want_sigma_x=True)
    V, s, sx = V.cpu().numpy(), s.cpu().numpy(), sx.cpu().numpy()
    ref = O.lazy_fit(X64, om, k)
    sp = O.spca_fit(X64, om, k)
    # orthonormal columns (the Jacobi stage stops at cosines <= 8 k u),
    # canonical order
    assert np.max(np.abs(V.T @ V - np.eye(k))) < 16 * max(k, 16) * U64
    assert np.all(np.diff(s) <= 0)
    if dtype == "f64":
        tol_s = tol_v = 1e-10
    else:
        bF, _ = pass_bound(X64, om, dtype)
        err = np.linalg.norm(bF)
        tol_s = err / ref["sigma"][-1] + 1e-12
        tol_v = subspace_tol(ref["sigma"][-1], err) + 1e-12
    assert np.max(np.abs(s - ref["sigma"]) / ref["sigma"]) <= max(tol_s, 1e-13)
    assert O.principal_sines(ref["V"], V).max() <= tol_v
    # Proposition 2 across implementations: the GPU Lazy basis spans the
    # oracle's SPCA subspace; sigma_x matches the oracle's Sigma^s
    assert O.principal_sines(sp["V"], V).max() <= max(tol_v, 1e-10)
    rel_sx = np.max(np.abs(sx - sp["sigma"]) / sp["sigma"])
    assert rel_sx <= (1e-10 if dtype == "f64" else 20 * tol_s), rel_sx


def test_fit_full_first_config_f64(gpu_lib):
    """20,000 x 1,000 FP64, sigma_i = 1/i (i <= 50), noise 0.01, Gaussian
    Omega, k = 50: every output within 1e-10 relative of the oracle."""
    from synth import config
    c = config(1)
    Xs = lowrank_np(c["m"], c["n"], c["r"], c["spectrum"], c["s"], c["data_seed"], "f64")
    V, s, sx = gpu_lib.fit(to_device(Xs, "f64"), c["k"], "gaussian", c["omega_seed"], want_sigma_x=True)
    V, s, sx = V.cpu().numpy(), s.cpu().numpy(), sx.cpu().numpy()
    om = P.omega(c["n"], c["k"], "gaussian", c["omega_seed"])
    ref = O.lazy_fit(Xs, om, c["k"])
    sp = O.spca_fit(Xs, om, c["k"])
    assert O.principal_sines(ref["V"], V).max() < 1e-10
    assert np.max(np.abs(s - ref["sigma"]) / ref["sigma"]) < 1e-10
    assert np.max(np.abs(sx - sp["sigma"]) / sp["sigma"]) < 1e-10
    # individual columns where the spectrum separates them
    gaps = np.minimum(np.r_[np.inf, -np.diff(ref["sigma"])], np.r_[-np.diff(ref["sigma"]), np.inf])
    sep = gaps > 1e-3 * ref["sigma"][0]
    assert np.max(np.abs(V[:, sep] - ref["V"][:, sep])) < 1e-10
    # Proposition 3 across implementations: pairwise distances
    rng = np.random.default_rng(0)
    pairs = rng.integers(0, c["m"], size=(2000, 2))
    dg = O.pairwise_distances(Xs @ V, pairs)
    ds = O.pairwise_distances(Xs @ sp["V"], pairs)
    assert np.max(np.abs(dg - ds) / np.maximum(ds, 1e-300)) < 1e-10


def test_fit_is_deterministic(gpu_lib):
    Xs, _ = _data(3001, 516, 64, "f32")
    X = to_device(Xs, "f32")
    V1, s1 = gpu_lib.fit(X, 64, "gaussian", 8)
    V2, s2 = gpu_lib.fit(X, 64, "gaussian", 8)
    assert np.array_equal(V1.cpu().numpy(), V2.cpu().numpy())
    assert np.array_equal(s1.cpu().numpy(), s2.cpu().numpy())


def test_rank_deficient_X_gives_erank(gpu_lib):
    """The sketch of a rank-3 X cannot have rank k = 6 (footnote to
    Corollary 1: U = X Omega is full rank only when rank(X) >= l)."""
    import torch
    Xs = lowrank_np(500, 40, 3, "inv", 0.0, 4, "f64")
    with pytest.raises(gpu_lib.LspcaError) as e:
        gpu_lib.fit(to_device(Xs, "f64"), 6, "gaussian", 1)
    assert e.value.name == "LSPCA_ERANK"
    torch.cuda.synchronize()


# ------------------------------------------------------------ small stage --

@pytest.mark.parametrize("k,n,spectrum", [(1, 9, "graded"), (7, 40, "graded"), (50, 1000, "graded"),
                                          (128, 1500, "graded"), (130, 700, "graded"),
                                          (256, 4096, "graded"), (300, 700, "graded"),
                                          (520, 1100, "graded"), (50, 1000, "flat"), (128, 1500, "flat"),
                                          (256, 4096, "flat"), (520, 1100, "flat")])
def test_factor_matches_oracle_svd(gpu_lib, k, n, spectrum):
    """Truncated SVD of a generated F = U diag(d) W^T with known, separated
    singular values, graded (condition 1e3: the preconditioned Jacobi) or
    flat (1.65 down to 1: Jacobi on R directly): V columns and D to 1e-10."""
    import torch
    rng = np.random.default_rng(k)
    Uf = random_orthonormal_np(k, k, rng)
    W = random_orthonormal_np(n, k, rng)
    if k == 1:
        d = np.array([3.0])
    else:
        d = np.geomspace(1e3, 1.0, k) if spectrum == "graded" else np.linspace(1.65, 1.0, k)
    F = (Uf * d) @ W.T
    V, s = gpu_lib.factor(torch.from_numpy(F).cuda())
    V, s = V.cpu().numpy(), s.cpu().numpy()
    Vr, dr = O.truncated_svd(F, k)
    assert np.max(np.abs(s - dr) / dr) < 1e-12
    assert np.max(np.abs(V - Vr)) < 1e-10
    assert np.max(np.abs(V.T @ V - np.eye(k))) < 16 * max(k, 16) * U64


@pytest.mark.parametrize("k,n", [(128, 2048), (256, 4096), (300, 700), (520, 1100)])
def test_factor_jacobi_cooperative_and_per_round_launches_agree(gpu_lib, monkeypatch, k, n):
    """The block Jacobi of k >= 128 runs all sweeps in one cooperative launch;
    LSPCA_JACOBI=launches runs the same rounds as separate launches: the
    same rotations in the same order, so the same bits."""
    import torch
    rng = np.random.default_rng(k + 1)
    F = (random_orthonormal_np(k, k, rng) * np.geomspace(30.0, 1.0, k)) @ random_orthonormal_np(n, k, rng).T
    Ft = torch.from_numpy(F).cuda()
    V1, s1 = gpu_lib.factor(Ft)
    monkeypatch.setenv("LSPCA_JACOBI", "launches")
    V2, s2 = gpu_lib.factor(Ft)
    monkeypatch.delenv("LSPCA_JACOBI")
    assert torch.equal(V1, V2) and torch.equal(s1, s2)
    Vr, dr = O.truncated_svd(F, k)
    assert np.max(np.abs(s1.cpu().numpy() - dr) / dr) < 1e-12


@pytest.mark.parametrize("k,n,top,knob", [(64, 1000, 1e3, None), (256, 4096, 30.0, None),
                                          (256, 2048, 1e6, None), (200, 700, 30.0, "launches")])
def test_jacobi_early_stop_gives_the_same_bits(gpu_lib, monkeypatch, k, n, top, knob):
    """The Jacobi stops after a sweep whose rotated pairs were all within
    1e-8 of orthogonal: the sweep it skips would only have confirmed
    convergence, so V and the singular values are the same bits as with the
    early stop turned off (LSPCA_JACOBI_EARLY=0), for the one-workgroup
    kernel, the cooperative block kernel and the per-round launches."""
    import torch
    rng = np.random.default_rng(k + 7)
    F = (random_orthonormal_np(k, k, rng) * np.geomspace(top, 1.0, k)) @ random_orthonormal_np(n, k, rng).T
    Ft = torch.from_numpy(F).cuda()
    if knob:
        monkeypatch.setenv("LSPCA_JACOBI", knob)
    V1, s1 = gpu_lib.factor(Ft)
    monkeypatch.setenv("LSPCA_JACOBI_EARLY", "0")
    V2, s2 = gpu_lib.factor(Ft)
    assert torch.equal(V1, V2) and torch.equal(s1, s2)
    # against the oracle: the QR of F^T costs relative accuracy in proportion
    # to the condition number (about 4e-12 at 1e6)
    Vr, dr = O.truncated_svd(F, k)
    assert np.max(np.abs(s1.cpu().numpy() - dr) / dr) < 1e-12 * max(1.0, top / 1e3)


@pytest.mark.parametrize("k,n", [(7, 40), (50, 1000), (130, 700), (256, 4096)])
def test_factor_eigenvalue_route_matches_oracle_svd(gpu_lib, k, n):
    """small_route = eig (F F^T = W Lambda W^T, D = Lambda^(1/2), V = F^T W
    D^-1, then a Cholesky QR pass): squaring the problem costs a factor
    kappa(F) against the default route, so D and span(V) agree with the
    oracle's SVD to c u kappa^2 (condition 30 here)."""
    import torch
    rng = np.random.default_rng(k + 7)
    d = np.geomspace(30.0, 1.0, k)
    F = (random_orthonormal_np(k, k, rng) * d) @ random_orthonormal_np(n, k, rng).T
    V, s = gpu_lib.factor(torch.from_numpy(F).cuda(), small_route="eig")
    V, s = V.cpu().numpy(), s.cpu().numpy()
    Vr, dr = O.truncated_svd(F, k)
    tol = 64 * k * U64 * (dr[0] / dr[-1]) ** 2
    assert np.max(np.abs(s - dr) / dr) < tol
    assert O.principal_sines(Vr, V).max() < tol
    assert np.max(np.abs(V.T @ V - np.eye(k))) < 16 * max(k, 16) * U64
    # the oracle's own eigenvalue route agrees as well
    Ve, de = O.eig_route_svd(F, k)
    assert np.max(np.abs(s - de) / de) < tol


def test_fit_eigenvalue_route_and_stripe_rows(gpu_lib):
    """lspca_fit with small_route = eig, and with caller-chosen stripes
    (stripe_rows), against the default fit on the same X."""
    import torch
    m, n, k = 5003, 300, 20
    Xs, X64 = _data(m, n, k, "f64")
    X = to_device(Xs, "f64")
    V0, s0 = gpu_lib.fit(X, k, "gaussian", 4)
    V1, s1 = gpu_lib.fit(X, k, "gaussian", 4, small_route="eig")
    V2, s2 = gpu_lib.fit(X, k, "gaussian", 4, stripe_rows=1000)
    V0, s0 = V0.cpu().numpy(), s0.cpu().numpy()
    kappa = s0[0] / s0[-1]
    assert O.principal_sines(V0, V1.cpu().numpy()).max() < 64 * k * U64 * kappa ** 2
    assert np.max(np.abs(s1.cpu().numpy() - s0) / s0) < 64 * k * U64 * kappa ** 2
    # stripes change only the FP64 summation order of F
    assert O.principal_sines(V0, V2.cpu().numpy()).max() < 1e-10
    assert np.max(np.abs(s2.cpu().numpy() - s0) / s0) < 1e-12


def test_factor_ill_conditioned_uses_shifted_path(gpu_lib):
    """Condition 1e9: the first Cholesky of F F^T fails in FP64, the shifted
    pass takes over. Any backward-stable SVD (the oracle's LAPACK one too)
    fixes the row space of F only to about c u kappa(F) (Wedin with a
    backward error c u ||F||), so the two agree to 64 u kappa = 7e-6."""
    import torch
    k, n = 12, 300
    rng = np.random.default_rng(3)
    F = (random_orthonormal_np(k, k, rng) * np.geomspace(1e9, 1.0, k)) @ random_orthonormal_np(n, k, rng).T
    V, s = gpu_lib.factor(torch.from_numpy(F).cuda())
    Vr, dr = O.truncated_svd(F, k)
    s = s.cpu().numpy()
    kappa = dr[0] / dr[-1]
    assert np.max(np.abs(s - dr) / dr) < 64 * U64 * kappa
    assert O.principal_sines(Vr, V.cpu().numpy()).max() < 64 * U64 * kappa


# -------------------------------------------------------------- transform --

@pytest.mark.parametrize("r,n,k,dtype", [(1, 50, 5, "f64"), (777, 203, 17, "f64"),
                                         (777, 203, 17, "f32"), (4099, 512, 64, "f32"),
                                         (777, 203, 17, "bf16"), (4099, 512, 256, "bf16"),
                                         (777, 203, 17, "f16"), (1025, 512, 128, "f16")])
def test_transform_matches_oracle(gpu_lib, r, n, k, dtype):
    Xs, X64 = _data(r, n, min(k, r), dtype, seed=2)
    V = random_orthonormal_np(n, k, np.random.default_rng(1))
    import torch
    Z = gpu_lib.transform(to_device(Xs, dtype), torch.from_numpy(V).cuda())
    Z = Z.double().cpu().numpy()
    Vq = V if dtype != "f32" else P.round_f32(V)
    ref = O.transform(X64, Vq)
    u = U64 if dtype == "f64" else U32
    bound = (n * u / (1 - n * u)) * (np.abs(X64) @ np.abs(Vq))
    if dtype in ("bf16", "f16"):
        # V = V_hi + V_lo in 16-bit parts: |V - V_hi - V_lo| <= u16^2 |V|,
        # plus V rounded to FP32 first (u32), plus the second product's sum
        u16 = 2.0 ** -8 if dtype == "bf16" else 2.0 ** -11
        bound = 2 * bound + (1.01 * u16 ** 2 + U32 + 2.0 ** -24) * (np.abs(X64) @ np.abs(V))
    assert np.all(np.abs(Z - ref) <= bound + 1e-300)
    if dtype == "f64":
        assert np.linalg.norm(Z - O.transform(X64, V)) <= 1e-10 * np.linalg.norm(O.transform(X64, V))


def test_transform_rows_are_independent(gpu_lib):
    """A row's projection is bitwise the same alone, in a batch, or at any
    offset: fixed per-row reduction order."""
    import torch
    Xs, _ = _data(1500, 300, 20, "f32", seed=9)
    X = to_device(Xs, "f32")
    V = torch.from_numpy(random_orthonormal_np(300, 20, np.random.default_rng(2))).cuda()
    Zall = gpu_lib.transform(X, V).cpu().numpy()
    for r0, r1 in [(0, 1), (17, 18), (100, 357), (1499, 1500)]:
        Zp = gpu_lib.transform(X[r0:r1], V).cpu().numpy()
        assert np.array_equal(Zp, Zall[r0:r1])


@pytest.mark.parametrize("dtype,n,k", [("bf16", 4096, 256), ("f16", 2048, 128), ("bf16", 203, 17),
                                       ("f16", 520, 100)])
def test_transform_small_and_standard_tiles_agree_bitwise(gpu_lib, monkeypatch, dtype, n, k):
    """16-bit projections of few rows take 32 x 64 tiles; every tile shape
    runs the same chain of matrix-core steps per output element, so the
    rows are bitwise those of the standard tiles (n = 203: element loads)."""
    import torch
    Xs, _ = _data(5000, n, min(k, 16), dtype, seed=4)
    X = to_device(Xs, dtype)
    V = torch.from_numpy(random_orthonormal_np(n, k, np.random.default_rng(3))).cuda()
    for r in (1, 31, 33, 300, 4096, 5000):
        monkeypatch.setenv("LSPCA_PROJ_SMALL_ROWS", "0")           # standard tiles only
        Zb = gpu_lib.transform(X[:r], V)
        monkeypatch.setenv("LSPCA_PROJ_SMALL_ROWS", "1000000")     # small tiles only
        Zs = gpu_lib.transform(X[:r], V)
        monkeypatch.delenv("LSPCA_PROJ_SMALL_ROWS")
        Zd = gpu_lib.transform(X[:r], V)                           # the default choice
        torch.cuda.synchronize()
        assert torch.equal(Zs, Zb), (dtype, n, k, r)
        assert torch.equal(Zd, Zb), (dtype, n, k, r)


# --------------------------------------------------------------- 16-bit --

@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_refinement_shrinks_the_factor_error(gpu_lib, dtype):
    """One refinement pass (F = Y_hi^T X + Y_lo^T X, X read once) against
    Y_hi alone: both within their bound, the refined error far smaller."""
    import torch
    m, n, k = 4000, 384, 48
    Xs, X64 = _data(m, n, k, dtype)
    om = P.omega(n, k, "gaussian", 31, dtype=dtype)
    ref = O.streaming_lazy_fit(X64, om, k)["F"]
    errs = {}
    for refine in (1, 0):
        F = torch.zeros((k, n), dtype=torch.float64, device="cuda")
        gpu_lib.accumulate(to_device(Xs, dtype), k, "gaussian", 31, F, refine=refine)
        torch.cuda.synchronize()
        e = np.abs(F.cpu().numpy() - ref)
        bF, _ = pass_bound(X64, om, dtype, refine=bool(refine))
        assert np.all(e <= bF), (refine, float(np.max(e / bF)))
        errs[refine] = np.linalg.norm(e) / np.linalg.norm(ref)
    # BF16 (u16 = 2^-8): refinement removes the split error, which dominates;
    # FP16 (u16 = 2^-11): the unrefined split error is closer to the FP32
    # accumulation floor that remains after refinement
    assert errs[1] < errs[0] / (20 if dtype == "bf16" else 4), errs


@pytest.mark.parametrize("dtype", ["bf16", "f16"])
def test_sparse_omega_fit_16bit(gpu_lib, dtype):
    """Very sparse Omega (p = 64) with 16-bit data and refinement: the max
    principal-angle sine against the FP64 oracle stays far below 1e-3."""
    m, n, k = 6000, 1024, 64
    Xs, X64 = _data(m, n, k, dtype)
    V, s = gpu_lib.fit(to_device(Xs, dtype), k, "sparse", 77, sparse_p=64)
    om = P.omega(n, k, "sparse", 77, p=64, dtype=dtype)
    ref = O.lazy_fit(X64, om, k)
    sine = O.principal_sines(ref["V"], V.cpu().numpy()).max()
    bF, _ = pass_bound(X64, om, dtype)
    err = np.linalg.norm(bF)
    assert sine <= subspace_tol(ref["sigma"][-1], err) + 1e-12
    assert sine < 1e-3
    assert np.max(np.abs(s.cpu().numpy() - ref["sigma"]) / ref["sigma"]) <= err / ref["sigma"][-1] + 1e-12


# (dtype, p, m, n, k, kernel): kernel "reg" requires the register-list kernel
# (lanes per column 16, 8, 4 for k <= 64, <= 128, <= 256; n <= 4096), "lds"
# selects the LDS-list kernel, None leaves the choice to the shape (p = 1:
# dense lists and n > 4096 take the LDS-list kernel)
SPARSE_CASES = [("bf16", 64, 2001, 517, 40, "reg"), ("f16", 64, 2001, 517, 40, "reg"),
                ("bf16", 1, 2001, 517, 40, None), ("bf16", 8, 2001, 517, 40, "reg"),
                ("f16", 16, 1999, 1000, 100, "reg"), ("bf16", 64, 3001, 4096, 256, "reg"),
                ("f16", 64, 1003, 4096, 256, "reg"), ("bf16", 64, 2001, 517, 40, "lds"),
                ("bf16", 32, 1500, 5000, 64, None), ("bf16", 64, 1007, 4096, 256, "lds")]


@pytest.mark.parametrize("dtype,p,m,n,k,kernel", SPARSE_CASES)
def test_sparse_sketch_accumulate_matches_oracle(gpu_lib, monkeypatch, dtype, p, m, n, k, kernel):
    """Gather-add sketch (Omega regenerated per workgroup, never stored):
    F and G within the componentwise bound of the oracle's, on ragged
    sizes (m not a multiple of the 8- or 4-row tile, n not of 8)."""
    import torch
    if kernel:
        monkeypatch.setenv("LSPCA_SPARSE_KERNEL", kernel)
    Xs, X64 = _data(m, n, min(k, 64), dtype)
    om = P.omega(n, k, "sparse", 1234, p=p, dtype=dtype)
    F = torch.zeros((k, n), dtype=torch.float64, device="cuda")
    G = torch.zeros((k, k), dtype=torch.float64, device="cuda")
    gpu_lib.accumulate(to_device(Xs, dtype), k, "sparse", 1234, F, G, sparse_p=p)
    torch.cuda.synchronize()
    ref = O.streaming_lazy_fit(X64, om, k)
    bF, bG = pass_bound(X64, om, dtype)
    assert np.all(np.abs(F.cpu().numpy() - ref["F"]) <= bF)
    assert np.all(np.abs(G.cpu().numpy() - ref["G"]) <= bG)


@pytest.mark.parametrize("kernel,env,m,n,k,p", [("reg", {"LSPCA_SPARSE_LQ": "1"}, 1500, 300, 32, 4),
                                                ("reg", {"LSPCA_SPARSE_LQ": "2"}, 1203, 777, 200, 16),
                                                ("reg", {"LSPCA_SPARSE_LQ": "3"}, 999, 640, 90, 8),
                                                ("lds", {"LSPCA_SPARSE_KERNEL": "lds", "LSPCA_SPARSE_CAP": "64"},
                                                 1500, 300, 32, 4)])
def test_sparse_sketch_fallback_gives_the_same_bits(gpu_lib, monkeypatch, kernel, env, m, n, k, p):
    """A list capacity below the number of nonzeros (forced from the host)
    switches the workgroups to on-the-fly regeneration: same summation
    order, so the same F bit for bit."""
    import torch
    Xs, _ = _data(m, n, min(k, 32), "bf16")
    X = to_device(Xs, "bf16")
    monkeypatch.setenv("LSPCA_SPARSE_KERNEL", kernel)
    F1 = torch.zeros((k, n), dtype=torch.float64, device="cuda")
    gpu_lib.accumulate(X, k, "sparse", 9, F1, sparse_p=p)
    torch.cuda.synchronize()
    for key, val in env.items():
        monkeypatch.setenv(key, val)
    F2 = torch.zeros((k, n), dtype=torch.float64, device="cuda")
    gpu_lib.accumulate(X, k, "sparse", 9, F2, sparse_p=p)
    torch.cuda.synchronize()
    for key in env:
        monkeypatch.delenv(key)
    assert np.array_equal(F1.cpu().numpy(), F2.cpu().numpy())


@pytest.mark.parametrize("dtype,kind,m,n,k,refine", [("bf16", "sparse", 3001, 520, 136, 1),
                                                     ("bf16", "sparse", 4099, 1024, 256, 0),
                                                     ("f16", "sparse", 777, 1032, 128, 1),
                                                     ("f16", "gaussian", 2050, 512, 64, 1),
                                                     ("bf16", "gaussian", 65, 264, 200, 1),
                                                     ("bf16", "sparse", 20000, 776, 24, 1)])
def test_direct_and_staged_F_products_agree_bitwise(gpu_lib, monkeypatch, dtype, kind, m, n, k, refine):
    """F = Y^T X from operands copied straight into LDS (the default) and from
    register-staged tiles (LSPCA_TN16_DIRECT=0): the same MFMA chain per
    element of F, so the same bits, also over ragged row chunks."""
    import torch
    Xs, _ = _data(m, n, min(k, 32), dtype)
    X = to_device(Xs, dtype)
    out = []
    for env in ("0", "1"):
        monkeypatch.setenv("LSPCA_TN16_DIRECT", env)
        F = torch.zeros((k, n), dtype=torch.float64, device="cuda")
        G = torch.zeros((k, k), dtype=torch.float64, device="cuda")
        gpu_lib.accumulate(X, k, kind, 21, F, G, sparse_p=64 if kind == "sparse" else 0, refine=refine)
        torch.cuda.synchronize()
        out.append((F.cpu().numpy(), G.cpu().numpy()))
    monkeypatch.delenv("LSPCA_TN16_DIRECT")
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
    assert np.all(np.isfinite(out[1][0])) and np.abs(out[1][0]).max() > 0


@pytest.mark.parametrize("dtype,m,n,k", [("f16", 3001, 512, 64), ("bf16", 4099, 1024, 128),
                                         ("bf16", 2050, 2048, 256), ("f16", 777, 512, 100),
                                         ("f16", 20000, 2048, 128), ("bf16", 300, 64, 8)])
def test_direct_and_staged_sketch_agree_bitwise(gpu_lib, monkeypatch, dtype, m, n, k):
    """The dense 16-bit sketch Y = X Omega by persistent workgroups with
    operands copied straight into LDS (the default) and by register-staged
    tiles (LSPCA_NT16_DIRECT=0): the same MFMA chain per element of Y, so F
    and G agree bit for bit (FP16: also the column scales from max |Y|)."""
    import torch
    Xs, _ = _data(m, n, min(k, 32), dtype)
    X = to_device(Xs, dtype)
    out = []
    for env in ("0", "1"):
        monkeypatch.setenv("LSPCA_NT16_DIRECT", env)
        F = torch.zeros((k, n), dtype=torch.float64, device="cuda")
        G = torch.zeros((k, k), dtype=torch.float64, device="cuda")
        gpu_lib.accumulate(X, k, "gaussian", 23, F, G, refine=1)
        torch.cuda.synchronize()
        out.append((F.cpu().numpy(), G.cpu().numpy()))
    monkeypatch.delenv("LSPCA_NT16_DIRECT")
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
    assert np.all(np.isfinite(out[1][0])) and np.abs(out[1][0]).max() > 0


@pytest.mark.parametrize("m,n,k", [(5003, 512, 100), (4500, 256, 200), (9000, 1024, 256)])
def test_streamed_and_tiled_fp32_sketch_and_projection_agree_bitwise(gpu_lib, monkeypatch, m, n, k):
    """The FP32 sketch and projection of a tall X by the streamed kernel (the
    default) and by the tiled k_nt (LSPCA_NT32_STREAM=0) sum the products of
    each output element in the same order: F, G and Z agree bit for bit, and
    F and G are within the oracle's bound."""
    import torch
    Xs, X64 = _data(m, n, min(k, 32), "f32")
    X = to_device(Xs, "f32")
    om = P.omega(n, k, "gaussian", 17, dtype="f32")
    ref = O.streaming_lazy_fit(X64, om, k)
    bF, bG = pass_bound(X64, om, "f32")
    V = torch.from_numpy(random_orthonormal_np(n, k, np.random.default_rng(8))).cuda()
    got = []
    for env in ("0", "1"):
        monkeypatch.setenv("LSPCA_NT32_STREAM", env)
        F = torch.zeros((k, n), dtype=torch.float64, device="cuda")
        G = torch.zeros((k, k), dtype=torch.float64, device="cuda")
        gpu_lib.accumulate(X, k, "gaussian", 17, F, G)
        Z = gpu_lib.transform(X, V)
        torch.cuda.synchronize()
        got.append((F.cpu().numpy(), G.cpu().numpy(), Z.cpu().numpy()))
    monkeypatch.delenv("LSPCA_NT32_STREAM")
    for a, b in zip(got[0], got[1]):
        assert np.array_equal(a, b)
    F, G, _ = got[1]
    assert np.all(np.abs(F - ref["F"]) <= bF), float(np.max(np.abs(F - ref["F"]) / bF))
    assert np.all(np.abs(G - ref["G"]) <= bG), float(np.max(np.abs(G - ref["G"]) / bG))


@pytest.mark.parametrize("m,n,k", [(5000, 4096, 256), (4099, 1024, 100), (70001, 512, 128), (777, 260, 12),
                                   (3, 64, 8), (10000, 2048, 300)])
def test_streamed_and_tiled_fp32_F_agree_bitwise(gpu_lib, monkeypatch, m, n, k):
    """F = Y^T X in FP32 from rows copied straight into LDS (the default) and
    from k_tn's register-staged tiles (LSPCA_TN32_STREAM=0): the same chunks
    and the same MFMA chain per element, so the same bits (F and G, which
    comes from F in the small stage's inputs only through the pass)."""
    import torch
    Xs, _ = _data(m, n, min(k, 32), "f32")
    X = to_device(Xs, "f32")
    out = []
    for env in ("0", "1"):
        monkeypatch.setenv("LSPCA_TN32_STREAM", env)
        F = torch.zeros((k, n), dtype=torch.float64, device="cuda")
        G = torch.zeros((k, k), dtype=torch.float64, device="cuda")
        gpu_lib.accumulate(X, k, "gaussian", 29, F, G)
        torch.cuda.synchronize()
        out.append((F.cpu().numpy(), G.cpu().numpy()))
    monkeypatch.delenv("LSPCA_TN32_STREAM")
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1])
    assert np.all(np.isfinite(out[1][0])) and np.abs(out[1][0]).max() > 0


@pytest.mark.parametrize("k,knob", [(40, None), (127, None), (128, None), (200, None), (200, "launches")])
def test_jacobi_sweep_limit_is_reported(gpu_lib, monkeypatch, k, knob):
    """A one-sided Jacobi run that reaches its sweep limit while its last
    sweep still rotated a pair further than 1e-8 from orthogonal is an error
    (LSPCA_ENOCONV), never a silent result.
    The limit is forced down to one sweep with the library's test knob; the
    single-workgroup kernel (k < 128), the cooperative block kernel and the
    per-round launches are each covered."""
    import torch
    rng = np.random.default_rng(k)
    F = torch.from_numpy(rng.standard_normal((k, 2 * k))).cuda()
    if knob:
        monkeypatch.setenv("LSPCA_JACOBI", knob)
    monkeypatch.setenv("LSPCA_JACOBI_SWEEPS", "1")
    with pytest.raises(gpu_lib.LspcaError) as e:
        gpu_lib.factor(F)
    assert e.value.name == "LSPCA_ENOCONV"
    monkeypatch.delenv("LSPCA_JACOBI_SWEEPS")
    V, s = gpu_lib.factor(F)
    Vr, dr = O.truncated_svd(F.cpu().numpy(), k)
    assert np.max(np.abs(s.cpu().numpy() - dr) / dr) < 1e-10
