"""GPU-vs-oracle parity of the sparse-X (CSR) path through the C ABI: the
pass (F, G), the fit, the projection, the stripe and slice forms, the
device-side input checks, and the workload at full size on sampled outputs.

The oracle's X is the dense matrix the CSR triple stands for
(oracle.csr_dense), or at full size the sparse products of
oracle.csr_factor_rows. Error model as tests/helpers.py: the sketch row i
sums nnz_i <= n products in the value type, F sums in FP64."""
import time

import numpy as np
import pytest

from oracle import lspca_oracle as O
from oracle import philox as P
from synth import CSR_CONFIG, csr_np, csr_torch
from tests.helpers import U32, U64, UNIT, gamma, pass_bound, subspace_tol

pytestmark = pytest.mark.gpu


def _log(msg):
    print(f"[csr] {time.strftime('%H:%M:%S')} {msg}", flush=True)


def _dev_csr(gpu_lib, rowptr, colidx, values, n):
    import torch
    return gpu_lib.CSR(torch.from_numpy(rowptr).cuda(), torch.from_numpy(colidx).cuda(),
                       torch.from_numpy(values).cuda(), n)


def _csr_from_dense(X, dtype):
    r, c = np.nonzero(X)
    rowptr = np.zeros(X.shape[0] + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum(np.bincount(r, minlength=X.shape[0]))
    vdt = np.float32 if dtype == "f32" else np.float64
    return rowptr, c.astype(np.int32), X[r, c].astype(vdt)


# (m, n, k, dtype, kind, density): ragged sizes; k = 1; k above 256 (two
# column passes); very low density (many empty rows)
CASES = [
    (1037, 203, 17, "f64", "gaussian", 0.05),
    (3001, 516, 64, "f32", "gaussian", 0.03),
    (2000, 1000, 136, "f32", "sparse", 0.0244),
    (1500, 700, 300, "f64", "sparse", 0.05),
    (600, 2000, 1, "f32", "gaussian", 0.01),
    (2500, 203, 16, "f32", "gaussian", 0.002),
]


def _case(m, n, dtype, density, seed=5):
    rowptr, colidx, values = csr_np(m, n, density=density, seed=seed, dtype=dtype)
    return rowptr, colidx, values, O.csr_dense(rowptr, colidx, values, n)


@pytest.mark.parametrize("m,n,k,dtype,kind,density", CASES)
def test_accumulate_csr_matches_oracle_within_bound(gpu_lib, m, n, k, dtype, kind, density):
    import torch
    rowptr, colidx, values, X64 = _case(m, n, dtype, density)
    _log(f"accumulate m={m} n={n} k={k} {dtype} {kind} nnz={rowptr[-1]}")
    X = _dev_csr(gpu_lib, rowptr, colidx, values, n)
    F = torch.zeros((k, n), dtype=torch.float64, device="cuda")
    G = torch.zeros((k, k), dtype=torch.float64, device="cuda")
    gpu_lib.accumulate_csr(X, k, kind, 99, F, G)
    torch.cuda.synchronize()
    om = P.omega(n, k, kind, 99, p=64, dtype=dtype)
    ref = O.streaming_lazy_fit(X64, om, k)
    bF, bG = pass_bound(X64, om, dtype)
    eF = np.abs(F.cpu().numpy() - ref["F"])
    eG = np.abs(G.cpu().numpy() - ref["G"])
    assert np.all(eF <= bF), float(np.max(eF / bF))
    assert np.all(eG <= bG), float(np.max(eG / bG))


def test_heavy_and_empty_columns(gpu_lib):
    """A column present in every row (split into many segments), one in
    exactly 256 rows (one full segment), empty columns and empty rows."""
    import torch
    rng = np.random.default_rng(3)
    m, n, k = 3000, 300, 40
    X64 = np.where(rng.random((m, n)) < 0.02, rng.standard_normal((m, n)), 0.0)
    X64[100:400] = 0.0
    X64[:, 7] = rng.standard_normal(m)
    X64[:, 11] = 0.0
    X64[rng.choice(np.r_[0:100, 400:m], 256, replace=False), 11] = 1.5
    X64[:, 200:230] = 0.0
    for dtype in ("f64", "f32"):
        rowptr, colidx, values = _csr_from_dense(X64, dtype)
        Xd = O.csr_dense(rowptr, colidx, values, n)
        X = _dev_csr(gpu_lib, rowptr, colidx, values, n)
        F = torch.zeros((k, n), dtype=torch.float64, device="cuda")
        gpu_lib.accumulate_csr(X, k, "gaussian", 4, F)
        torch.cuda.synchronize()
        om = P.omega(n, k, "gaussian", 4, dtype=dtype)
        ref = O.lazy_factor(Xd, O.sketch(Xd, om))
        bF, _ = pass_bound(Xd, om, dtype)
        Fh = F.cpu().numpy()
        assert np.all(np.abs(Fh - ref) <= bF), dtype
        assert np.all(Fh[:, 200:230] == 0.0)


@pytest.mark.parametrize("how", ["nnz_cap", "stripe_rows", "slices"])
def test_stripes_and_row_slices(gpu_lib, monkeypatch, how):
    """Algorithm 4 over any split of the rows: several stripes inside one
    call (by an entry cap or by stripe_rows), or several calls on row
    slices of one CSR matrix (rowptr with a positive first entry)."""
    import torch
    m, n, k, dtype = 2999, 260, 24, "f32"
    rowptr, colidx, values, X64 = _case(m, n, dtype, 0.05, seed=8)
    X = _dev_csr(gpu_lib, rowptr, colidx, values, n)
    F = torch.zeros((k, n), dtype=torch.float64, device="cuda")
    G = torch.zeros((k, k), dtype=torch.float64, device="cuda")
    if how == "nnz_cap":
        monkeypatch.setenv("LSPCA_CSR_STRIPE_NNZ", "3000")     # ~ 4 blocks of 64 rows per stripe
        gpu_lib.accumulate_csr(X, k, "sparse", 5, F, G)
    elif how == "stripe_rows":
        gpu_lib.accumulate_csr(X, k, "sparse", 5, F, G, stripe_rows=333)
    else:
        for r0, r1 in [(0, 1000), (1000, 1001), (1001, 1700), (1700, m)]:
            gpu_lib.accumulate_csr(X.rows(r0, r1), k, "sparse", 5, F, G)
    torch.cuda.synchronize()
    om = P.omega(n, k, "sparse", 5, p=64, dtype=dtype)
    ref = O.streaming_lazy_fit(X64, om, k)
    bF, bG = pass_bound(X64, om, dtype)
    assert np.all(np.abs(F.cpu().numpy() - ref["F"]) <= bF)
    assert np.all(np.abs(G.cpu().numpy() - ref["G"]) <= bG)


@pytest.mark.parametrize("m,n,k,dtype,kind,density", CASES[:4])
def test_fit_csr_matches_oracle(gpu_lib, m, n, k, dtype, kind, density):
    rowptr, colidx, values, X64 = _case(m, n, dtype, density, seed=6)
    X = _dev_csr(gpu_lib, rowptr, colidx, values, n)
    V, s, sx = gpu_lib.fit_csr(X, k, kind, 21, want_sigma_x=True)
    V, s, sx = V.cpu().numpy(), s.cpu().numpy(), sx.cpu().numpy()
    om = P.omega(n, k, kind, 21, p=64, dtype=dtype)
    ref = O.lazy_fit(X64, om, k)
    sp = O.spca_fit(X64, om, k)
    assert np.max(np.abs(V.T @ V - np.eye(k))) < 16 * max(k, 16) * U64
    assert np.all(np.diff(s) <= 0)
    bF, _ = pass_bound(X64, om, dtype)
    err = np.linalg.norm(bF)
    tol_s = err / ref["sigma"][-1] + 1e-12
    tol_v = subspace_tol(ref["sigma"][-1], err) + 1e-12
    assert np.max(np.abs(s - ref["sigma"]) / ref["sigma"]) <= tol_s
    assert O.principal_sines(ref["V"], V).max() <= tol_v
    assert O.principal_sines(sp["V"], V).max() <= max(tol_v, 1e-10)
    assert np.max(np.abs(sx - sp["sigma"]) / sp["sigma"]) <= max(20 * tol_s, 1e-10)


def test_fit_csr_is_deterministic(gpu_lib):
    rowptr, colidx, values, _ = _case(2000, 400, "f32", 0.04, seed=2)
    X = _dev_csr(gpu_lib, rowptr, colidx, values, 400)
    V1, s1 = gpu_lib.fit_csr(X, 32, "gaussian", 3)
    V2, s2 = gpu_lib.fit_csr(X, 32, "gaussian", 3)
    assert bool((V1 == V2).all()) and bool((s1 == s2).all())


@pytest.mark.parametrize("dtype,k", [("f64", 17), ("f32", 64), ("f32", 300)])
def test_transform_csr_matches_oracle(gpu_lib, dtype, k):
    m, n = 1777, 640
    rowptr, colidx, values, X64 = _case(m, n, dtype, 0.03, seed=7)
    rng = np.random.default_rng(1)
    V64 = np.linalg.qr(rng.standard_normal((n, k)))[0]
    import torch
    X = _dev_csr(gpu_lib, rowptr, colidx, values, n)
    Z = gpu_lib.transform_csr(X, torch.from_numpy(V64).cuda()).double().cpu().numpy()
    Vq = P.round_f32(V64) if dtype == "f32" else V64            # V as the FP32 product uses it
    ref = O.transform(X64, Vq)
    nz = int(np.diff(rowptr).max())
    bound = gamma(nz, UNIT[dtype]) * (np.abs(X64) @ np.abs(Vq))
    assert np.all(np.abs(Z - ref) <= bound + 1e-300)
    # rows whose columns are not in order take the row-parallel path
    rng2 = np.random.default_rng(5)
    ci2, v2 = colidx.copy(), values.copy()
    for i in range(0, m, 3):
        p = rowptr[i] + rng2.permutation(rowptr[i + 1] - rowptr[i])
        ci2[rowptr[i]:rowptr[i + 1]], v2[rowptr[i]:rowptr[i + 1]] = colidx[p], values[p]
    Zu = gpu_lib.transform_csr(_dev_csr(gpu_lib, rowptr, ci2, v2, n),
                               torch.from_numpy(V64).cuda()).double().cpu().numpy()
    assert np.all(np.abs(Zu - ref) <= bound + 1e-300)
    # a row's result does not depend on the others (row slice)
    Z2 = gpu_lib.transform_csr(X.rows(500, 900), torch.from_numpy(V64).cuda()).double().cpu().numpy()
    assert np.array_equal(Z2, Z[500:900])


def test_empty_matrix_leaves_f_and_g_unchanged(gpu_lib):
    import torch
    m, n, k = 300, 50, 8
    X = gpu_lib.CSR(torch.zeros(m + 1, dtype=torch.int64, device="cuda"),
                    torch.zeros(0, dtype=torch.int32, device="cuda"),
                    torch.zeros(0, dtype=torch.float32, device="cuda"), n)
    F = torch.full((k, n), 2.0, dtype=torch.float64, device="cuda")
    G = torch.full((k, k), 3.0, dtype=torch.float64, device="cuda")
    gpu_lib.accumulate_csr(X, k, "gaussian", 1, F, G)
    torch.cuda.synchronize()
    assert bool((F == 2.0).all()) and bool((G == 3.0).all())


def test_bad_csr_arrays_are_rejected_on_the_device(gpu_lib):
    """rowptr and colidx are checked on the device before any kernel
    indexes with them; the error names the array."""
    import ctypes
    import torch
    lib = gpu_lib.load()
    m, n, k = 50, 40, 4
    rowptr, colidx, values, _ = _case(m, n, "f32", 0.1, seed=1)
    F = torch.zeros((k, n), dtype=torch.float64, device="cuda")
    o = gpu_lib._opts()

    def call(rp, ci, nnz):
        rp_d, ci_d = torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda()
        v_d = torch.from_numpy(values).cuda()
        st = lib.lspca_accumulate_csr(rp_d.data_ptr(), ci_d.data_ptr(), v_d.data_ptr(), gpu_lib.F32,
                                      m, n, nnz, k, gpu_lib.GAUSSIAN, 1, ctypes.byref(o), F.data_ptr(), None)
        return st, lib.lspca_last_error().decode()

    nnz = int(rowptr[-1])
    st, msg = call(rowptr, colidx, nnz)
    assert st == 0, msg
    bad = colidx.copy()
    bad[nnz // 2] = n
    st, msg = call(rowptr, bad, nnz)
    assert st == -1 and "colidx" in msg
    bad = colidx.copy()
    bad[3] = -1
    assert call(rowptr, bad, nnz)[0] == -1
    rp = rowptr.copy()
    rp[10], rp[11] = rp[11], rp[10] - 1                      # decreasing
    st, msg = call(rp, colidx, nnz)
    assert st == -1 and "rowptr" in msg
    st, msg = call(rowptr, colidx, nnz - 1)                    # rowptr[m] != nnz
    assert st == -1 and "rowptr" in msg


# ------------------------------------------------------------- full size --

@pytest.mark.slow
def test_full_size_sparse_workload_sampled(gpu_lib):
    """The sparse workload at full size (131,072 x 98,450 at density 0.0244,
    k = 500, very sparse Omega, FP32 values), one call as bench.py makes
    it: whole rows of F and a block of G for sampled sketch columns against
    the oracle's sparse products, with the componentwise bound evaluated for
    those entries; the small stage on the device's F against the oracle SVD;
    sampled rows of Z = X V."""
    import scipy.sparse as sp
    import torch
    c = CSR_CONFIG
    m, n, k = c["m"], c["n"], c["k"]
    _log(f"generating {m}x{n} CSR at density {c['density']}")
    rp, ci, vv = csr_torch(m, n, c["density"], c["data_seed"], c["alpha"], c["binary"], c["dtype"])
    X = gpu_lib.CSR(rp, ci, vv, n)
    _log(f"nnz = {X.nnz}; pass")
    F = torch.zeros((k, n), dtype=torch.float64, device="cuda")
    G = torch.zeros((k, k), dtype=torch.float64, device="cuda")
    gpu_lib.accumulate_csr(X, k, c["kind"], c["omega_seed"], F, G, sparse_p=c["p"])
    torch.cuda.synchronize()
    _log("copying to host")
    rph, cih, vvh = rp.cpu().numpy(), ci.cpu().numpy(), vv.cpu().numpy()
    cols = np.array([0, 1, 257, k - 1])
    om = P.omega(n, k, c["kind"], c["omega_seed"], p=c["p"], dtype=c["dtype"])
    _log("oracle sparse products")
    U, Fc = O.csr_factor_rows(rph, cih, vvh, n, om[:, cols])
    A = sp.csr_matrix((np.abs(vvh).astype(np.float64), cih, rph), shape=(m, n))
    aU = A @ np.abs(om[:, cols])                              # |X| |Omega_C|
    nz = int(np.diff(rph).max())
    u = UNIT[c["dtype"]]
    aY = np.abs(U) + gamma(nz, u) * aU
    bF = gamma(nz, u) * np.asarray((A.T @ aU).T) + gamma(m, U64) * np.asarray((A.T @ aY).T)
    Fd = F.cpu().numpy()
    eF = np.abs(Fd[cols] - Fc)
    assert np.all(eF <= bF), float(np.max(eF / bF))
    Gc = U.T @ U
    bG = 2 * gamma(nz, u) * (aU.T @ aY) + gamma(m, u) * (aY.T @ aY)
    eG = np.abs(G.cpu().numpy()[np.ix_(cols, cols)] - Gc)
    assert np.all(eG <= bG), float(np.max(eG / bG))
    _log("small stage against the oracle SVD of the device's F")
    V, s = gpu_lib.factor(F)
    Vr, sr = O.truncated_svd(Fd, k)
    kappa = sr[0] / sr[-1]
    tol = 64 * U64 * kappa * k
    assert np.max(np.abs(s.cpu().numpy() - sr) / sr) <= tol
    assert O.principal_sines(Vr, V.cpu().numpy()).max() <= tol
    _log("projection rows")
    Z = gpu_lib.transform_csr(X, V)
    rows = np.array([0, 1, 4097, m // 2, m - 1])
    Zh = Z[torch.from_numpy(rows).cuda()].double().cpu().numpy()
    Vq = P.round_f32(V.cpu().numpy())                           # V as the FP32 product uses it
    for t, i in enumerate(rows):
        Xi = O.csr_dense(rph[i:i + 2], cih, vvh, n)
        zr = O.transform(Xi, Vq)[0]
        bz = gamma(nz, U32) * (np.abs(Xi) @ np.abs(Vq))[0]
        assert np.all(np.abs(Zh[t] - zr) <= bz + 1e-300)
    _log("done")


@pytest.mark.parametrize("kind", ["gaussian", "sparse"])
def test_unordered_rows(gpu_lib, kind):
    """Rows whose columns are not in order: the Gaussian sketch takes the
    row-parallel kernel instead of the column blocks; same bound."""
    import torch
    m, n, k, dtype = 1500, 9000, 40, "f32"                   # two column blocks of 8,192 features
    rowptr, colidx, values, X64 = _case(m, n, dtype, 0.01, seed=12)
    rng = np.random.default_rng(2)
    ci2, v2 = colidx.copy(), values.copy()
    for i in range(0, m, 2):
        p = rowptr[i] + rng.permutation(rowptr[i + 1] - rowptr[i])
        ci2[rowptr[i]:rowptr[i + 1]], v2[rowptr[i]:rowptr[i + 1]] = colidx[p], values[p]
    om = P.omega(n, k, kind, 31, p=64, dtype=dtype)
    ref = O.streaming_lazy_fit(X64, om, k)
    bF, bG = pass_bound(X64, om, dtype)
    for ci, vv in ((colidx, values), (ci2, v2)):
        F = torch.zeros((k, n), dtype=torch.float64, device="cuda")
        G = torch.zeros((k, k), dtype=torch.float64, device="cuda")
        gpu_lib.accumulate_csr(_dev_csr(gpu_lib, rowptr, ci, vv, n), k, kind, 31, F, G)
        torch.cuda.synchronize()
        assert np.all(np.abs(F.cpu().numpy() - ref["F"]) <= bF)
        assert np.all(np.abs(G.cpu().numpy() - ref["G"]) <= bG)


# ------------------------------------------------------------- SPCA (Alg. 1) --

@pytest.mark.parametrize("m,n,k,kind", [(1037, 203, 17, "gaussian"), (129, 60, 7, "sparse"),
                                        (3 * 128 + 5, 400, 20, "sparse")])
def test_spca_fit_csr_f64_matches_oracle(gpu_lib, m, n, k, kind):
    rowptr, colidx, values, X64 = _case(m, n, "f64", 0.2, seed=13)
    V, s = gpu_lib.spca_fit_csr(_dev_csr(gpu_lib, rowptr, colidx, values, n), k, kind, 3)
    ref = O.spca_fit(X64, P.omega(n, k, kind, 3, p=64), k)
    assert O.principal_sines(ref["V"], V.cpu().numpy()).max() < 1e-10
    assert np.max(np.abs(s.cpu().numpy() - ref["sigma"]) / ref["sigma"]) < 1e-10


@pytest.mark.parametrize("m,n,k,kind,cap", [(2600, 512, 64, "sparse", 0), (1500, 9000, 40, "gaussian", 0),
                                            (2999, 260, 24, "sparse", 3000)])
def test_spca_fit_csr_f32_within_bound(gpu_lib, monkeypatch, m, n, k, kind, cap):
    """FP32 values; a Gaussian Omega over two column blocks; several stripes."""
    from tests.test_gpu_spca import _f_bound
    if cap:
        monkeypatch.setenv("LSPCA_CSR_STRIPE_NNZ", str(cap))
    rowptr, colidx, values, X64 = _case(m, n, "f32", 0.05 if n < 5000 else 0.01, seed=14)
    V, s = gpu_lib.spca_fit_csr(_dev_csr(gpu_lib, rowptr, colidx, values, n), k, kind, 11)
    ref = O.spca_fit(X64, P.omega(n, k, kind, 11, p=64, dtype="f32"), k)
    err = np.linalg.norm(_f_bound(X64, ref["Q"], k, "f32"))
    s = s.cpu().numpy()
    assert np.max(np.abs(s - ref["sigma"]) / ref["sigma"]) <= err / ref["sigma"][-1] + 1e-12
    assert O.principal_sines(ref["V"], V.cpu().numpy()).max() <= subspace_tol(ref["sigma"][-1], err) + 1e-12


def test_proposition_2_across_csr_fits(gpu_lib):
    """Prop. 2 on sparse X: the GPU SPCA and Lazy SPCA bases span the same
    subspace; Prop. 3: identical pairwise distances after projection."""
    m, n, k = 3000, 350, 24
    rowptr, colidx, values, _ = _case(m, n, "f64", 0.1, seed=15)
    X = _dev_csr(gpu_lib, rowptr, colidx, values, n)
    # Gaussian Omega: with n = 350 a very sparse Omega (p = 64) has an empty
    # column with a few per cent probability, and the Lazy fit then reports
    # ERANK (F has a zero row), as it should
    Vs, _ = gpu_lib.spca_fit_csr(X, k, "gaussian", 8)
    Vl, _ = gpu_lib.fit_csr(X, k, "gaussian", 8)
    assert O.principal_sines(Vs.cpu().numpy(), Vl.cpu().numpy()).max() < 1e-10
    Zs = gpu_lib.transform_csr(X, Vs).cpu().numpy()
    Zl = gpu_lib.transform_csr(X, Vl).cpu().numpy()
    pairs = np.random.default_rng(0).integers(0, m, size=(3000, 2))
    ds, dl = O.pairwise_distances(Zs, pairs), O.pairwise_distances(Zl, pairs)
    assert np.max(np.abs(ds - dl)) <= 1e-10 * np.max(ds)
