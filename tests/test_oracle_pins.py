"""Pins of the FP64 oracle to what the paper and the mathematics fix.

Nothing here compares the oracle with itself: each test checks it against a
published known-answer vector, a closed form, a proposition of the paper, an
exact special case, a theorem, or brute force on a tiny input.
"""
import math
import os

import numpy as np
import pytest

from oracle import lspca_oracle as O
from oracle import philox as P
from synth import lowrank_np, random_orthonormal_np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _noisy(m=400, n=60, r=12, s=0.05, seed=3):
    return lowrank_np(m, n, r, "invsqrt", s, seed, "f64")


def _orth(A):
    q, _ = np.linalg.qr(A)
    return q


# ---------------------------------------------------------------- generator --

def test_philox_known_answers():
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for row in rows:
        v = [int(x, 16) for x in row]
        out = P.philox4x32_10(np.array(v[:4]), np.array(v[4:6]))
        assert [int(x) for x in out] == v[6:10]


def test_gaussian_omega_is_standard_normal():
    """Sec. I-A: Gaussian RP takes Omega_ij iid N(0,1)."""
    om = P.gaussian_omega(2000, 64, seed=11)
    z = om.ravel()
    N = z.size
    assert abs(z.mean()) < 5 / math.sqrt(N)
    assert abs(z.var() - 1) < 5 * math.sqrt(2 / N)
    assert abs(np.mean(z ** 4) - 3) < 5 * math.sqrt(96 / N)
    # Kolmogorov-Smirnov distance to the N(0,1) CDF (critical value at 1e-4 ~ 2.1/sqrt(N))
    zs = np.sort(z)
    cdf = 0.5 * (1 + np.vectorize(math.erf)(zs / math.sqrt(2)))
    ks = max(np.max(np.arange(1, N + 1) / N - cdf), np.max(cdf - np.arange(N) / N))
    assert ks < 2.1 / math.sqrt(N)
    # neighbouring entries of one Box-Muller pair are uncorrelated
    assert abs(np.corrcoef(om[:, 0], om[:, 1])[0, 1]) < 5 / math.sqrt(om.shape[0])


def test_omega_is_a_function_of_seed_row_and_column():
    a = P.gaussian_omega(50, 9, seed=5)
    b = P.gaussian_omega(80, 16, seed=5)
    assert np.array_equal(a, b[:50, :9])                 # prefix-stable in n and k
    assert not np.array_equal(a, P.gaussian_omega(50, 9, seed=6))
    s1 = P.sparse_omega(70, 11, seed=5, p=4)
    s2 = P.sparse_omega(90, 20, seed=5, p=4)
    assert np.array_equal(s1, s2[:70, :11])
    big = (1 << 40) + 3                                  # both key words matter
    assert not np.array_equal(P.gaussian_omega(10, 4, big), P.gaussian_omega(10, 4, 3))


@pytest.mark.parametrize("p", [1, 2, 64])
def test_sparse_omega_probabilities(p):
    """Sec. I-A: entries {-1, 0, +1} with probabilities {1/(2p), 1-1/p, 1/(2p)}."""
    om = P.sparse_omega(4096, 256, seed=7, p=p)
    N = om.size
    assert set(np.unique(om)) <= {-1.0, 0.0, 1.0}
    for val, prob in [(1.0, 1 / (2 * p)), (-1.0, 1 / (2 * p)), (0.0, 1 - 1 / p)]:
        cnt = np.count_nonzero(om == val)
        sd = math.sqrt(N * prob * (1 - prob)) if 0 < prob < 1 else 0
        assert abs(cnt - N * prob) <= 5 * sd + 1e-9


def test_sparse_omega_rejects_bad_p():
    for p in (0, 3, 48, 2 ** 31):
        with pytest.raises(ValueError):
            P.sparse_omega(4, 4, 1, p)


def test_rounding_to_nearest_even():
    one = 1.0
    # BF16 has 8 significant bits: 1 + 2^-8 is a tie -> even (1.0); 1 + 3*2^-8 -> 1 + 2^-6
    assert P.round_bf16(np.array([one + 2 ** -8]))[0] == 1.0
    assert P.round_bf16(np.array([one + 3 * 2 ** -8]))[0] == 1 + 2 ** -6
    assert P.round_bf16(np.array([one + 2 ** -8 + 2 ** -20]))[0] == 1 + 2 ** -7
    assert P.round_bf16(np.array([-3.0]))[0] == -3.0
    # FP16 has 11 significant bits: 1 + 2^-11 is a tie -> 1.0
    assert P.round_f16(np.array([one + 2 ** -11]))[0] == 1.0
    assert P.round_f16(np.array([one + 3 * 2 ** -11]))[0] == 1 + 2 ** -9
    assert P.round_f32(np.array([one + 2 ** -24]))[0] == 1.0


# ------------------------------------------------------- exact special cases --

def test_exact_recovery_on_exactly_rank_k_X():
    """Sec. II-B eq. (subcover_approx): when the sketch spans im(X) the
    approximation is exact; then V spans the row space of X and Sigma^s are
    the singular values of X (known here by construction)."""
    rng = np.random.default_rng(1)
    m, n, k = 300, 40, 6
    A = random_orthonormal_np(m, k, rng)
    B = random_orthonormal_np(n, k, rng)
    sig = np.array([9.0, 5.0, 3.0, 2.0, 1.5, 0.7])
    X = (A * sig) @ B.T
    om = P.gaussian_omega(n, k, seed=2)
    lz = O.lazy_fit(X, om, k)
    sp = O.spca_fit(X, om, k)
    assert O.principal_sines(B, lz["V"]).max() < 1e-12
    assert O.principal_sines(B, sp["V"]).max() < 1e-12
    assert np.allclose(sp["sigma"], sig, rtol=1e-12, atol=0)
    Q = sp["Q"]
    assert np.linalg.norm(Q @ (Q.T @ X) - X) < 1e-12 * np.linalg.norm(X)
    # the exact SVD's right vectors are B's columns (distinct sigma): compare vectors
    Bc, _ = O.canonicalize(B, sig)
    assert np.max(np.abs(sp["V"] - Bc)) < 1e-11


def test_closed_form_diagonal_case():
    """X = [D; 0] with D diagonal (distinct, decreasing) and Omega = [I_k; 0]:
    U = X Omega, F = U^T X = [diag(d_1..d_k)^2, 0], so V = [I_k; 0], the Lazy
    singular values are d_i^2 and Sigma^s = d_i. Scaling Omega by c (eq. (rp))
    scales D by c and leaves V and Sigma^s unchanged."""
    n, k, m = 8, 3, 12
    d = np.array([5.0, 4.0, 3.0, 2.5, 2.0, 1.0, 0.5, 0.25])
    X = np.zeros((m, n))
    X[:n, :n] = np.diag(d)
    om = np.zeros((n, k))
    om[:k, :k] = np.eye(k)
    E = np.zeros((n, k))
    E[:k, :k] = np.eye(k)
    for c in (1.0, 3.0, 0.125):
        lz = O.lazy_fit(X, c * om, k)
        sp = O.spca_fit(X, c * om, k)
        assert np.allclose(lz["V"], E, atol=1e-15)
        assert np.allclose(sp["V"], E, atol=1e-15)
        assert np.allclose(lz["sigma"], c * d[:k] ** 2, rtol=1e-15)
        assert np.allclose(sp["sigma"], d[:k], rtol=1e-15)


def test_svd_step_against_brute_force_on_the_sphere():
    """Tiny case: the first right singular vector maximises ||F v|| over the
    unit sphere (variational characterisation). Brute force over a dense
    Fibonacci lattice on S^2 must find the oracle's v_1 (up to sign) within
    the lattice resolution, and the same maximum."""
    X = _noisy(m=30, n=3, r=3, s=0.1, seed=5)
    om = P.gaussian_omega(3, 2, seed=9)
    lz = O.lazy_fit(X, om, 2)
    F = lz["F"]
    N = 400_000
    i = np.arange(N) + 0.5
    phi = np.arccos(1 - 2 * i / N)
    th = math.pi * (1 + 5 ** 0.5) * i
    pts = np.stack([np.cos(th) * np.sin(phi), np.sin(th) * np.sin(phi), np.cos(phi)], 1)
    vals = np.linalg.norm(pts @ F.T, axis=1)
    best = pts[np.argmax(vals)]
    res = math.sqrt(4 * math.pi / N) * 3
    v1 = lz["V"][:, 0]
    assert min(np.linalg.norm(best - v1), np.linalg.norm(best + v1)) < res
    assert abs(vals.max() - lz["sigma"][0]) <= lz["sigma"][0] * res ** 2


# ----------------------------------------------------------- propositions --

def test_proposition_1_lazy_amd_equals_amd():
    """Prop. 1: Q Q^T X = U' U^T X, with U' = U (U^T U)^-1 the pseudo-inverse
    of eqs. (updown)/(downup); also eq. (updown): U^T U' = I."""
    X = _noisy()
    om = P.gaussian_omega(X.shape[1], 10, seed=4)
    U = O.sketch(X, om)
    Up = np.linalg.solve(U.T @ U, U.T).T
    Q = O.spca_fit(X, om, 10)["Q"]
    lhs = Q @ (Q.T @ X)
    rhs = Up @ O.lazy_factor(X, U)
    assert np.linalg.norm(lhs - rhs) < 1e-12 * np.linalg.norm(X)
    assert np.max(np.abs(U.T @ Up - np.eye(10))) < 1e-12


def test_proposition_2_same_subspace():
    """Prop. 2: V^s and V^l are orthonormal bases of <X^T u_1 .. X^T u_l>."""
    X = _noisy()
    k = 10
    om = P.gaussian_omega(X.shape[1], k, seed=4)
    lz = O.lazy_fit(X, om, k)
    sp = O.spca_fit(X, om, k)
    for V in (lz["V"], sp["V"]):
        assert np.max(np.abs(V.T @ V - np.eye(k))) < 1e-13
    assert O.principal_sines(sp["V"], lz["V"]).max() < 1e-12
    cf = _orth(O.closed_form_basis(X, om))
    assert O.principal_sines(cf, lz["V"]).max() < 1e-11
    # footnote to eq. (dim_reduction_maps): the bases themselves differ
    assert np.max(np.abs(np.abs(sp["V"]) - np.abs(lz["V"]))) > 1e-3


def test_proposition_3_identical_distances():
    """Prop. 3: d(pi^s v_i, pi^s v_j) = d(pi^l v_i, pi^l v_j) <= d(v_i, v_j);
    with k = n the maps are isometries (Lemma on orthonormal V)."""
    X = _noisy(m=300, n=40)
    k = 8
    om = P.gaussian_omega(40, k, seed=8)
    Vs = O.spca_fit(X, om, k)["V"]
    Vl = O.lazy_fit(X, om, k)["V"]
    rng = np.random.default_rng(0)
    pairs = rng.integers(0, X.shape[0], size=(500, 2))
    ds = O.pairwise_distances(O.transform(X, Vs), pairs)
    dl = O.pairwise_distances(O.transform(X, Vl), pairs)
    d0 = O.pairwise_distances(X, pairs)
    assert np.max(np.abs(ds - dl)) <= 1e-12 * np.max(d0)
    assert np.all(dl <= d0 * (1 + 1e-14))
    omf = P.gaussian_omega(40, 40, seed=8)
    Vf = O.lazy_fit(X, omf, 40)["V"]
    df = O.pairwise_distances(O.transform(X, Vf), pairs)
    assert np.max(np.abs(df - d0)) <= 1e-12 * np.max(d0)


def test_lemma_norm_contraction():
    """Lemma (norm before and after an orthonormal V): ||V^T v|| <= ||v||,
    with equality exactly for v in the span of V."""
    rng = np.random.default_rng(2)
    V = random_orthonormal_np(30, 5, rng)
    for _ in range(50):
        v = rng.standard_normal(30)
        assert np.linalg.norm(O.transform(v[None], V)) <= np.linalg.norm(v) * (1 + 1e-15)
        w = V @ rng.standard_normal(5)
        assert abs(np.linalg.norm(O.transform(w[None], V)) - np.linalg.norm(w)) < 1e-14 * np.linalg.norm(w)


def test_gram_is_factor_times_omega():
    """G = U^T U = U^T X Omega = F Omega (associativity of U = X Omega): a
    transposed or misplaced operand in F or G breaks it."""
    X = _noisy(m=200, n=30)
    om = P.gaussian_omega(30, 7, seed=1)
    lz = O.lazy_fit(X, om, 7)
    assert np.linalg.norm(lz["G"] - lz["F"] @ om) < 1e-12 * np.linalg.norm(lz["G"])
    assert np.allclose(lz["G"], lz["G"].T, rtol=0, atol=1e-12 * np.abs(lz["G"]).max())
    w = np.random.default_rng(3).standard_normal(30)
    assert np.linalg.norm(lz["F"] @ w - O.factor_probe(X, om, w)) < 1e-12 * np.linalg.norm(lz["F"] @ w)


def test_eig_route_matches_svd_route():
    """Dagger note of the algorithm table: the SVD of F via the eigensolution
    of F F^T gives the same D and V (well-separated spectrum)."""
    X = lowrank_np(500, 50, 8, "inv", 0.01, 7, "f64", scale=10.0)
    om = P.gaussian_omega(50, 8, seed=3)
    F = O.lazy_fit(X, om, 8)["F"]
    V1, d1 = O.truncated_svd(F, 8)
    V2, d2 = O.eig_route_svd(F, 8)
    assert np.allclose(d1, d2, rtol=1e-9)
    assert np.max(np.abs(V1 - V2)) < 1e-7


@pytest.mark.parametrize("S", [1, 2, 7])
def test_streaming_lazy_equals_in_core(S):
    """Algorithm 4 equals Algorithm 2 for any horizontal slicing; a row
    permutation of X leaves F, G and V unchanged."""
    X = _noisy(m=350, n=40)
    om = P.gaussian_omega(40, 9, seed=6)
    a = O.lazy_fit(X, om, 9)
    b = O.streaming_lazy_fit(X, om, 9, S=S)
    assert np.linalg.norm(a["F"] - b["F"]) < 1e-13 * np.linalg.norm(a["F"])
    assert np.linalg.norm(a["G"] - b["G"]) < 1e-13 * np.linalg.norm(a["G"])
    perm = np.random.default_rng(S).permutation(X.shape[0])
    c = O.streaming_lazy_fit(X[perm], om, 9, S=S)
    assert np.linalg.norm(a["F"] - c["F"]) < 1e-13 * np.linalg.norm(a["F"])
    assert O.principal_sines(a["V"], c["V"]).max() < 1e-12


def test_streaming_spca_equals_spca():
    """Algorithm 3 equals Algorithm 1: same Sigma^s and subspace."""
    X = _noisy(m=300, n=40)
    om = P.gaussian_omega(40, 8, seed=6)
    a = O.spca_fit(X, om, 8)
    b = O.streaming_spca_fit(X, om, 8, S=5)
    assert np.allclose(a["sigma"], b["sigma"], rtol=1e-12)
    assert O.principal_sines(a["V"], b["V"]).max() < 1e-11


def test_kxk_route_gives_spca_result():
    """Eq. (simplified_approx_svd) with R = chol(U^T U): R^-T F = Q^T X, so its
    SVD gives SPCA's Sigma^s and V^s from k x k work only."""
    X = _noisy()
    om = P.gaussian_omega(X.shape[1], 10, seed=12)
    lz = O.lazy_fit(X, om, 10)
    sp = O.spca_fit(X, om, 10)
    V, s = O.sigma_x_kxk(lz["F"], lz["G"], 10)
    assert np.allclose(s, sp["sigma"], rtol=1e-11)
    assert O.principal_sines(V, sp["V"]).max() < 1e-11


def test_interlacing_and_eckart_young():
    """X_hat = Q Q^T X is X projected onto a k-dimensional subspace, so
    Sigma^s_i <= sigma_i(X); and ||X - X_hat||_F is at least the best rank-k
    error (sum_{i>k} sigma_i^2)^(1/2) (Eckart-Young)."""
    X = _noisy(m=250, n=45, s=0.2)
    k = 9
    om = P.gaussian_omega(45, k, seed=13)
    sp = O.spca_fit(X, om, k)
    sx = np.linalg.svd(X, compute_uv=False)
    assert np.all(sp["sigma"] <= sx[:k] * (1 + 1e-13))
    Q = sp["Q"]
    err = np.linalg.norm(X - Q @ (Q.T @ X))
    assert err >= math.sqrt(np.sum(sx[k:] ** 2)) * (1 - 1e-13)


# ---------------------------------------------------------------- metrics --

def test_principal_sines_of_known_angles():
    """Subspaces at known principal angles theta_i: span(e_i) vs
    span(cos t_i e_i + sin t_i e_{k+i}); sines must be sin t_i exactly and the
    chordal distance sqrt(2) ||sin t||."""
    k, n = 4, 10
    t = np.array([0.0, 1e-9, 0.3, 1.2])
    Va = np.zeros((n, k))
    Vb = np.zeros((n, k))
    for i in range(k):
        Va[i, i] = 1
        Vb[i, i] = math.cos(t[i])
        Vb[k + i, i] = math.sin(t[i])
    rng = np.random.default_rng(0)
    Rot = random_orthonormal_np(n, n, rng)
    s = O.principal_sines(Rot @ Va, Rot @ Vb)
    assert np.allclose(np.sort(s), np.sort(np.sin(t)), rtol=1e-7, atol=1e-15)
    assert abs(s.min() - 0) < 1e-15 and abs(sorted(s)[1] - 1e-9) < 1e-15
    cd = O.chordal_distance(Rot @ Va, Rot @ Vb)
    assert abs(cd - math.sqrt(2) * np.linalg.norm(np.sin(t))) < 1e-14


def test_pairwise_distances_hand_example():
    """Euclidean distances of listed row pairs, written out by hand: a 3-4-5
    triangle and more. A squared distance (25, 13, 2), the L1 distance (7, 5,
    2) or an index mix-up gives other numbers."""
    Z = np.array([[0.0, 0.0, 0.0],
                  [3.0, 4.0, 0.0],
                  [1.0, 1.0, 0.0],
                  [1.0, 2.0, 2.0]])
    pairs = [(0, 1), (1, 2), (0, 2), (3, 0), (2, 2)]
    d = O.pairwise_distances(Z, pairs)
    assert d.shape == (5,)
    assert d[0] == 5.0
    assert d[1] == math.sqrt(13.0)
    assert d[2] == math.sqrt(2.0)
    assert d[3] == 3.0                      # sqrt(1 + 4 + 4)
    assert d[4] == 0.0
    # symmetric in the pair's order, and one row of Z per index
    assert np.array_equal(O.pairwise_distances(Z, [(1, 0), (2, 1)]), d[:2])


def test_canonical_order_and_sign():
    V = np.array([[0.6, -0.8], [-0.8, -0.6]])
    s = np.array([1.0, 2.0])
    Vc, sc = O.canonicalize(V, s)
    assert list(sc) == [2.0, 1.0]
    assert np.allclose(Vc, [[0.8, -0.6], [0.6, 0.8]])
    # ties in magnitude: the lowest index decides
    Vt, _ = O.canonicalize(np.array([[-0.5], [0.5]]), np.array([1.0]))
    assert Vt[0, 0] == 0.5


# ------------------------------------------------------------ sparse X (CSR) --

def test_csr_dense_hand_example():
    """A 4 x 5 matrix written out by hand: an empty row, unsorted columns and
    a repeated column (whose values add)."""
    rowptr = [0, 2, 2, 5, 6]
    colidx = [3, 0, 4, 1, 4, 2]
    values = [2.0, -1.0, 0.5, 3.0, 0.25, 7.0]
    want = np.array([[-1, 0, 0, 2, 0],
                     [0, 0, 0, 0, 0],
                     [0, 3, 0, 0, 0.75],
                     [0, 0, 7, 0, 0]], dtype=np.float64)
    assert np.array_equal(O.csr_dense(rowptr, colidx, values, 5), want)


def test_csr_dense_matches_scipy_and_row_slices():
    """Against scipy.sparse (an independent CSR implementation), including a
    row slice given by an offset rowptr."""
    import scipy.sparse as sp
    rng = np.random.default_rng(4)
    m, n = 57, 41
    counts = rng.integers(0, 9, m)
    counts[[3, 17, 40]] = 0
    rowptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    colidx = rng.integers(0, n, rowptr[-1]).astype(np.int32)       # repeats allowed
    values = rng.standard_normal(rowptr[-1])
    want = sp.csr_matrix((values, colidx, rowptr), shape=(m, n)).toarray()
    assert np.allclose(O.csr_dense(rowptr, colidx, values, n), want, rtol=0, atol=1e-15)
    r0, r1 = 11, 44
    got = O.csr_dense(rowptr[r0:r1 + 1], colidx, values, n)
    assert np.allclose(got, want[r0:r1], rtol=0, atol=1e-15)


def test_csr_generator_density():
    """The synthetic feature matrix has the requested mean density and sorted,
    unique columns in every row."""
    from synth import csr_np
    rowptr, colidx, values = csr_np(300, 5000, density=0.0244, seed=9)
    assert abs(rowptr[-1] / (300 * 5000) - 0.0244) < 0.002
    for i in range(0, 300, 37):
        c = colidx[rowptr[i]:rowptr[i + 1]]
        assert np.all(np.diff(c) > 0)
    assert np.all((values > 0) & (values <= 1))


def test_csr_factor_rows_brute_force():
    """U_C = X Omega_C and F_C = U_C^T X by explicit loops over the stored
    entries of a tiny CSR matrix (brute force)."""
    rng = np.random.default_rng(12)
    m, n, c = 9, 7, 3
    counts = rng.integers(0, 5, m)
    rowptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    colidx = rng.integers(0, n, rowptr[-1]).astype(np.int32)
    values = rng.standard_normal(rowptr[-1])
    om = rng.standard_normal((n, c))
    U = np.zeros((m, c))
    for i in range(m):
        for e in range(rowptr[i], rowptr[i + 1]):
            for a in range(c):
                U[i, a] += values[e] * om[colidx[e], a]
    F = np.zeros((c, n))
    for i in range(m):
        for e in range(rowptr[i], rowptr[i + 1]):
            for a in range(c):
                F[a, colidx[e]] += U[i, a] * values[e]
    gotU, gotF = O.csr_factor_rows(rowptr, colidx, values, n, om)
    assert np.allclose(gotU, U, rtol=1e-14, atol=1e-14)
    assert np.allclose(gotF, F, rtol=1e-14, atol=1e-14)
    # the same on a row slice (offset rowptr)
    gotU2, _ = O.csr_factor_rows(rowptr[2:7], colidx, values, n, om)
    assert np.allclose(gotU2, U[2:6], rtol=1e-14, atol=1e-14)
