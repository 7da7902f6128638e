"""Plain FP64 CPU oracle for SPCA and Lazy SPCA.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module. It shares no code with
the HIP library and never imports it.

Paper: M. Wojnowicz, D. Nguyen, L. Li, X. Zhao, "Lazy stochastic principal
component analysis", arXiv 1709.07175. Every function below follows the
passage named in its docstring, in the paper's notation (U = X Omega is the
sketch the library calls Y; F = U^T X is the factor the library calls F or B).
Library primitives serve as single steps: matrix products (numpy @), the
Householder QR of LAPACK (numpy.linalg.qr) for the "qr" of Algorithms 1 and 3,
and the LAPACK SVD (numpy.linalg.svd) for the truncated SVD of F.

Readings taken where the paper is silent (each pinned by a test):
  * no centering of X (Sec. I-B, the paragraph after eq. (spca_eqn));
  * c = 1 in eq. (rp): V and Sigma^s do not depend on it;
  * l = k (Sec. IV-A: the experiments set l = k);
  * columns ordered by decreasing singular value; each column's sign is
    chosen so that its entry of largest magnitude is positive (lowest row
    index on ties) -- the paper fixes no basis (footnote to eq.
    (dim_reduction_maps): the two methods need not find the same basis);
  * the Lazy singular values returned are D of Algorithm 2 (singular values
    of F = U^T X); Sigma^s of eq. (approx_svd) is returned separately.
"""
import numpy as np

__all__ = [
    "sketch", "lazy_factor", "gram", "truncated_svd", "canonicalize",
    "lazy_fit", "spca_fit", "streaming_lazy_fit", "streaming_spca_fit",
    "transform", "eig_route_svd", "closed_form_basis", "sigma_x_kxk",
    "factor_probe", "principal_sines", "chordal_distance", "pairwise_distances",
    "csr_dense", "csr_factor_rows",
]


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def sketch(X, Omega):
    """U = X Omega (eq. (rp) with c = 1; Algorithm 2 step 1)."""
    return _f64(X) @ _f64(Omega)


def lazy_factor(X, U):
    """F = U^T X (Algorithm 2 step 2, eq. (simplified_approx_svd))."""
    return _f64(U).T @ _f64(X)


def gram(U):
    """G = U^T U, the k x k Gram of the sketch (U' = U G^-1 satisfies
    eq. (updown); the Cholesky factor of G is the R of Algorithm 3)."""
    U = _f64(U)
    return U.T @ U


def canonicalize(V, s):
    """Order columns by decreasing s (stable) and fix each column's sign so
    that its largest-magnitude entry is positive (lowest index on ties)."""
    V = _f64(V).copy()
    s = _f64(s).copy()
    order = np.argsort(-s, kind="stable")
    V, s = V[:, order], s[order]
    if V.shape[0]:
        idx = np.argmax(np.abs(V), axis=0)          # first maximum on ties
        sign = np.sign(V[idx, np.arange(V.shape[1])])
        sign[sign == 0] = 1.0
        V = V * sign
    return V, s


def truncated_svd(F, k):
    """Truncated SVD of F, keeping the k dominant triplets (Algorithm 2
    step 3 and the dagger note of the algorithm table). Returns (V, D) with
    V (n x k) the right singular vectors and D (k) the singular values."""
    _, d, wt = np.linalg.svd(_f64(F), full_matrices=False)
    return canonicalize(wt[:k].T, d[:k])


def lazy_fit(X, Omega, k):
    """Algorithm 2 (Lazy SPCA): U = X Omega; F = U^T X; truncated SVD of F.

    Returns V^l (n x k), D (k) and the intermediates F (k x n), G (k x k)."""
    U = sketch(X, Omega)
    F = lazy_factor(X, U)
    V, d = truncated_svd(F, k)
    return {"V": V, "sigma": d, "F": F, "G": gram(U)}


def spca_fit(X, Omega, k):
    """Algorithm 1 (SPCA): U = X Omega; Q, R = qr(U); F = Q^T X; truncated
    SVD of F gives V^s and Sigma^s of eq. (approx_svd)."""
    X = _f64(X)
    U = sketch(X, Omega)
    Q, R = np.linalg.qr(U, mode="reduced")
    F = Q.T @ X
    V, s = truncated_svd(F, k)
    return {"V": V, "sigma": s, "Q": Q, "R": R, "F": F}


def _slices(m, S):
    edges = np.linspace(0, m, S + 1).round().astype(int)
    return [(edges[i], edges[i + 1]) for i in range(S)]


def streaming_lazy_fit(X, Omega, k, S=1, slices=None):
    """Algorithm 4 (Streaming Lazy SPCA): F += U_s^T X_s over horizontal
    slices X_s, then the truncated SVD of F. Also accumulates G = sum U_s^T U_s.
    `slices` may list (row0, row1) pairs; otherwise S equal slices."""
    Omega = _f64(Omega)
    n = X.shape[1]
    F = np.zeros((Omega.shape[1], n))
    G = np.zeros((Omega.shape[1], Omega.shape[1]))
    for r0, r1 in (slices if slices is not None else _slices(X.shape[0], S)):
        X_s = _f64(X[r0:r1])          # each slice is upcast on its own
        U_s = X_s @ Omega
        F += U_s.T @ X_s
        G += U_s.T @ U_s
    V, d = truncated_svd(F, k)
    return {"V": V, "sigma": d, "F": F, "G": G}


def streaming_spca_fit(X, Omega, k, S=1):
    """Algorithm 3 (Streaming SPCA): F += U_s^T X_s; R from qr([R; U_s]);
    then F = R^-T F and the truncated SVD of F."""
    X, Omega = _f64(X), _f64(Omega)
    sl = _slices(X.shape[0], S)
    r0, r1 = sl[0]
    U1 = X[r0:r1] @ Omega
    R = np.linalg.qr(U1, mode="r")
    F = U1.T @ X[r0:r1]
    for r0, r1 in sl[1:]:
        U_s = X[r0:r1] @ Omega
        F += U_s.T @ X[r0:r1]
        R = np.linalg.qr(np.vstack([R, U_s]), mode="r")
    F = np.linalg.solve(R.T, F)
    V, s = truncated_svd(F, k)
    return {"V": V, "sigma": s, "R": R}


def transform(X, V):
    """Z = X V: the dimensionality-reduction map pi(x) = V^T x applied to
    every sample (row) of X (eq. (dim_reduction_maps))."""
    return _f64(X) @ _f64(V)


def eig_route_svd(F, k):
    """SVD of F through the eigensolution of F F^T (dagger note of the
    algorithm table): F F^T = W Lambda W^T, D = Lambda^(1/2),
    V = F^T W D^-1."""
    F = _f64(F)
    lam, W = np.linalg.eigh(F @ F.T)
    order = np.argsort(-lam, kind="stable")[:k]
    lam, W = lam[order], W[:, order]
    d = np.sqrt(lam)
    V = (F.T @ W) / d
    return canonicalize(V, d)


def closed_form_basis(X, Omega):
    """range(X^T X Omega) = <X^T u_1, ..., X^T u_l> (Proposition 2), formed
    as the columns of (X^T X) Omega without the sketch U."""
    X = _f64(X)
    return (X.T @ X) @ _f64(Omega)


def sigma_x_kxk(F, G, k):
    """Sigma^s and V^s from F and G alone (eq. (simplified_approx_svd) and
    Algorithm 3 step 3): with G = R^T R (Cholesky; R is Algorithm 3's R up to
    row signs), Q^T X = R^-T F, whose truncated SVD gives (V^s, Sigma^s)."""
    R = np.linalg.cholesky(_f64(G)).T
    return truncated_svd(np.linalg.solve(R.T, _f64(F)), k)


def factor_probe(X, Omega, w):
    """F w = Omega^T (X^T (X w)) for a probe vector w (n), by three
    matrix-vector products; any entry or direction of F = U^T X can be checked
    this way at any m without forming U."""
    X = _f64(X)
    return _f64(Omega).T @ (X.T @ (X @ _f64(w)))


def csr_dense(rowptr, colidx, values, n):
    """The m x n matrix a CSR triple stands for (the sparse slices of
    Experiment 1, "Data and Method"): row i holds value values[e] at column
    colidx[e] for e in [rowptr[i], rowptr[i + 1]); repeated columns of a row
    add. rowptr[0] may be positive (a row slice of a larger matrix)."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    m = rowptr.size - 1
    e0, e1 = int(rowptr[0]), int(rowptr[-1])
    rows = np.repeat(np.arange(m), np.diff(rowptr))
    X = np.zeros((m, n), dtype=np.float64)
    np.add.at(X, (rows, np.asarray(colidx[e0:e1], dtype=np.int64)), _f64(values[e0:e1]))
    return X


def csr_factor_rows(rowptr, colidx, values, n, Omega_C):
    """U_C = X Omega_C and F_C = U_C^T X (Algorithm 2 steps 1 and 2 for a few
    columns C of Omega) for the CSR matrix of csr_dense, at any m: the two
    sparse products are the matrix-product step, by scipy.sparse (no dense
    X is formed). Returns (U_C, F_C)."""
    import scipy.sparse as sp
    rowptr = np.asarray(rowptr, dtype=np.int64)
    m = rowptr.size - 1
    e0, e1 = int(rowptr[0]), int(rowptr[-1])
    X = sp.csr_matrix((_f64(values[e0:e1]), np.asarray(colidx[e0:e1]), rowptr - e0), shape=(m, n))
    U = X @ _f64(Omega_C)
    return U, np.asarray((X.T @ U).T)


def principal_sines(Va, Vb):
    """Sines of the principal angles between span(Va) and span(Vb), both with
    orthonormal columns, as the singular values of Vb - Va (Va^T Vb)
    (Bjorck and Golub, Math. Comp. 27, 1973), sorted decreasingly."""
    Va, Vb = _f64(Va), _f64(Vb)
    W = Vb - Va @ (Va.T @ Vb)
    return np.linalg.svd(W, compute_uv=False)


def chordal_distance(Va, Vb):
    """Chordal distance on the Grassmannian, ||Va Va^T - Vb Vb^T||_F
    (Sec. V-A, the subspace distance of Experiment 2)."""
    Va, Vb = _f64(Va), _f64(Vb)
    return np.linalg.norm(Va @ Va.T - Vb @ Vb.T)


def pairwise_distances(Z, pairs):
    """d(z_i, z_j) for the listed index pairs (rows of Z)."""
    Z = _f64(Z)
    pairs = np.asarray(pairs)
    return np.linalg.norm(Z[pairs[:, 0]] - Z[pairs[:, 1]], axis=1)
