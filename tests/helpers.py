"""Shared helpers of the GPU tests: moving seeded inputs to the device and
the error bounds the parity checks use.

Error model (stated once, used by every FP32/FP64 parity test). For a
product C = A B accumulated over K terms in a floating-point type with unit
roundoff u, the computed result obeys the componentwise bound
|C_hat - C| <= gamma_K |A| |B|, gamma_K = K u / (1 - K u) (Higham, Accuracy
and Stability of Numerical Algorithms, 2nd ed., Sec. 3.5). For the two
products of the pass, Y = X Omega (K = n) and F = Y^T X (K = rows summed in
the working type, at most m), this gives
  |F_hat - F| <= gamma_n |Omega|^T |X|^T |X| + gamma_m |Y|^T |X|
and likewise for G = Y^T Y. For 16-bit data (BF16, FP16) the products of 16-bit values are exact in
FP32 and accumulate in FP32 (u = 2^-24); the FP32 sketch Y enters F as
Y_hi + Y_lo (refinement) or Y_hi, each part rounded to the 16-bit type, so
|Y - Y_hi - Y_lo| <= rho |Y| with rho = u16^2 (refined) or u16 (not), u16 =
2^-8 (BF16) or 2^-11 (FP16). That adds rho |Y|^T |X| to the bound on F, and
G = F Omega (FP64) inherits |bound_F| |Omega|.
The singular values then move by at most
||F_hat - F||_2 <= ||bound||_F (Weyl), and the row space of F (= span V) by
sin theta <= ||bound||_F / (sigma_k - ||bound||_F) (Wedin).
"""
import math

import numpy as np

U32 = 2.0 ** -24
U64 = 2.0 ** -53
UNIT = {"f64": U64, "f32": U32, "bf16": U32, "f16": U32}
U16 = {"bf16": 2.0 ** -8, "f16": 2.0 ** -11}


def gamma(K, u):
    return K * u / (1 - K * u)


def to_device(Xs, dtype, device="cuda"):
    """numpy storage array (synth.to_storage_np) -> torch device tensor."""
    import torch
    if dtype == "bf16":
        t = torch.from_numpy(np.ascontiguousarray(Xs).view(np.int16)).view(torch.bfloat16)
    else:
        t = torch.from_numpy(np.ascontiguousarray(Xs))
    return t.to(device)


def pass_bound(X64, Om64, dtype, refine=True):
    """Componentwise bounds on F and G for the pass computed in `dtype`."""
    u = UNIT[dtype]
    m, n = X64.shape
    aX, aO = np.abs(X64), np.abs(Om64)
    Y = X64 @ Om64
    aXO = aX @ aO                                   # |X| |Omega| (m x k), reused below
    aY = np.abs(Y) + gamma(n, u) * aXO
    bF = gamma(n, u) * (aXO.T @ aX) + gamma(m, u) * (aY.T @ aX)
    if dtype in U16:
        rho = U16[dtype] ** 2 if refine else U16[dtype]
        # split error, plus FP16's subnormal floor (columns scaled so the
        # largest |Y| is near 2^14: spacing 2^-24 there is 2^-38 max|Y|)
        bF = bF + (rho * 1.01) * (aY.T @ aX) + 2.0 ** -37 * aY.max(axis=0)[:, None] * aX.sum(axis=0)[None, :]
        bG = bF @ aO + 1e-12 * np.abs(Y.T @ Y)
        return bF, bG
    bG = 2 * gamma(n, u) * (aXO.T @ aY) + gamma(m, u) * (aY.T @ aY)
    return bF, bG


def subspace_tol(sigma_k, err):
    """Wedin-type bound on the principal-angle sine between row spaces."""
    if err >= sigma_k / 2:
        return 1.0
    return err / (sigma_k - err)


# ------------------------------------------------------------------------
# Full-size checks of the pass. The library sums at most MAX_FP32_DEPTH rows
# in one FP32 partial of F (and of G) and adds the partials in FP64
# (include/lspca.h), so the accumulation error of F is that of a sum over at
# most `depth` rows in the working type plus an FP64 sum over the partials,
# not a sum over all m rows.
MAX_FP32_DEPTH = 65536

# Norm-wise tolerance: a few standard deviations of the probabilistic
# rounding model (Higham and Mary, SIAM J. Sci. Comput. 41, 2019: the error
# of a length-K sum is O(sqrt(K) u) relative to its terms with high
# probability). Errors made independently per row of X -- the sketch's own
# rounding (length n sums) and the split of the 16-bit sketch -- average out
# in the sum over rows F = sum_r y_r^T x_r and enter F at most with a factor
# sqrt(n / m) relative to ||F||; the accumulation over the rows of one
# partial (depth c) is not averaged within the partial but is across the
# m / c independent partials: u sqrt(c) / sqrt(m / c) = u c / sqrt(m).
NORM_LAMBDA = 8.0


def factor_norm_tol(dtype, m, n, depth, refine=True):
    """Stated bound on ||F_hat - F||_F / ||F||_F for the pass in `dtype`."""
    u = UNIT[dtype]
    rho = 0.0
    if dtype in U16:
        rho = U16[dtype] ** 2 if refine else U16[dtype]
    avg = math.sqrt(n / m)
    return NORM_LAMBDA * (u * math.sqrt(n) * avg + u * depth / math.sqrt(m) + rho * avg)


class PassReference:
    """F = Y^T X, G = Y^T Y of the oracle (FP64) accumulated over row chunks,
    with the sums of absolute values the componentwise bound needs:
      t1 = (|X| |Omega|)^T |X|, t2 = |Y|^T |X| with |Y| inflated by the
      sketch's own bound, g1 = (|X| |Omega|)^T |Y|, g2 = |Y|^T |Y|.
    FP16 data also keep the parts of F carried by the stored entries below
    FP16's normal range (|x| < 2^-14), an allowance for matrix-core products
    that treat such inputs as zero: with X_sub those entries and Y_sub =
    X_sub Omega, the sketch's part fl_sketch = Y_sub^T (X - X_sub) and the
    factor's part fl_factor = Y^T X_sub (signed: the change of F if either
    product drops them), and flush = |X_sub Omega|^T |X| + |Y|^T |X_sub|
    (the componentwise allowance)."""

    def __init__(self, om, dtype):
        from oracle import lspca_oracle as O
        self.O = O
        self.om = np.asarray(om, dtype=np.float64)
        self.aom = np.abs(self.om)
        self.dtype = dtype
        n, k = self.om.shape
        self.m = 0
        self.F = np.zeros((k, n))
        self.G = np.zeros((k, k))
        self.t1 = np.zeros((k, n))
        self.t2 = np.zeros((k, n))
        self.g1 = np.zeros((k, k))
        self.g2 = np.zeros((k, k))
        self.ymax = np.zeros(k)
        self.colsum = np.zeros(n)
        f16 = dtype == "f16"
        self.flush = np.zeros((k, n)) if f16 else None
        self.fl_sketch = np.zeros((k, n)) if f16 else None
        self.fl_factor = np.zeros((k, n)) if f16 else None
        self.nsub = 0

    def add(self, Xc):
        """Rows Xc (FP64 values of the stored X) of the next chunk."""
        O = self.O
        n = self.om.shape[0]
        u = UNIT[self.dtype]
        U = O.sketch(Xc, self.om)
        self.F += O.lazy_factor(Xc, U)
        self.G += O.gram(U)
        aX = np.abs(Xc)
        aXO = aX @ self.aom
        aY = np.abs(U) + gamma(n, u) * aXO
        self.t1 += aXO.T @ aX
        self.t2 += aY.T @ aX
        self.g1 += aXO.T @ aY
        self.g2 += aY.T @ aY
        self.ymax = np.maximum(self.ymax, aY.max(axis=0))
        self.colsum += aX.sum(axis=0)
        if self.flush is not None:
            sub = (aX < 2.0 ** -14) & (aX > 0)
            if sub.any():
                import scipy.sparse as sp
                Xs = sp.csr_matrix(np.where(sub, Xc, 0.0))
                aXs = abs(Xs)
                self.nsub += int(Xs.nnz)
                Ysub = np.asarray(Xs @ self.om)
                self.fl_sketch += Ysub.T @ (Xc - Xs.toarray())
                self.fl_factor += np.asarray(Xs.T @ U).T
                self.flush += np.asarray(aXs @ self.aom).T @ aX + np.asarray(aXs.T @ aY).T
        self.m += Xc.shape[0]

    def bounds(self, depth, refine=True):
        """Componentwise bounds (bF, bG) on the device's F and G: sketch
        error gamma_n, FP32 accumulation over at most `depth` rows per
        partial, the FP64 sum of the m / depth partials, and for 16-bit data
        the split error, the FP16 subnormal floor of the scaled parts and the
        FP16 flush allowance; G = F Omega in FP64 for 16-bit data."""
        n = self.om.shape[0]
        d = self.dtype
        u = UNIT[d]
        parts = max(1, -(-self.m // depth))
        acc = gamma(min(depth, self.m), u) + 1.01 * gamma(parts, U64)
        bF = gamma(n, u) * self.t1 + acc * self.t2
        if d in U16:
            rho = U16[d] ** 2 if refine else U16[d]
            bF = bF + 1.01 * rho * self.t2 + 2.0 ** -37 * self.ymax[:, None] * self.colsum[None, :]
            if self.flush is not None:
                bF = bF + 1.01 * self.flush
            bG = bF @ self.aom + gamma(n, U64) * np.abs(self.F) @ self.aom + 1e-15 * np.abs(self.G)
        else:
            bG = 2 * gamma(n, u) * self.g1 + acc * self.g2
        return bF, bG


def check_pass(Fd, Gd, ref, depth, refine=True):
    """Compares the device's F, G with the oracle's. Returns a dict with the
    largest componentwise error / bound ratios, the norm-wise relative
    errors and their stated tolerance (factor_norm_tol, plus for FP16 data
    the norm of the two flush parts), and "ok"."""
    n = ref.om.shape[0]
    bF, bG = ref.bounds(depth, refine)
    nF = np.linalg.norm(ref.F)
    relF = np.linalg.norm(Fd - ref.F) / nF
    relG = np.linalg.norm(Gd - ref.G) / np.linalg.norm(ref.G) if Gd is not None else 0.0
    tol = factor_norm_tol(ref.dtype, ref.m, n, min(depth, ref.m), refine)
    out = {
        "comp_ratio_F": float(np.max(np.abs(Fd - ref.F) / bF)),
        "comp_ratio_G": float(np.max(np.abs(Gd - ref.G) / bG)) if Gd is not None else 0.0,
        "rel_F": float(relF), "rel_G": float(relG), "tol": float(tol),
    }
    if ref.flush is not None:
        fs = np.linalg.norm(ref.fl_sketch) / nF
        ff = np.linalg.norm(ref.fl_factor) / nF
        out.update(nsub=ref.nsub, flush_sketch_rel=float(fs), flush_factor_rel=float(ff))
        # the device against the oracle with the subnormal inputs dropped
        # from the sketch, and from both products (diagnostics)
        out["rel_F_flush_sketch"] = float(np.linalg.norm(Fd - ref.F + ref.fl_sketch) / nF)
        out["rel_F_flush_both"] = float(np.linalg.norm(Fd - ref.F + ref.fl_sketch + ref.fl_factor) / nF)
        tol = tol + fs + ff
        out["tol"] = float(tol)
    gtol = tol * (2.0 if ref.dtype not in U16 else 4.0)
    out["tol_G"] = float(gtol)
    out["ok"] = bool(out["comp_ratio_F"] <= 1.0 and out["comp_ratio_G"] <= 1.0 and relF <= tol
                     and relG <= gtol)
    return out
