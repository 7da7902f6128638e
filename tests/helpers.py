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
