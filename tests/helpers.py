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
and likewise for G = Y^T Y. The singular values then move by at most
||F_hat - F||_2 <= ||bound||_F (Weyl), and the row space of F (= span V) by
sin theta <= ||bound||_F / (sigma_k - ||bound||_F) (Wedin).
"""
import numpy as np

U32 = 2.0 ** -24
U64 = 2.0 ** -53
UNIT = {"f64": U64, "f32": U32}


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


def pass_bound(X64, Om64, dtype):
    """Componentwise bounds on F and G for the pass computed in `dtype`."""
    u = UNIT[dtype]
    m, n = X64.shape
    aX, aO = np.abs(X64), np.abs(Om64)
    Y = X64 @ Om64
    aY = np.abs(Y) + gamma(n, u) * (aX @ aO)
    bF = gamma(n, u) * (aO.T @ (aX.T @ aX)) + gamma(m, u) * (aY.T @ aX)
    bG = 2 * gamma(n, u) * ((aX @ aO).T @ aY) + gamma(m, u) * (aY.T @ aY)
    return bF, bG


def subspace_tol(sigma_k, err):
    """Wedin-type bound on the principal-angle sine between row spaces."""
    if err >= sigma_k / 2:
        return 1.0
    return err / (sigma_k - err)
