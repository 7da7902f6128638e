"""Parity at the workloads' full sizes, in the launch configuration bench.py
times (the pass over all rows in one call, default stripes and tiles), on
outputs the FP64 oracle can compute one by one:

  * whole rows of F = Y^T X and blocks of G = Y^T Y for a few sketch columns
    C: the oracle streams X from the device in row chunks and forms
    Y[:, C] = X Omega[:, C] (oracle.sketch) and Y[:, C]^T X (oracle.
    lazy_factor), with the componentwise bound of tests/helpers.py evaluated
    for exactly those entries;
  * the small stage on the device's own F against the oracle's truncated SVD
    of that F (subspace and singular values, within c u kappa(F));
  * sampled rows of the projection Z = X V against oracle.transform.

Each workload takes well under a minute; progress is printed per stage."""
import time

import numpy as np
import pytest

from oracle import lspca_oracle as O
from oracle import philox as P
from synth import config, lowrank_torch
from tests.helpers import U16, U32, U64, UNIT, gamma

pytestmark = pytest.mark.gpu

CHUNK = 1 << 16


def _log(msg):
    print(f"[fullsize] {time.strftime('%H:%M:%S')} {msg}", flush=True)


def _sampled_pass_reference(X, om, cols, dtype):
    """F[C, :], G[C, C] by definition in FP64, and their componentwise
    bounds, streaming X (device) in row chunks."""
    m, n = X.shape
    oC = om[:, cols]
    aoC = np.abs(oC)
    u = UNIT[dtype]
    F = np.zeros((len(cols), n))
    G = np.zeros((len(cols), len(cols)))
    t1 = np.zeros((len(cols), n))            # |Omega_C|^T |X|^T |X|
    t2 = np.zeros((len(cols), n))            # |Y_C|^T |X| with |Y| inflated by its own bound
    g1 = np.zeros((len(cols), len(cols)))    # (|X| |Omega_C|)^T |Y_C|
    g2 = np.zeros((len(cols), len(cols)))    # |Y_C|^T |Y_C|
    ymax = np.zeros(len(cols))
    colsum = np.zeros(n)                     # column sums of |X|
    for r0 in range(0, m, CHUNK):
        Xc = X[r0:r0 + CHUNK].double().cpu().numpy()
        U = O.sketch(Xc, oC)
        F += O.lazy_factor(Xc, U)
        G += U.T @ U
        aX = np.abs(Xc)
        aXO = aX @ aoC
        aY = np.abs(U) + gamma(n, u) * aXO
        t1 += aXO.T @ aX
        t2 += aY.T @ aX
        g1 += aXO.T @ aY
        g2 += aY.T @ aY
        ymax = np.maximum(ymax, aY.max(axis=0))
        colsum += aX.sum(axis=0)
        if (r0 // CHUNK) % 16 == 0:
            _log(f"oracle rows {r0 + len(Xc)} of {m}")
    bF = gamma(n, u) * t1 + gamma(m, u) * t2
    if dtype in U16:
        # split error of the refined 16-bit sketch and the subnormal floor of
        # the scaled parts (the terms of pass_bound)
        bF = bF + 1.01 * U16[dtype] ** 2 * t2 + 2.0 ** -37 * ymax[:, None] * colsum[None, :]
        bG = bF @ np.abs(om[:, cols]) + 1e-12 * np.abs(G)
    else:
        bG = 2 * gamma(n, u) * g1 + gamma(m, u) * g2
    return F, G, bF, bG


@pytest.mark.parametrize("cfg_id", [2, 3, 4])
def test_full_size_pass_factor_and_projection(gpu_lib, cfg_id):
    import torch
    cfg = config(cfg_id)
    m, n, k, dtype = cfg["m"], cfg["n"], cfg["k"], cfg["dtype"]
    _log(f"workload {cfg_id}: X {m}x{n} {dtype}, {cfg['kind']} Omega, k={k}")
    X = lowrank_torch(m, n, cfg["r"], cfg["spectrum"], cfg["s"], cfg["data_seed"], dtype, device="cuda")
    torch.cuda.synchronize()
    kw = {"sparse_p": cfg.get("p", 64)}
    F = torch.zeros((k, n), dtype=torch.float64, device="cuda")
    G = torch.zeros((k, k), dtype=torch.float64, device="cuda")
    gpu_lib.accumulate(X, k, cfg["kind"], cfg["omega_seed"], F, G, **kw)
    torch.cuda.synchronize()
    _log("device pass done")
    om = P.omega(n, k, cfg["kind"], cfg["omega_seed"], cfg.get("p", 64), dtype=dtype)
    rng = np.random.default_rng(cfg_id)
    cols = np.sort(rng.choice(k, 4, replace=False))
    cols[0] = 0
    cols[-1] = k - 1
    Fr, Gr, bF, bG = _sampled_pass_reference(X, om, cols, dtype)
    Fd = F.cpu().numpy()[cols]
    Gd = G.cpu().numpy()[np.ix_(cols, cols)]
    assert np.all(np.abs(Fd - Fr) <= bF), np.max(np.abs(Fd - Fr) / bF)
    assert np.all(np.abs(Gd - Gr) <= bG), np.max(np.abs(Gd - Gr) / bG)
    _log(f"F rows {[int(c) for c in cols]} and G block within bound (max ratio {np.max(np.abs(Fd - Fr) / bF):.3g})")

    # small stage on the device's own F
    V, s = gpu_lib.factor(F)
    Vd, sd = V.cpu().numpy(), s.cpu().numpy()
    Vr, dr = O.truncated_svd(F.cpu().numpy(), k)
    kappa = dr[0] / dr[-1]
    assert np.max(np.abs(sd - dr) / dr) < 64 * U64 * kappa * k
    assert O.principal_sines(Vr, Vd).max() < 64 * U64 * kappa * k
    assert np.max(np.abs(Vd.T @ Vd - np.eye(k))) < 16 * k * U64
    _log(f"factor: kappa(F) {kappa:.3g}, sigma rel err {np.max(np.abs(sd - dr) / dr):.3g}")

    # projection on sampled rows (the full Z, as lspca_transform computes it)
    Z = gpu_lib.transform(X, V)
    torch.cuda.synchronize()
    rows = np.sort(rng.choice(m, 64, replace=False))
    rows[-1] = m - 1
    Xr = X[torch.from_numpy(rows).cuda()].double().cpu().numpy()
    Vq = P.round_f32(Vd) if dtype == "f32" else Vd
    ref = O.transform(Xr, Vq)
    u = U64 if dtype == "f64" else U32
    bound = gamma(n, u) * (np.abs(Xr) @ np.abs(Vq))
    if dtype in U16:
        bound = 2 * bound + (1.01 * U16[dtype] ** 2 + U32 + 2.0 ** -24) * (np.abs(Xr) @ np.abs(Vd))
    Zs = Z[torch.from_numpy(rows).cuda()].double().cpu().numpy()
    assert np.all(np.abs(Zs - ref) <= bound + 1e-300)
    _log(f"projection rows within bound (max ratio {np.max(np.abs(Zs - ref) / (bound + 1e-300)):.3g})")
