"""Parity at the workloads' full sizes, in the launch configuration bench.py
times (lspca_fit over all rows in one call, default stripes and tiles),
against the FP64 oracle streamed over ALL rows of X:

  * the whole F = Y^T X and G = Y^T Y of the pass (lspca_accumulate, the
    same kernels and plan as the fit) against the oracle's F and G
    (oracle.sketch / lazy_factor / gram over row chunks, Algorithms 2 and 4):
    every entry within the componentwise rounding bound of tests/helpers.py
    (FP32 sums over at most 65,536 rows per partial, the library's
    contract, then FP64), and the norm-wise relative errors within the
    stated tolerance of the probabilistic rounding model
    (helpers.factor_norm_tol);
  * the fit (lspca_fit) against the oracle's fit of the same X (truncated
    SVD of the oracle's F): the max principal-angle sine within the Wedin
    bound of the measured ||F_device - F||_2 and within the workload's stated
    target (BF16 with refinement: 1e-3), singular values within Weyl's bound;
  * the small stage on the device's own F against the oracle's truncated SVD
    of that F (subspace and singular values, within c u kappa(F));
  * sampled rows of the projection Z = X V against oracle.transform.

Each workload prints its measured errors and their ratio to the bounds."""
import time

import numpy as np
import pytest

from oracle import lspca_oracle as O
from oracle import philox as P
from synth import config, lowrank_torch
from tests.helpers import (MAX_FP32_DEPTH, U16, U32, U64, PassReference, check_pass, gamma,
                           subspace_tol)

pytestmark = pytest.mark.gpu

CHUNK = 1 << 15
# Max principal-angle sine of the fit against the oracle's fit of the same X
# (BASELINE target for BF16 with refinement; FP32 and FP16: stated here).
SINE_TARGET = {2: 1e-4, 3: 1e-3, 4: 1e-3}


def _log(msg):
    print(f"[fullsize] {time.strftime('%H:%M:%S')} {msg}", flush=True)


def _oracle_pass(X, om, dtype):
    """The oracle's pass over all rows of X (device tensor), chunk by chunk:
    each chunk's stored values are copied to the host exactly (FP64)."""
    import torch
    m = X.shape[0]
    ref = PassReference(om, dtype)
    for r0 in range(0, m, CHUNK):
        Xc = X[r0:r0 + CHUNK].to(torch.float64).cpu().numpy()
        ref.add(Xc)
        if (r0 // CHUNK) % 32 == 0:
            _log(f"oracle rows {r0 + len(Xc)} of {m}")
    return ref


@pytest.mark.timeout(900)
@pytest.mark.parametrize("cfg_id", [2, 3, 4])
def test_full_size_pass_fit_and_projection(gpu_lib, cfg_id):
    import torch
    cfg = config(cfg_id)
    m, n, k, dtype = cfg["m"], cfg["n"], cfg["k"], cfg["dtype"]
    kw = {"sparse_p": cfg.get("p", 64)}
    _log(f"workload {cfg_id}: X {m}x{n} {dtype}, {cfg['kind']} Omega, k={k}")
    X = lowrank_torch(m, n, cfg["r"], cfg["spectrum"], cfg["s"], cfg["data_seed"], dtype, device="cuda")
    torch.cuda.synchronize()
    F = torch.zeros((k, n), dtype=torch.float64, device="cuda")
    G = torch.zeros((k, k), dtype=torch.float64, device="cuda")
    gpu_lib.accumulate(X, k, cfg["kind"], cfg["omega_seed"], F, G, **kw)
    V, s = gpu_lib.fit(X, k, cfg["kind"], cfg["omega_seed"], **kw)
    torch.cuda.synchronize()
    _log("device pass and fit done")
    Fd, Gd = F.cpu().numpy(), G.cpu().numpy()

    om = P.omega(n, k, cfg["kind"], cfg["omega_seed"], cfg.get("p", 64), dtype=dtype)
    ref = _oracle_pass(X, om, dtype)
    r = check_pass(Fd, Gd, ref, MAX_FP32_DEPTH)
    _log(f"pass: {r}")
    _log(f"F rel error {r['rel_F']:.3g} = {r['rel_F'] / r['tol']:.3g} of the stated tolerance "
         f"{r['tol']:.3g}; G {r['rel_G']:.3g} = {r['rel_G'] / r['tol_G']:.3g} of {r['tol_G']:.3g}; "
         f"componentwise ratios F {r['comp_ratio_F']:.3g}, G {r['comp_ratio_G']:.3g}")
    assert r["comp_ratio_F"] <= 1.0 and r["comp_ratio_G"] <= 1.0, r
    assert r["rel_F"] <= r["tol"] and r["rel_G"] <= r["tol_G"], r

    # the fit against the oracle's fit of the same X (Algorithm 2 in FP64)
    Vr, Dr = O.truncated_svd(ref.F, k)
    Vd, sd = V.cpu().numpy(), s.cpu().numpy()
    dF2 = np.linalg.norm(Fd - ref.F, 2)
    sine = O.principal_sines(Vr, Vd).max()
    wedin = subspace_tol(Dr[-1], dF2)
    serr = np.max(np.abs(sd - Dr))
    _log(f"fit: max sine {sine:.3g} (Wedin bound of ||dF||_2 = {dF2:.3g}: {wedin:.3g}; target "
         f"{SINE_TARGET[cfg_id]:g}), sigma max abs err {serr:.3g} (Weyl {dF2:.3g}), "
         f"max rel {np.max(np.abs(sd - Dr) / Dr):.3g}")
    assert sine <= 1.05 * wedin + 1e-12
    assert sine <= SINE_TARGET[cfg_id]
    assert serr <= 1.01 * dF2 + 1e-12 * Dr[0]

    # small stage on the device's own F
    Vf, sf = gpu_lib.factor(F)
    Vfd, sfd = Vf.cpu().numpy(), sf.cpu().numpy()
    Vo, do = O.truncated_svd(Fd, k)
    kappa = do[0] / do[-1]
    assert np.max(np.abs(sfd - do) / do) < 64 * U64 * kappa * k
    assert O.principal_sines(Vo, Vfd).max() < 64 * U64 * kappa * k
    assert np.max(np.abs(Vfd.T @ Vfd - np.eye(k))) < 16 * k * U64
    _log(f"factor: kappa(F) {kappa:.3g}, sigma rel err {np.max(np.abs(sfd - do) / do):.3g}")

    # projection on sampled rows (the full Z, as lspca_transform computes it)
    Z = gpu_lib.transform(X, V)
    torch.cuda.synchronize()
    rng = np.random.default_rng(cfg_id)
    rows = np.sort(rng.choice(m, 64, replace=False))
    rows[-1] = m - 1
    Xr = X[torch.from_numpy(rows).cuda()].double().cpu().numpy()
    Vq = P.round_f32(Vd) if dtype == "f32" else Vd
    zref = O.transform(Xr, Vq)
    u = U64 if dtype == "f64" else U32
    bound = gamma(n, u) * (np.abs(Xr) @ np.abs(Vq))
    if dtype in U16:
        bound = 2 * bound + (1.01 * U16[dtype] ** 2 + U32 + 2.0 ** -24) * (np.abs(Xr) @ np.abs(Vd))
        if dtype == "f16":   # subnormal inputs of the FP16 products (the pass's allowance)
            sub = (np.abs(Xr) < 2.0 ** -14)
            bound = bound + np.where(sub, np.abs(Xr), 0.0) @ np.abs(Vd)
    Zs = Z[torch.from_numpy(rows).cuda()].double().cpu().numpy()
    assert np.all(np.abs(Zs - zref) <= bound + 1e-300)
    _log(f"projection rows within bound (max ratio {np.max(np.abs(Zs - zref) / (bound + 1e-300)):.3g})")
