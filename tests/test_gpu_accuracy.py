"""Stated accuracy of each precision form against the FP64 oracle.

For the shapes of the FP32 / BF16 workloads (n = 4,096, k = 256, sigma_i =
i^-1/2, noise 0.05) and of the FP16 workload (n = 2,048, k = 128, sigma_i =
1/i, noise 0.02), at m = 32,768 rows so that the oracle finishes in seconds,
both as specified (noise-dominated: the noise norm exceeds sigma_1) and with
the signal scaled so that sigma_1 = 20 s (sqrt(m) + sqrt(n)) (signal-
dominated): the GPU fit's basis against the oracle's Lazy SPCA basis on the
same stored values and the same Omega, as

  * the largest principal-angle sine between the two subspaces, checked
    against the Wedin bound of the pass's componentwise error bound
    (tests/helpers.py; vacuous at these sizes), against the Wedin bound of
    the measured error of the same pass's F (plus the small stage's
    rounding), and against 1e-3 for BF16 with refinement;
  * the relative error of pairwise distances after projection, GPU
    (lspca_transform with the GPU basis) against the oracle (the oracle's
    basis), over 2,000 seeded row pairs: reported (Proposition 3 makes them
    depend on the subspace only).

Each case prints one "[accuracy]" line with these figures."""
import numpy as np
import pytest

from oracle import lspca_oracle as O
from oracle import philox as P
from synth import lowrank_np, storage_to_f64
from tests.helpers import pass_bound, subspace_tol, to_device

pytestmark = pytest.mark.gpu

M = 32_768
FAMILIES = {
    "fp32-shape": dict(n=4096, k=256, r=256, spectrum="invsqrt", s=0.05, seed=501),
    "fp16-shape": dict(n=2048, k=128, r=128, spectrum="inv", s=0.02, seed=502),
}
# (family, signal, dtype, omega kind, refine)
CASES = [
    ("fp32-shape", "specified", "f32", "gaussian", True),
    ("fp32-shape", "specified", "bf16", "sparse", True),
    ("fp32-shape", "specified", "bf16", "sparse", False),
    ("fp32-shape", "dominant", "f32", "gaussian", True),
    ("fp32-shape", "dominant", "bf16", "sparse", True),
    ("fp16-shape", "specified", "f16", "gaussian", True),
    ("fp16-shape", "dominant", "f16", "gaussian", True),
]

_DATA = {}


def _data(family, signal, dtype):
    key = (family, signal, dtype)
    if key not in _DATA:
        f = FAMILIES[family]
        scale = 20 * f["s"] * (np.sqrt(M) + np.sqrt(f["n"])) if signal == "dominant" else 1.0
        Xs = lowrank_np(M, f["n"], f["r"], f["spectrum"], f["s"], f["seed"], dtype, scale=scale)
        _DATA.clear()                                 # one matrix alive at a time
        _DATA[key] = (Xs, storage_to_f64(Xs, dtype))
    return _DATA[key]


@pytest.mark.parametrize("family,signal,dtype,kind,refine", CASES)
def test_precision_form_accuracy(gpu_lib, family, signal, dtype, kind, refine):
    import torch
    f = FAMILIES[family]
    n, k = f["n"], f["k"]
    Xs, X64 = _data(family, signal, dtype)
    X = to_device(Xs, dtype)
    seed = 7300 + k
    V, s = gpu_lib.fit(X, k, kind, seed, sparse_p=64, refine=1 if refine else 0)
    om = P.omega(n, k, kind, seed, p=64, dtype=dtype)
    ref = O.lazy_fit(X64, om, k)
    Vg = V.cpu().numpy()
    sine = O.principal_sines(ref["V"], Vg).max()
    bF, _ = pass_bound(X64, om, dtype, refine=refine)
    bound = subspace_tol(ref["sigma"][-1], np.linalg.norm(bF))
    # the same pass's F (the fit's own launch sequence): Wedin with the
    # measured perturbation, plus the small stage's own rounding
    F = torch.zeros((k, n), dtype=torch.float64, device="cuda")
    gpu_lib.accumulate(X, k, kind, seed, F, sparse_p=64, refine=1 if refine else 0)
    dF = np.linalg.norm(F.cpu().numpy() - ref["F"], 2)
    kappa = ref["sigma"][0] / ref["sigma"][-1]
    bound_meas = subspace_tol(ref["sigma"][-1], dF) + 64 * k * 2.0 ** -53 * kappa
    # pairwise distances after projection
    rng = np.random.default_rng(11)
    pairs = rng.integers(0, M, size=(2000, 2))
    pairs = pairs[pairs[:, 0] != pairs[:, 1]]
    rows = np.unique(pairs)
    Zg = gpu_lib.transform(X[torch.from_numpy(rows).cuda()], V).double().cpu().numpy()
    pos = {r: i for i, r in enumerate(rows)}
    idx = np.array([[pos[a], pos[b]] for a, b in pairs])
    dg = O.pairwise_distances(Zg, idx)
    dr = O.pairwise_distances(O.transform(X64[rows], ref["V"]), idx)
    rel = np.abs(dg - dr) / dr
    print(f"[accuracy] {family} {signal} {dtype} {kind} refine={int(refine)}: "
          f"|dF|/|F| {dF / ref['sigma'][0]:.3e}, max sine {sine:.3e} (from |dF|: {bound_meas:.3e}; "
          f"a priori: {bound:.3g}); pairwise-distance rel. error "
          f"max {rel.max():.3e} median {np.median(rel):.3e}", flush=True)
    assert sine <= bound + 1e-12
    assert sine <= bound_meas
    if dtype == "bf16" and refine:
        assert sine < 1e-3
