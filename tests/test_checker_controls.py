"""Controls of the full-size pass checker (tests/helpers.check_pass), on the
CPU: an FP32 emulation of the pass with the library's accumulation
structure (FP32 sketch; FP32 partial sums of F and G over at most `depth`
rows; the partials added in FP64) passes, and plausible device mistakes
fail it -- one partial's rows dropped (a lost split), one partial added twice,
rows past an index wrapped onto earlier rows (an integer overflow), and the
sketch of another Omega. The emulation uses numpy's FP32 products, whose
summation order differs from the device's; the error model covers any
order."""
import numpy as np
import pytest

from oracle import philox as P
from synth import lowrank_np, storage_to_f64
from tests.helpers import PassReference, check_pass

M, N, K, DEPTH = 32768, 256, 16, 4096


def _data():
    Xs = lowrank_np(M, N, 16, "invsqrt", 0.05, 11, "f32")
    om = P.omega(N, K, "gaussian", 5, dtype="f32")
    return Xs, om


def _emulate(X32, om32, depth):
    """F, G and the FP64 list of FP32 partials, as the library sums them."""
    Y = X32 @ om32                                    # FP32 sketch
    Fp, Gp = [], []
    for r0 in range(0, X32.shape[0], depth):
        Yc, Xc = Y[r0:r0 + depth], X32[r0:r0 + depth]
        Fp.append((Yc.T @ Xc).astype(np.float64))     # FP32 partial sums
        Gp.append((Yc.T @ Yc).astype(np.float64))
    return Fp, Gp


def _reference(Xs, om):
    ref = PassReference(om, "f32")
    X64 = storage_to_f64(Xs, "f32")
    for r0 in range(0, M, 8192):
        ref.add(X64[r0:r0 + 8192])
    return ref


@pytest.fixture(scope="module")
def case():
    Xs, om = _data()
    return Xs, om, _reference(Xs, om), _emulate(Xs, om.astype(np.float32), DEPTH)


def test_checker_accepts_the_fp32_pass(case):
    _, _, ref, (Fp, Gp) = case
    r = check_pass(sum(Fp), sum(Gp), ref, DEPTH)
    assert r["ok"], r
    # the stated norm tolerance is not vacuous: the emulated error uses a
    # visible share of it
    assert r["rel_F"] > 1e-3 * r["tol"], r


@pytest.mark.parametrize("mistake", ["dropped_partial", "partial_twice", "index_wrap", "other_omega"])
def test_checker_rejects_device_mistakes(case, mistake):
    Xs, om, ref, (Fp, Gp) = case
    if mistake == "dropped_partial":
        F, G = sum(Fp[:-3] + Fp[-2:]), sum(Gp[:-3] + Gp[-2:])
    elif mistake == "partial_twice":
        F, G = sum(Fp) + Fp[2], sum(Gp) + Gp[2]
    elif mistake == "index_wrap":
        # rows from M/2 on read as rows from 0 on
        Xw = np.concatenate([Xs[:M // 2], Xs[:M // 2]])
        Fw, Gw = _emulate(Xw, om.astype(np.float32), DEPTH)
        F, G = sum(Fw), sum(Gw)
    else:
        om2 = P.omega(N, K, "gaussian", 6, dtype="f32")
        Fo, Go = _emulate(Xs, om2.astype(np.float32), DEPTH)
        F, G = sum(Fo), sum(Go)
    r = check_pass(F, G, ref, DEPTH)
    assert not r["ok"], (mistake, r)
    assert r["rel_F"] > 10 * r["tol"], (mistake, r)
