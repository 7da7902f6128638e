"""Philox4x32-10 counter-based generator and the random test matrix Omega.

TEST INFRASTRUCTURE ONLY. This module belongs to the FP64 CPU oracle. Only the
test suite, the smoke check and the benchmark's CPU-baseline leg may import it;
the library never does, and it shares no code with the library.

The paper draws Omega but names no generator (Sec. I-A, eq. (rp) and the
paragraph after it: Gaussian entries N(0,1), or the very sparse {-1,0,+1}
entries with probabilities {1/(2p), 1-1/p, 1/(2p)}). To make the library and
the oracle draw the same Omega from a seed, both implement one published
counter-based generator independently:

  Philox4x32-10: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw,
  "Parallel random numbers: as easy as 1, 2, 3", SC'11 (Sec. 4 and Table 2).

Omega specification (the same text sits in the public C header):
  key      = (seed & 0xffffffff, seed >> 32)
  Gaussian : entry pair (j, 2q), (j, 2q+1) from one call with counter
             (q, j & 0xffffffff, j >> 32, 0x47415553).  With x0..x3 the four
             output words, u1 = ((x1*2^32 + x0) >> 11) * 2^-53 + 2^-54 and
             u2 = ((x3*2^32 + x2) >> 11) * 2^-53, the Box-Muller pair
             r = sqrt(-2 ln u1), Omega[j,2q] = r cos(2 pi u2),
             Omega[j,2q+1] = r sin(2 pi u2), all in FP64.
  Very sparse (p a power of two): entries (j, 4q+t), t = 0..3, from one call
             with counter (q, j & 0xffffffff, j >> 32, 0x53505253); word x_t
             gives +1 if x_t < 2^32/(2p), -1 if x_t < 2^32/p, else 0.
  Lower precision: the FP64 Gaussian value is rounded to FP32 (round to
             nearest even) and, for BF16/FP16 data, from FP32 to that type
             (round to nearest even). Sparse entries are exact in every type.
"""
import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)

TAG_GAUSSIAN = 0x47415553
TAG_SPARSE = 0x53505253


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds (Salmon et al., SC'11, Sec. 4).

    ctr: integer array (..., 4) of 32-bit words; key: pair of 32-bit words,
    or an array (..., 2) broadcastable against ctr. Returns uint32 (..., 4).
    One round maps (c0,c1,c2,c3) with key (k0,k1) to
    (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0));
    the key is bumped by the Weyl constants (W0, W1) between rounds.
    """
    c = np.asarray(ctr, dtype=np.uint64) & _MASK
    k = np.asarray(key, dtype=np.uint64) & _MASK
    c0, c1, c2, c3 = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
    k0 = np.broadcast_to(k[..., 0], c0.shape).copy()
    k1 = np.broadcast_to(k[..., 1], c0.shape).copy()
    for rnd in range(10):
        if rnd:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0          # < 2^64, exact in uint64
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def _key(seed):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return np.array([seed & 0xFFFFFFFF, seed >> 32], dtype=np.uint64)


def _counters(n, blocks, tag):
    j = np.arange(n, dtype=np.uint64)[:, None]
    q = np.arange(blocks, dtype=np.uint64)[None, :]
    ctr = np.empty((n, blocks, 4), dtype=np.uint64)
    ctr[..., 0] = q
    ctr[..., 1] = j & _MASK
    ctr[..., 2] = j >> np.uint64(32)
    ctr[..., 3] = tag
    return ctr


def gaussian_omega(n, k, seed):
    """FP64 Gaussian Omega (n x k), entries iid N(0,1) (Sec. I-A)."""
    blocks = (k + 1) // 2
    x = philox4x32_10(_counters(n, blocks, TAG_GAUSSIAN), _key(seed)).astype(np.uint64)
    a = ((x[..., 1] << np.uint64(32)) | x[..., 0]) >> np.uint64(11)
    b = ((x[..., 3] << np.uint64(32)) | x[..., 2]) >> np.uint64(11)
    u1 = a.astype(np.float64) * 2.0 ** -53 + 2.0 ** -54
    u2 = b.astype(np.float64) * 2.0 ** -53
    r = np.sqrt(-2.0 * np.log(u1))
    th = 2.0 * np.pi * u2
    out = np.empty((n, 2 * blocks), dtype=np.float64)
    out[:, 0::2] = r * np.cos(th)
    out[:, 1::2] = r * np.sin(th)
    return out[:, :k]


def sparse_omega(n, k, seed, p=64):
    """Very sparse Omega (n x k) with entries in {-1, 0, +1} (Sec. I-A).

    P(+1) = P(-1) = 1/(2p), P(0) = 1 - 1/p; p must be a power of two so the
    thresholds on a uniform 32-bit word give these probabilities exactly.
    """
    p = int(p)
    if p < 1 or p & (p - 1) or p > 2 ** 30:
        raise ValueError("p must be a power of two in [1, 2^30]")
    blocks = (k + 3) // 4
    x = philox4x32_10(_counters(n, blocks, TAG_SPARSE), _key(seed)).astype(np.uint64)
    t_plus = np.uint64(2 ** 32 // (2 * p))
    t_minus = np.uint64(2 ** 32 // p)
    val = np.where(x < t_plus, 1.0, np.where(x < t_minus, -1.0, 0.0))
    return val.reshape(n, 4 * blocks)[:, :k]


def round_f32(a):
    """FP64 -> FP32, round to nearest even, returned as FP64."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_bf16(a):
    """FP64 -> FP32 -> BF16 (round to nearest even at each step), as FP64."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) >> np.uint64(16) << np.uint64(16)
    return (u & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32).astype(np.float64)


def round_f16(a):
    """FP64 -> FP32 -> FP16 (round to nearest even at each step), as FP64."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    return f.astype(np.float16).astype(np.float64)


ROUNDERS = {"f64": lambda a: np.asarray(a, dtype=np.float64),
            "f32": round_f32, "bf16": round_bf16, "f16": round_f16}


def omega(n, k, kind, seed, p=64, dtype="f64"):
    """Omega as the library's compute type holds it, returned in FP64.

    kind: "gaussian" or "sparse"; dtype: the data type of X ("f64", "f32",
    "bf16", "f16"), which is the type Omega is rounded to.
    """
    if kind == "gaussian":
        om = gaussian_omega(n, k, seed)
    elif kind == "sparse":
        om = sparse_omega(n, k, seed, p)
    else:
        raise ValueError(kind)
    return ROUNDERS[dtype](om)
