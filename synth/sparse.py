"""Sparse feature matrices in CSR form, seeded.

They stand in for the malware feature matrix of Experiment 1 (Data and
Method): 98,450 mostly binary features at mean density 0.0244, stored as
horizontal slices. Recipe, identical for the numpy and the torch generator
(the two draw from different random streams, so their matrices differ):

  * column j (after a seeded shuffle of the feature order) has density
    rho_j = min(1, c (rank_j + 1)^-alpha), a power law in the feature's
    popularity rank; c is set by bisection so that mean(rho_j) = density;
  * entry (i, j) is present with probability rho_j, independently;
  * a present entry is 1 (binary feature) with probability `binary`, else
    uniform in (0, 1];
  * rows are stored with sorted, unique columns (rowptr int64, colidx int32,
    values FP32 or FP64).

No arithmetic of the method is done here.
"""
import numpy as np

# Experiment 1's matrix shape and density
FEATURES = 98_450
DENSITY = 0.0244
CSR_CONFIG = dict(name="sparse-malware-like", m=131_072, n=FEATURES, density=DENSITY, alpha=0.5,
                  binary=0.9, k=500, kind="sparse", p=64, dtype="f32", data_seed=17090706,
                  omega_seed=7181)


def column_density(n, density, alpha, rng_perm):
    """rho_j of the recipe above (rng_perm: a permutation of range(n))."""
    w = (np.arange(n, dtype=np.float64) + 1.0) ** -alpha
    lo, hi = 0.0, 1.0 / w[-1]
    for _ in range(200):
        c = 0.5 * (lo + hi)
        if np.minimum(1.0, c * w).mean() < density:
            lo = c
        else:
            hi = c
    rho = np.minimum(1.0, 0.5 * (lo + hi) * w)
    return rho[np.argsort(rng_perm)]        # column j gets the density of its rank


def csr_np(m, n, density=DENSITY, seed=0, alpha=0.5, binary=0.9, dtype="f32", rows_per_chunk=4096):
    """Seeded CSR matrix (numpy): returns rowptr (m + 1 int64), colidx
    (int32), values (float32 or float64)."""
    rng = np.random.default_rng(seed)
    rho = column_density(n, density, alpha, rng.permutation(n))
    vdt = np.float32 if dtype == "f32" else np.float64
    counts, cols, vals = [], [], []
    for r0 in range(0, m, rows_per_chunk):
        rows = min(rows_per_chunk, m - r0)
        hit = rng.random((rows, n)) < rho
        ri, cj = np.nonzero(hit)
        counts.append(np.bincount(ri, minlength=rows))
        cols.append(cj.astype(np.int32))
        v = np.where(rng.random(cj.size) < binary, 1.0, 1.0 - rng.random(cj.size))
        vals.append(v.astype(vdt))
    rowptr = np.zeros(m + 1, dtype=np.int64)
    rowptr[1:] = np.cumsum(np.concatenate(counts))
    return rowptr, np.concatenate(cols), np.concatenate(vals)


def csr_torch(m, n, density=DENSITY, seed=0, alpha=0.5, binary=0.9, dtype="f32", device="cuda",
              rows_per_chunk=2048):
    """Seeded CSR matrix generated on the device (torch): same recipe as
    csr_np, for sizes where the host generator is too slow."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    perm = torch.randperm(n, generator=g, device=device).cpu().numpy()
    rho = torch.from_numpy(column_density(n, density, alpha, perm).astype(np.float32)).to(device)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    counts, cols, vals = [], [], []
    for r0 in range(0, m, rows_per_chunk):
        rows = min(rows_per_chunk, m - r0)
        hit = torch.rand((rows, n), generator=g, device=device) < rho
        ri, cj = torch.nonzero(hit, as_tuple=True)
        counts.append(torch.bincount(ri, minlength=rows))
        cols.append(cj.to(torch.int32))
        u = torch.rand(cj.numel(), generator=g, device=device, dtype=torch.float64)
        b = torch.rand(cj.numel(), generator=g, device=device, dtype=torch.float64)
        vals.append(torch.where(b < binary, torch.ones_like(u), 1.0 - u).to(tdt))
        del hit, ri
    rowptr = torch.zeros(m + 1, dtype=torch.int64, device=device)
    rowptr[1:] = torch.cumsum(torch.cat(counts), 0)
    return rowptr, torch.cat(cols), torch.cat(vals)
