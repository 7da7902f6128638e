"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no arithmetic of the method: it only draws data matrices
(low-rank plus noise, X = A diag(sigma) B^T + E with A, B orthonormalised
Gaussian matrices and E iid N(0, s^2)), probe vectors and request sizes, and
converts between storage types. It stands in for the paper's datasets
(Sec. IV-A malware features, Sec. V-A TF-IDF), which are not available.
"""
from .lowrank import (  # noqa: F401
    CONFIGS, config, sigmas, lowrank_np, lowrank_torch, to_storage_np,
    storage_to_f64, request_sizes, random_orthonormal_np,
)
from .sparse import (  # noqa: F401
    CSR_CONFIG, FEATURES, DENSITY, column_density, csr_np, csr_torch,
)
