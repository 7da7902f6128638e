"""FP64 CPU oracle for Lazy SPCA and SPCA (arXiv 1709.07175).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the library. It shares no code with the
HIP path.
"""
from . import philox, lspca_oracle  # noqa: F401
