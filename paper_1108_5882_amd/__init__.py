"""MI355X (gfx950) partial-wave-analysis likelihood: HIP kernels behind a C ABI.

Implements the unbinned negative log-likelihood of Berger, "Partial Wave
Analysis using Graphics Cards" (Section 2, Eq. 1-3) and its gradient with
respect to the complex production amplitudes, over precomputed decay
amplitudes held in GPU memory.  The arithmetic runs in the library's HIP
kernels (csrc/); this package is the ctypes binding.  Importing the package
does not load the library; creating a Context does, and raises if it is
missing.
"""
from ._lib import (Context, DomainError, KinContext, Mlp, MultiFit, PwaError, EXPORTS, LIB_PATH, load,  # noqa: F401
                   nll_grad_noalloc)

__all__ = ["Context", "DomainError", "KinContext", "Mlp", "MultiFit", "PwaError", "EXPORTS", "LIB_PATH", "load",
           "nll_grad_noalloc"]
