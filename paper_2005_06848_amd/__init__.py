"""MI355X-native CFUST mixture EM: Python binding of the HIP library.

Argument marshalling only: every step of the E-step, M-step, log-likelihood
and EM fit runs in the HIP kernels of ``libcfust.so`` (see include/cfust.h).
PyTorch supplies device memory and the current HIP stream.  There is no CPU
fallback: if the library is missing the import of ``native`` fails loudly.
"""
from . import inputs  # noqa: F401  (seeded generators; no method arithmetic)

__all__ = ["inputs"]
