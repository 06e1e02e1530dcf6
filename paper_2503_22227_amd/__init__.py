"""MI355X-native RNS-FHE hot path: negacyclic NTT and hybrid key switching
(HMult+Relin, HRotate, rescale, modulus switch) in hand-written HIP for gfx950,
behind the C ABI of include/rnsfhe.h.  This package holds the ctypes binding
(``fhe``), the prime-chain derivation (``params``) and the build script."""
from . import params  # noqa: F401
from ._lib import RFError, lib  # noqa: F401  (raises ImportError when the library is not built)
from .fhe import BatchPlan, Context  # noqa: F401

__all__ = ["BatchPlan", "Context", "RFError", "params", "lib"]
