"""MI355X-native semiempirical (NDDO) CIS / TDHF excited states.

The computation lives in libseqx.so (HIP for gfx950, C ABI in include/seqx.h);
`seqx` is its thin ctypes binding.  Import does not touch the GPU.
"""
from . import seqx  # noqa: F401
from .seqx import (BF16, BF16X3, CIS, FP32, FP64, GUESS_GAP, GUESS_LEARNED, GUESS_USER, TDHF,  # noqa: F401
                   Context, Job, SeqxError, load_library, params_table, validate)

__all__ = ["seqx", "Context", "Job", "SeqxError", "load_library", "params_table", "validate",
           "CIS", "TDHF", "FP64", "FP32", "BF16", "BF16X3", "GUESS_GAP", "GUESS_LEARNED", "GUESS_USER"]
