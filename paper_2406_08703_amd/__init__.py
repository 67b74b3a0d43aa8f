"""MI355X-native forward model and gradient of the dLux joint phase-retrieval / flat-field path.

The compute lives in libdlx.so (HIP for gfx950, C ABI in include/dlx.h);
``dlx`` is its ctypes binding and ``psf`` a torch wrapper (device memory,
streams, autograd). Nothing here falls back to a CPU implementation.
"""
from .psf import BatchPlan, CapturedEval, EvalBuffers, Geometry, PsfPlan, evaluate, psf_loss  # noqa: F401
