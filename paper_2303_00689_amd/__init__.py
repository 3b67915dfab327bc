"""MI355X-native (gfx950, HIP) per-step electronic hot path of shadow KSA-XL-BOMD.

The compute lives in libxlbomd.so (C ABI in include/xlbomd.h); ``binding``
marshals torch device tensors into it.  Build with ``build.build()``.
"""

__all__ = ["binding", "build"]
