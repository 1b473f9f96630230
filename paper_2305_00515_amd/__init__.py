"""MI355X-native four-directional 5x5 Sobel operator (Chang et al., arXiv 2305.00515).

The operator runs in hand-written HIP kernels behind the C ABI declared in
``include/sobel4x5.h``; this package is a thin ctypes binding over that
library (``libsobel4x5.so``, built in-tree), plus a torch.autograd.Function for
the fp32 path and seeded synthetic input generators (``synth``).

The binding is imported lazily so that ``paper_2305_00515_amd.synth`` can be
used without loading the GPU library.
"""
__all__ = [
    "sobel4x5_u8", "sobel4x5_batched", "Plan", "sobel4x5_f32_fwd", "sobel4x5_f32_bwd",
    "Sobel4x5Magnitude", "sobel4x5_magnitude", "SobelError",
    "BORDER_REPLICATE", "BORDER_VALID", "DIR_NONE", "DIR_S16", "DIR_S32",
]


def __getattr__(name):
    if name in ("Sobel4x5Magnitude", "sobel4x5_magnitude"):
        from . import autograd
        return getattr(autograd, name)
    if name in __all__:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
