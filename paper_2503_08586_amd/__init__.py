"""MI355X-native batched lens-modelling log-likelihood (SIE + shear, Sersic light).

The compute path is a C-ABI shared library of hand-written HIP kernels for
gfx950 (``csrc/``); ``binding`` marshals numpy arrays and torch device memory
into it.  Importing this package loads nothing; ``binding.load()`` loads the
library and fails loudly if it has not been built.
"""
__all__ = ["binding", "synth", "build"]
