"""MI355X-native stepper for the two-variable Oregonator reaction-diffusion
model (Stovold, RDCSim, arXiv 1901.06535, Sec. 2, Eq. (1)).

The compute path is the C-ABI library ``librdc.so`` (hand-written HIP for
gfx950) declared in ``include/rdc.h``; ``paper_1901_06535_amd.rdc`` is its
thin Python binding.  ``paper_1901_06535_amd.inputs`` draws seeded synthetic
inputs.  Importing this package loads nothing; the binding loads the library
on first use and fails loudly if it has not been built.
"""
__all__ = ["inputs", "rdc"]
