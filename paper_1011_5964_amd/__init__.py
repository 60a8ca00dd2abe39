"""MI355X-native lagged-diffusivity TV deblurring with reflective and
anti-reflective boundary conditions and fast-transform preconditioners.

The compute path is the HIP/C-ABI library libtvdeblur.so (csrc/); this package
is its thin Python binding.  Importing the package does not load the library;
`paper_1011_5964_amd.lib` does, and fails loudly when it is missing.
"""

__all__ = ["lib", "synth"]
