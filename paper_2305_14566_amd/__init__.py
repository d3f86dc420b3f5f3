"""MI355X (gfx950) slide-wise Omni-Seg hot path: HIP kernels behind a C ABI.

The package holds the HIP sources (csrc/), the build script and the ctypes
binding.  Importing it does not load the library; omniseg.lib() does, and
fails loudly when the built libomniseg.so is missing.
"""
