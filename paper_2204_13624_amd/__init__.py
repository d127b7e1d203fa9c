"""MI355X-native FFT-based finite-strain homogenization with composite boxels.

The compute path is libcombo.so (HIP kernels for gfx950 behind the C-ABI of
include/combo.h); `combo` is its Python binding and `synth` the seeded input
generator.  Importing the package loads nothing; the library is loaded on the
first call into `combo`.
"""
__all__ = ["combo", "synth", "build"]
