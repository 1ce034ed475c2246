"""MI355X-native Fourier PlenOctree render and fine-tune path.

The compute path is libfpo.so (C ABI in include/fpo.h; HIP kernels for
gfx950).  `_lib` is its ctypes binding; `synth` generates seeded synthetic
inputs.  Importing this package does not load the library; the first call
into `_lib` does, and raises if it has not been built.
"""
