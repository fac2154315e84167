"""MI355X-native NOHAP/OUCS3 compressible Navier-Stokes hot path.

The GPU library (``libnopcs.so``: HIP kernels for gfx950 behind a C ABI declared
in ``include/nopcs.h``) is loaded lazily by ``paper_2203_00879_amd.nopcs``;
importing this package alone does not touch the GPU.
"""
