"""MI355X-native Fourier-Galerkin FFT homogenization (arXiv 1508.02045).

The compute path lives in the HIP library ``libfgh.so`` (C-ABI declared in include/fgh.h);
``paper_1508_02045_amd.fgh`` is its thin ctypes binding.  Importing this package loads nothing.
"""
