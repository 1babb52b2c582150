"""FP64 CPU oracle for Fourier-Galerkin FFT homogenization (arXiv 1508.02045).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's CPU-baseline leg
are the only users.  The GPU product path never imports this package.
"""
