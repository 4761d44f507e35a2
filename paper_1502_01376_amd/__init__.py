"""MI355X-native hybrid Yee-FFT particle-in-cell step (arXiv:1502.01376).

``paper_1502_01376_amd.hpic`` is the Python binding of the C-ABI library
``libhpic.so`` (HIP kernels for gfx950); ``workloads`` holds the seeded input
generators.  Nothing is loaded at import time.
"""
