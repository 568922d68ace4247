"""MI355X-native MR-STORM control step (arXiv 2602.10114): HIP kernels behind
a C-ABI library, with a thin ctypes binding."""
