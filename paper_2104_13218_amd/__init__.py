"""MI355X (gfx950) library for the stochastic Chebyshev-moment typicality method
(arXiv:2104.13218): HIP kernels behind the C ABI of include/kpm.h, with a thin
ctypes binding in `kpm`."""
