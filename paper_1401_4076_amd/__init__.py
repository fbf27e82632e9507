"""MI355X (gfx950) implementation of the equilibrium parallel multicanonical
iteration of Zierenberg, Wiedenmann and Janke (arXiv:1401.4076) for the 2D and
3D lattice gas.  The compute path is libmuca.so (hand-written HIP kernels
behind the C ABI of include/muca.h); `muca` is its Python binding."""
