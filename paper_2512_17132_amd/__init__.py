"""MI355X (gfx950) implementation of the 2D TMz FDTD hot path of arXiv 2512.17132:
hand-written HIP kernels behind the C ABI of include/fdtd.h (libfdtd.so), with a
thin ctypes binding (``fdtd``) and a torch.autograd wrapper (``autograd``)."""
