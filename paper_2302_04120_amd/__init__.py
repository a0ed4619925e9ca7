"""MI355X-native dimensional lattice Boltzmann hot path (arXiv 2302.04120).

``lbm`` is the thin ctypes binding over the C-ABI library ``liblbm.so``
(HIP kernels for gfx950); ``workloads`` holds the seeded SI inputs shaped like
the paper's cases.  Submodules are imported on demand so that importing the
package never loads the GPU library by itself.
"""
__all__ = ["lbm", "workloads", "adjoint"]
