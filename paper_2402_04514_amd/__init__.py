"""MI355X (gfx950) implementation of the per-stage sweep of the graph-based
DG scheme of arXiv 2402.04514 for the compressible Euler equations.

``gdg``        binding of the C-ABI library libgdg.so (HIP kernels)
``workloads``  seeded synthetic inputs shaped like the paper's test problems
``build``      hipcc build of libgdg.so
"""
