"""MI355X (gfx950) implementation of the P-TRT lattice Boltzmann hot path.

The fused per-node stream-and-collide update of arXiv 2602.06686 (Eq. PTRT)
on D2Q9 and D3Q19 lattices, as hand-written HIP kernels behind the C
interface in ``include/ptrt.h`` (``libptrt.so``).  ``ptrt`` is the Python
binding (``from paper_2602_06686_amd import ptrt``); ``build`` compiles the
library.
"""
__all__ = ["ptrt", "build"]
