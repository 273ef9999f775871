"""paper_1908_06972_amd: RNS-CKKS primitives of PrivFT (arXiv:1908.06972) as
HIP kernels for AMD Instinct MI355X (gfx950), behind the C ABI of
include/pft.h.  `native` is the ctypes binding, `ckks` a thin Python front end
that allocates device buffers with torch."""

from . import native  # noqa: F401
