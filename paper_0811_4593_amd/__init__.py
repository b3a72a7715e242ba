"""MI355X-native D3Q19 lattice Boltzmann with the on-site velocity boundary
condition of Hecht & Harting (arXiv:0811.4593).

The product is the HIP library ``liblbm.so`` (C ABI in ``include/lbm.h``);
``paper_0811_4593_amd.lbm`` is its thin ctypes binding.
"""
from . import lbm  # noqa: F401
from .lbm import LBMError, Lattice  # noqa: F401
