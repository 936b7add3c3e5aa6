"""MI355X-native double-MRT lattice Boltzmann solver for 3-D natural
convection in a cubic cavity (Li, Yang & Zhang, arXiv:1511.04633).

The compute path is the HIP library ``liblbmx.so`` (C-ABI in
``include/lbmx.h``); ``lbmx`` is its Python binding.  Importing the package
loads nothing; the binding loads the library on first use and raises if it
is not built.
"""

__all__ = ["lbmx", "inputs"]
