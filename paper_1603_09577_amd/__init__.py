"""MI355X-native MRT lattice Boltzmann sweep for nonlinear anisotropic
convection-diffusion equations (Chai, Shi & Guo).

The compute path is the C-ABI library ``liblbm.so`` (HIP kernels for gfx950)
declared in ``include/lbm.h``; ``paper_1603_09577_amd.lbm`` is its thin ctypes
binding.  Importing this package loads nothing; the binding raises when the
library has not been built.
"""
