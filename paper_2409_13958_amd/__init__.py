"""MI355X-native PM-FEM effective-field library (periodic micromagnetic FEM, arXiv 2409.13958).

The compute path is the in-tree shared library ``libpmfem.so`` (host FP64
setup in C++, gfx950 HIP kernels) behind the C ABI declared in
``include/pmfem.h``; ``binding`` only marshals arguments to it with ctypes
and uses PyTorch for device memory and streams.
"""
from .binding import Context, Status, PmfemError, load_library, pgf_eval, TERM_EX, TERM_MS  # noqa: F401
