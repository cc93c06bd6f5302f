"""MI355X-native hot path of the matrix-free Rosenbrock-Krylov (ROK) integrator.

The kernels live in librok.so (HIP for gfx950, C-ABI in include/rok.h);
`paper_1607_06834_amd.rok` is the Python binding.
"""
from .rok import Rok, RokError, load_library, make_tableau  # noqa: F401
