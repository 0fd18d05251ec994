"""MI355X-native BMMC permutations (paper arxiv 2306.07795) behind a C ABI.

The compute path is libbmmc.so (HIP kernels for gfx950 plus a C++ host
planner); ``binding`` is its thin ctypes face.  Importing this package loads
nothing; the first call into ``binding`` loads the library and fails loudly
if it is missing.
"""
from . import binding  # noqa: F401
from .binding import BmmcError  # noqa: F401
