"""TT-IGA on MI355X: HIP kernels behind a C ABI (include/ttiga.h) and a ctypes binding.

Import ``paper_2509_13224_amd.ttiga`` for the binding; ``build.py`` compiles the
library in-tree for gfx950.
"""
