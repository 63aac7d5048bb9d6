"""MI355X (gfx950) p-multigrid Poisson solver for nodal DG on Cartesian grids.

The solver lives in ``libdgmg.so`` (hand-written HIP behind the C ABI of
``include/dgmg.h``); ``paper_1603_02524_amd.dgmg`` is its ctypes binding.
Importing this package loads nothing; ``dgmg.load_library`` raises if the
library has not been built.
"""

__all__ = ["dgmg", "build_lib"]
