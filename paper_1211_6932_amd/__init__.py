"""MI355X-native improved MRT pseudopotential lattice Boltzmann (D2Q9).

Method: Li, Luo & Li, "Lattice Boltzmann modeling of multiphase flows at large
density ratio with an improved pseudopotential model" (arXiv:1211.6932).

The product is the HIP library ``liblbmp.so`` (C ABI in ``include/lbmp.h``);
``paper_1211_6932_amd.lbmp`` is its ctypes binding.
"""
__all__ = ["lbmp", "build"]
