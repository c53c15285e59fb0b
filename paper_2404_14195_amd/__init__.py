"""MI355X-native meshless pore-flow solvers (arXiv 2404.14195): RBF-FD weights,
artificial-compressibility Navier-Stokes and meshless TRT lattice Boltzmann
steps, permeability and drag, behind the C ABI of libmpf (include/mpf.h)."""
from ._lib import MPF_F32, MPF_F32_KAHAN, MPF_F64, MPF_MIXED, SO_PATH, MPFDiverged, MPFError, build  # noqa: F401

__all__ = ["MPF_F32", "MPF_F32_KAHAN", "MPF_F64", "MPF_MIXED", "SO_PATH", "MPFDiverged", "MPFError", "build"]
