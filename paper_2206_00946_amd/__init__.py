"""MI355X-native coupled D3Q19 / D3Q7 thermal pseudopotential lattice
Boltzmann step (Huang, Wang, He & Huang, arXiv 2206.00946): a HIP library
for gfx950 behind the C ABI of include/lbm3d.h, with a ctypes binding."""
from .lbm3d import (Lbm3D, LbmError, LbmParams, from_workload, load_library, make_params,  # noqa: F401
                    params_from_workload, evaporated_mass_function, FP64, FP32_DEV, FP16_DEV, BF16_DEV, PERIODIC, WALL, PRESSURE)
