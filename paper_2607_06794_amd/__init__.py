"""MI355X-native hot path of the drying-droplet lattice Boltzmann simulation.

Two-component Shan-Chen D3Q19 fluid with wettability-patterned walls, a
reservoir plane for evaporation and rigid nanowire rods, as hand-written HIP
kernels for gfx950 behind the C ABI of include/lbm.h (liblbm.so).

Importing the package does not load the library; ``sim.Lattice`` and
``_lib.load()`` do, and fail loudly when it has not been built.
"""

__all__ = ["inputs", "sim", "build"]
