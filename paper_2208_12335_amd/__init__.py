"""MI355X-native NAO real-space grid integration (density update, Hamiltonian/overlap
integration and their backward) behind the C ABI of include/aims_grid.h.

The Python layer only marshals arguments; the computation runs in the gfx950 kernels of
``libaimsgrid.so`` (built by ``paper_2208_12335_amd.build.build()``)."""
from .grid import AimsEnergy, AimsGrid, StepGraph  # noqa: F401
from ._lib import AimsError, PRECISION  # noqa: F401
