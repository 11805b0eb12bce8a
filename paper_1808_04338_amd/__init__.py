"""MI355X-native hot path of the dual-porosity oil-water simulator.

The compute lives in ``libdpsim.so`` (hand-written HIP for gfx950 behind the C
ABI of ``include/dpsim.h``); this package only loads it and marshals
arguments.  PyTorch supplies device memory and streams.
"""
from ._lib import DpError, load  # noqa: F401
from .sim import Sim, batch_timestep, footprint, make_desc  # noqa: F401
from .serve import Request, serve  # noqa: F401,E402
