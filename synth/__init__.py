"""Seeded synthetic inputs for the dual-porosity oil-water model.

This package only draws and lays out *data*: grids, permeability and porosity
fields, well placements, fluid constants and timestep schedules.  It holds none
of the simulator's arithmetic (no transmissibility, no well index, no residual),
so both the CPU oracle and the GPU library can read the same inputs without
sharing any code of the method.
"""
from .models import (  # noqa: F401
    MD,
    DAY,
    base_physics,
    make_model,
    model_small,
    model_layered,
    model_channelised,
    model_channelised_fp32,
    served_size_classes,
    served_stream,
    served_realisation,
    model_1d,
    model_single_cell,
    model_tiny,
    random_state,
)
from .examples import paper_example  # noqa: F401
