"""MI355X-native DPSNN: mixed time/event-driven simulation of grids of cortical columns of
LIF neurons with spike-frequency adaptation (arXiv:1511.09325), as hand-written HIP
kernels for gfx950 behind the C ABI of include/dpsnn.h.

Public Python surface:
    Simulation           -- one sim_t handle (plain or batched networks)
    workloads            -- the seeded synthetic workloads (parameter sets, no arithmetic)
    build                -- compile libdpsnn.so with hipcc for gfx950
"""
from . import workloads
from ._lib import (DELIVERY_ARRIVAL, DELIVERY_AUTO, DELIVERY_PUSH, DpsnnError, EXPORTS,
                   LIB_PATH)
from .sim import Simulation

__all__ = ["Simulation", "workloads", "DpsnnError", "EXPORTS", "LIB_PATH", "DELIVERY_AUTO",
           "DELIVERY_ARRIVAL", "DELIVERY_PUSH"]
