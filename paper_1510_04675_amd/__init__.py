"""MI355X-native (gfx950, HIP) library for the rethermalization path of
multiscale Monte Carlo equilibration of pure SU(3) Yang-Mills theory
(arXiv:1510.04675): Cabibbo-Marinari heat bath with Kennedy-Pendleton draws,
overrelaxation, HMC, prolongation, Wilson flow and clover charge.

The Python layer only marshals arguments into the C ABI of
``lib/libmsmc.so`` (declared in ``include/msmc.h``); PyTorch supplies device
memory and streams.
"""
from .capi import *  # noqa: F401,F403
from .capi import Field, SU3Error, hb_params, lib  # noqa: F401
