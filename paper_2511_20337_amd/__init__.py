"""MI355X-native (gfx950, HIP) finite-volume ideal-MHD step.

The hot path — primitive recovery, PLM reconstruction, HLL/HLLD Riemann
fluxes, upwind constrained-transport EMF, SSP-RK2 update and the CFL time
step — lives in hand-written HIP kernels behind the C ABI of include/mhd.h
(libmhd.so). ``mhd`` is the ctypes binding; ``workloads`` holds the seeded
initial conditions; ``adjoint`` the autograd wrapper with step checkpointing.
"""
from . import workloads  # noqa: F401
