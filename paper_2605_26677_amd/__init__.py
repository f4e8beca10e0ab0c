"""MI355X library for the total-Lagrangian vectorial lattice Boltzmann method (D2Q4 lattice,
six-component vector populations) of Feng & Chu, arXiv 2605.26677.

The compute path is the HIP library ``liblbm.so`` (C ABI in include/lbm.h); ``_lib`` holds
its ctypes binding, ``solver`` the device-resident state, ``rollout`` the differentiable
rollout with checkpointed adjoint.  Build with ``python -m paper_2605_26677_amd.build``.
"""
from . import _lib  # noqa: F401

__all__ = ["_lib"]
