"""MI355X (gfx950) state / adjoint solver for the Darcy / Boussinesq / convection-
diffusion model of arXiv 1904.00182, behind a C ABI (include/nc.h) with a thin
ctypes binding (nc.py)."""

__all__ = ["nc", "inputs", "workloads"]
