"""MI355X (gfx950) solver for the tau-preconditioned GMRES time stepper of the
quasi-compact Crank-Nicolson scheme for variable-coefficient Riesz space
fractional diffusion equations.  The compute lives in librsfde.so (HIP); the
Python side only marshals arguments (see rsfde.py)."""
from . import rsfde  # noqa: F401
