"""Plain, slow FP64 CPU oracle for the tau-preconditioned GMRES time stepper.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import or call anything in this package.  It
shares no code with the GPU library and imports nothing from it.
"""
from .rsfde_oracle import *  # noqa: F401,F403
