"""Helpers shared by the GPU parity tests (inputs are generated on the host from
seeds and copied to the device; expected values come from the oracle only)."""
import sys

import numpy as np

import oracle as O
from paper_2404_10221_amd import rsfde as R


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64).ravel()).to("cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().to("cpu").numpy().astype(np.float64)


def empty(n):
    import torch
    return torch.empty(int(n), dtype=torch.float64, device="cuda")


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def solver_for(inst, ebar=None, **over):
    p = R.params_from_instance(inst, **over)
    if ebar is not None:
        p.e_min, p.e_max = ebar
    S = R.Solver([p])
    R.rsfde_set_fields(S.h, 0, inst.e, inst.f, inst.psi)
    return S


def oracle_problem(inst):
    return O.OracleProblem(inst)


# Tolerance of the oracle's "tight" solves: the reference a solver form is held to
# when it reaches the stopping bound along another Krylov sequence than the
# oracle's FP64 GMRES (the mixed form), so that the comparison measures that form's
# own error and not the oracle's distance cond * rtol from the exact solution.
TIGHT_RTOL = 1e-13


def tight(inst):
    from dataclasses import replace
    return replace(inst, rtol=TIGHT_RTOL, max_cycles=max(inst.max_cycles, 20))
