"""Edge and degenerate cases of the GPU path against the oracle: the smallest and
largest transform lengths, an axis without fractional diffusion (kappa_i = 0), a
zero right-hand side, GMRES(1), a zero start, a solve that hits its cycle limit,
and alpha = 2 with constant e (B P = A: one iteration)."""
from dataclasses import replace

import numpy as np
import pytest

import oracle as O
from paper_2404_10221_amd import rsfde as R
from rsfde_workloads import FieldSpec, Instance, config, with_grid

from gpu_helpers import dev, empty, host, rel, say, solver_for

pytestmark = pytest.mark.gpu


def _inst(d, n, M=3, **kw):
    base = dict(name="edge", d=d, n=tuple(n), alpha=(1.3, 1.6, 1.8)[:d], kappa=(1.0, 0.7, 1.2)[:d],
                T=1.0, M=M, e=FieldSpec("poly_t", (1.0, 0.5, 1.0, 1.0)),
                f=FieldSpec("manufactured", (1.0, 2.0)),
                psi=FieldSpec("manufactured", (1.0, 2.0), time_dependent=False), restart=20, rtol=1e-10)
    base.update(kw)
    return Instance(**base)


def _solve(inst, **over):
    S = solver_for(inst, **over)
    u = empty(inst.size)
    R.rsfde_eval_field(S.h, 0, R.WHICH_PSI, 0.0, u)
    status, st = R.rsfde_solve(S.h, inst.M, [u])
    got = host(u)
    S.close()
    return status, st[0], got


def _check(inst, max_iter_diff=None, **over):
    x0 = over.get("x0_mode", 0)
    ref = O.run(inst, x0_mode=x0)
    status, st, got = _solve(inst, **over)
    d = rel(got, ref["u"]) if np.max(np.abs(ref["u"])) > 0 else float(np.max(np.abs(got)))
    say(f"   {inst.n}: status {status}, rel diff {d:.2e}, iters {st['iters']} oracle {sum(ref['iters'])}")
    assert d <= 1e-10
    lim = max(1, inst.M // 8) if max_iter_diff is None else max_iter_diff
    assert abs(st["iters"] - sum(ref["iters"])) <= lim
    return status, st, ref


@pytest.mark.parametrize("d,n", [(1, (3,)), (2, (3, 5)), (3, (3, 3, 5)), (1, (2047,)), (1, (1535,)),
                                 (2, (2047, 7)), (2, (5, 1535)),
                                 # strided axes with 64-thread transforms (L = 512, 768): the
                                 # operator pass's per-thread runs, beside a one-thread axis (L = 12)
                                 (2, (5, 255)), (2, (3, 383)), (3, (3, 255, 5))])
def test_smallest_and_largest_transform_lengths(d, n):
    say(f"[edges] d={d} n={n}")
    status, _, _ = _check(_inst(d, n))
    assert status == R.RSFDE_OK


@pytest.mark.parametrize("d", [2, 3])
def test_axis_without_fractional_diffusion(d):
    # kappa_2 = 0: eta_2 = 0, the S_alpha term of that axis vanishes
    kappa = (1.0, 0.0, 0.8)[:d]
    inst = _inst(d, (31, 23, 15)[:d], kappa=kappa)
    status, _, _ = _check(inst)
    assert status == R.RSFDE_OK


def test_zero_right_hand_side_converges_without_iterations():
    inst = _inst(2, (31, 47), f=FieldSpec("zero", time_dependent=False),
                 psi=FieldSpec("zero", time_dependent=False))
    status, st, got = _solve(inst)
    assert status == R.RSFDE_OK and st["iters"] == 0
    assert np.all(got == 0.0)


@pytest.mark.parametrize("x0_mode", [0, 1])
def test_gmres1_and_zero_start(x0_mode):
    # GMRES(1): one iteration per cycle, many cycles per step
    inst = _inst(2, (23, 31), restart=1, max_cycles=400, rtol=1e-9)
    status, st, _ = _check(inst, max_iter_diff=3, x0_mode=x0_mode)
    assert status == R.RSFDE_OK and st["cycles"] == st["iters"]


def test_cycle_limit_reached():
    # GMRES(2) with two cycles per step cannot reach 1e-14: the step ends with the
    # last iterate, as in the oracle, and the solve reports it
    inst = _inst(2, (31, 31), M=2, restart=2, max_cycles=2, rtol=1e-14)
    status, st, ref = _check(inst, max_iter_diff=0)
    assert status == R.RSFDE_W_NOT_CONVERGED and st["converged"] == 0
    assert st["iters"] == 2 * 2 * inst.M


def test_alpha_two_with_constant_e_takes_one_iteration():
    # alpha = 2: tau(S) = S, and with e = ebar the preconditioner B P equals A
    inst = _inst(2, (31, 47), alpha=(2.0 - 1e-12, 2.0 - 1e-12), e=FieldSpec("const", (1.3,)), M=2)
    status, st, _ = _solve(inst)
    say(f"   iterations {st['iters']} over {inst.M} steps")
    assert status == R.RSFDE_OK and st["iters"] <= inst.M
