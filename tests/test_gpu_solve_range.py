"""GPU: rsfde_solve_range continues the time loop of rsfde_solve from step m0.
A run split into ranges, the whole run, and the same steps through rsfde_step
with the fields evaluated at each midpoint give the same u bit for bit (the
same kernels on the same inputs); the batched form likewise."""
import numpy as np
import pytest

from paper_2404_10221_amd import rsfde as R
from rsfde_workloads import config, with_grid

from gpu_helpers import empty, host, say, solver_for

pytestmark = pytest.mark.gpu


def _psi(S, k, inst):
    u = empty(inst.size)
    R.rsfde_eval_field(S.h, k, R.WHICH_PSI, 0.0, u)
    return u


@pytest.mark.parametrize("wl,n,M", [("C2", (63, 47), 6), ("C3", (15, 23, 11), 4), ("C1", (127,), 5)])
def test_ranges_equal_the_whole_run_and_single_steps(wl, n, M):
    inst = with_grid(config(wl), n, M=M)
    say(f"[solve_range] {wl} n={n} M={M}")
    S = solver_for(inst)
    R.rsfde_prescan_ebar(S.h, 0, M)
    whole = _psi(S, 0, inst)
    s_whole, st_whole = R.rsfde_solve(S.h, M, [whole])
    split = _psi(S, 0, inst)
    its = 0
    for m0, k in ((0, 2), (2, 1), (3, M - 3)):
        s, st = R.rsfde_solve_range(S.h, m0, k, [split])
        assert s == R.RSFDE_OK
        its += st[0]["iters"]
    # one step at a time with the fields evaluated by the caller
    step = _psi(S, 0, inst)
    e, f = empty(inst.size), empty(int(np.prod([v + 2 for v in n])))
    its1 = 0
    for m in range(M):
        th = (m + 0.5) * inst.dt
        R.rsfde_eval_field(S.h, 0, R.WHICH_E, th, e)
        R.rsfde_eval_field(S.h, 0, R.WHICH_F, th, f)
        s, st = R.rsfde_step(S.h, m * inst.dt, [e], [f], [step])
        assert s == R.RSFDE_OK
        its1 += st[0]["iters"]
    a, b, c = host(whole), host(split), host(step)
    S.close()
    assert s_whole == R.RSFDE_OK and st_whole[0]["converged"] == 1
    assert its == st_whole[0]["iters"] == its1
    assert np.array_equal(a, b) and np.array_equal(a, c)


def test_batched_ranges_equal_the_whole_run():
    insts = [with_grid(config("C2"), (31, 23), M=4), with_grid(config("C2"), (15, 47), M=4)]
    S = R.Solver([R.params_from_instance(i) for i in insts])
    for k, inst in enumerate(insts):
        R.rsfde_set_fields(S.h, k, inst.e, inst.f, inst.psi)
        R.rsfde_prescan_ebar(S.h, k, inst.M)
    whole = [_psi(S, k, i) for k, i in enumerate(insts)]
    split = [_psi(S, k, i) for k, i in enumerate(insts)]
    s0, _ = R.rsfde_solve(S.h, 4, whole)
    s1, _ = R.rsfde_solve_range(S.h, 0, 1, split)
    s2, _ = R.rsfde_solve_range(S.h, 1, 3, split)
    same = all(np.array_equal(host(a), host(b)) for a, b in zip(whole, split))
    S.close()
    assert s0 == s1 == s2 == R.RSFDE_OK and same


def test_negative_first_step_is_rejected():
    inst = with_grid(config("C2"), (15, 15), M=2)
    S = solver_for(inst)
    u = _psi(S, 0, inst)
    with pytest.raises(R.RsfdeError) as ex:
        R.rsfde_solve_range(S.h, -1, 1, [u])
    S.close()
    assert ex.value.status == R.RSFDE_E_INVALID_ARG
