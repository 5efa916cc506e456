"""GPU: the mixed form's FP32 pass kernels at every long transform length, on the
contiguous and the strided axes, against the FP64 oracle; the recomputed true
residual of rsfde_stats; and the non-finite status of rsfde_step."""
import numpy as np
import pytest

import oracle as O
from paper_2404_10221_amd import rsfde as R
from rsfde_workloads import config, with_grid

from gpu_helpers import dev, empty, host, rel, say, solver_for, tight

pytestmark = pytest.mark.gpu

# (workload, grid): transform lengths L = 2(N+1) of 512, 768, 1024, 2048, 3072 and
# 4096 on axis 1 (contiguous) and on a strided axis, beside short axes
LONG_AXES = [
    ("C2", (1023, 7)), ("C2", (7, 1023)),
    ("C2", (383, 5)), ("C2", (5, 383)),
    ("C2", (2047, 3)), ("C2", (3, 2047)),
    ("C2", (1535, 3)), ("C2", (3, 1535)),
    ("C3", (255, 5, 7)), ("C3", (5, 7, 255)),
    ("C5", (5, 7, 511)), ("C5", (511, 3, 5)), ("C5", (3, 511, 5)),
]


@pytest.mark.parametrize("wl,n", LONG_AXES, ids=[f"{w}-{'x'.join(map(str, n))}" for w, n in LONG_AXES])
def test_mixed_form_long_axes_against_oracle(wl, n):
    inst = with_grid(config(wl), n, M=3)
    say(f"[mixed long] {wl} n={n} M={inst.M}")
    ref = O.run(tight(inst))
    S = solver_for(inst, precision=R.RSFDE_MIXED)
    u = empty(inst.size)
    R.rsfde_eval_field(S.h, 0, R.WHICH_PSI, 0.0, u)
    status, st = R.rsfde_solve(S.h, inst.M, [u])
    d = rel(host(u), ref["u"])
    say(f"   rel diff {d:.3e}  iters {st[0]['iters']} sweeps {st[0]['outer_sweeps']} "
        f"true res {st[0]['rel_true_res']:.2e}")
    S.close()
    assert status == R.RSFDE_OK and st[0]["converged"] == 1
    # the refinement stops at a tenth of rtol on the FP64 residual; the result is
    # compared with the oracle solved to rounding level (TIGHT_RTOL), because the
    # mixed form reaches its bound along another Krylov sequence than the oracle's
    # FP64 GMRES, whose own solution at rtol may sit ~cond * rtol from the exact one
    assert 0.0 <= st[0]["rel_true_res"] <= 0.1 * inst.rtol
    assert d <= 1e-10


def _one_step_residual(P, e, F, u_old, u_new):
    """||(BP)^{-1}(b - A u_new)|| / ||(BP)^{-1}(b - A u_old)||, b from u_old (oracle)."""
    b = P.rhs(e, F, u_old)
    z = P.apply_prec_inv(b - P.apply_A(e, u_new))
    z0 = P.apply_prec_inv(b - P.apply_A(e, u_old))
    return float(np.linalg.norm(z) / np.linalg.norm(z0))


@pytest.mark.parametrize("wl,n", [("C2", (63, 47)), ("C3", (15, 23, 11))])
def test_true_residual_of_a_step(wl, n):
    """rel_true_res is the FP64 preconditioned residual of the returned u relative to
    ||z_0||, recomputed from u: the oracle's operators applied to the GPU's u give
    the same ratio.  It is -1 while the check is off (FP64 form)."""
    inst = with_grid(config(wl), n, M=1)
    P = O.OracleProblem(inst)
    S = solver_for(inst, ebar=(P.ebar, P.ebar))
    t = P.t_half(0)
    e, f, u = empty(inst.size), empty(np.prod([v + 2 for v in n])), empty(inst.size)
    R.rsfde_eval_field(S.h, 0, R.WHICH_E, t, e)
    R.rsfde_eval_field(S.h, 0, R.WHICH_F, t, f)
    R.rsfde_eval_field(S.h, 0, R.WHICH_PSI, 0.0, u)
    u_old = host(u).reshape(P.shape)
    status, st = R.rsfde_step(S.h, 0.0, [e], [f], [u])
    assert status == R.RSFDE_OK and st[0]["rel_true_res"] == -1.0
    R.rsfde_eval_field(S.h, 0, R.WHICH_PSI, 0.0, u)
    R.rsfde_set_true_residual(S.h, True)
    status, st = R.rsfde_step(S.h, 0.0, [e], [f], [u])
    u_new = host(u).reshape(P.shape)
    F = P.F_from_closure(P.f_closure_at(t))
    want = _one_step_residual(P, P.e_at(t), F, u_old, u_new)
    got = st[0]["rel_true_res"]
    say(f"[true res] {wl} n={n}: gpu {got:.4e} oracle {want:.4e} gmres {st[0]['rel_pres']:.4e}")
    S.close()
    assert status == R.RSFDE_OK
    assert 0.0 < got <= inst.rtol
    # both sides evaluate the same residual of the same u; at the 1e-10 level its
    # rounding noise is a few 1e-16 / 1e-10 relative
    assert abs(got - want) <= 1e-4 * want


def _nonfinite_case(precision, batched, which):
    insts = [with_grid(config("C2"), (31, 23), M=1), with_grid(config("C2"), (15, 47), M=1)]
    insts = insts if batched else insts[:1]
    S = R.Solver([R.params_from_instance(i, precision=precision, e_min=2.0, e_max=3.0)
                  for i in insts])
    es, fs, us = [], [], []
    for k, inst in enumerate(insts):
        R.rsfde_set_fields(S.h, k, inst.e, inst.f, inst.psi)
        e, f, u = empty(inst.size), empty(np.prod([v + 2 for v in inst.n])), empty(inst.size)
        R.rsfde_eval_field(S.h, k, R.WHICH_E, 0.5 * inst.dt, e)
        R.rsfde_eval_field(S.h, k, R.WHICH_F, 0.5 * inst.dt, f)
        R.rsfde_eval_field(S.h, k, R.WHICH_PSI, 0.0, u)
        es.append(e), fs.append(f), us.append(u)
    k = len(insts) - 1
    if which == "f":
        fs[k][fs[k].numel() // 2] = float("nan")
    elif which == "u":
        us[k][7] = float("inf")
    else:
        es[k][3] = float("nan")
    try:
        with pytest.raises(R.RsfdeError) as ex:
            R.rsfde_step(S.h, 0.0, es, fs, us)
        return ex.value.status
    finally:
        S.close()


@pytest.mark.parametrize("which", ["f", "u", "e"])
@pytest.mark.parametrize("precision,batched", [(R.RSFDE_FP64, False), (R.RSFDE_MIXED, False),
                                               (R.RSFDE_FP64, True), (R.RSFDE_MIXED, True)])
def test_nonfinite_input_returns_nonfinite_status(precision, batched, which):
    """A NaN or Inf in f, u or e reaches ||z_0|| and the step returns
    RSFDE_E_NONFINITE (NaN only propagates through the kernels)."""
    say(f"[nonfinite] precision={precision} batched={batched} in {which}")
    assert _nonfinite_case(precision, batched, which) == R.RSFDE_E_NONFINITE
