"""The two-sided form (eq. Pls) on the GPU against the oracle's two-sided form:
the sine-basis factors P^{-1/2} B^{-1} and P^{-1/2} alone, then whole time loops
(GMRES on P^{-1/2} Atilde P^{-1/2} utilde = P^{-1/2} btilde from P^{1/2} u^m),
with restarts and a zero start, and the TPGM Iter columns of Tables 2-4 at the
printed sizes."""
import os
from dataclasses import replace

import numpy as np
import pytest

import oracle as O
from paper_2404_10221_amd import rsfde as R
from rsfde_workloads import config, paper_example, with_grid

from gpu_helpers import dev, empty, host, rel, say, solver_for
from test_gpu_parity import SHAPES, SOLVE_CASES, _inst

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("d,n", SHAPES)
def test_prec_forms(d, n):
    say(f"[prec forms] d={d} n={n}")
    inst = _inst(d, n, seed=5)
    P = O.OracleProblem(inst, ebar=1.3)
    r = np.random.default_rng(6).standard_normal(P.shape)
    S = solver_for(inst, ebar=(1.3, 1.3))
    refs = {
        R.PREC_BP_INV: P.apply_prec_inv(r),
        R.PREC_PHALF_BINV: P.apply_P_power(P.apply_B_inv(r), -0.5),
        R.PREC_PHALF: P.apply_P_power(r, -0.5),
    }
    mu, lam = P.mu(), P.lam_K()
    diag = {R.PREC_BP_INV: 1 / mu, R.PREC_PHALF_BINV: 1 / np.sqrt(lam * mu), R.PREC_PHALF: np.sqrt(lam / mu)}
    out = empty(r.size)
    for form, ref in refs.items():
        R.rsfde_apply_prec_form(S.h, 0, form, dev(r), out)
        d_ = rel(host(out), ref.ravel())
        # the rounding of the first transform (either side) reaches the result scaled
        # by the diagonal's peak-to-rms ratio: 2e-13 per unit of that ratio (the FFT
        # twiddles are products of two table values, two roundings), at least 1e-12
        g = diag[form]
        tol = max(1e-12, 2e-13 * g.max() / np.sqrt((g ** 2).mean()))
        say(f"   form {form}: rel diff {d_:.2e} (bound {tol:.1e})")
        assert d_ < tol
    S.close()


def _solve(inst, **over):
    S = solver_for(inst, method=R.RSFDE_TPGM, **over)
    u = empty(inst.size)
    R.rsfde_eval_field(S.h, 0, R.WHICH_PSI, 0.0, u)
    status, st = R.rsfde_solve(S.h, inst.M, [u])
    got = host(u)
    S.close()
    return status, st[0], got


@pytest.mark.parametrize("name,mk", SOLVE_CASES, ids=[c[0] for c in SOLVE_CASES])
def test_time_loop_parity_two_sided(name, mk):
    inst = mk()
    say(f"[solve tpgm] {name} n={inst.n} M={inst.M}")
    ref = O.run(inst, two_sided=True)
    status, st, got = _solve(inst)
    d = rel(got, ref["u"])
    say(f"   rel diff {d:.3e}  iters gpu {st['iters']} oracle {sum(ref['iters'])}")
    assert status == R.RSFDE_OK and st["converged"] == 1
    assert d <= 1e-10
    assert abs(st["iters"] - sum(ref["iters"])) <= max(1, inst.M // 8)


@pytest.mark.parametrize("x0_mode", [0, 1])
def test_two_sided_restarts_and_zero_start(x0_mode):
    # GMRES(3) forces several cycles per step (each ends with u += P^{-1/2} V y)
    inst = replace(with_grid(config("C2"), (31, 47), M=3), restart=3, max_cycles=80)
    ref = O.run(inst, two_sided=True, x0_mode=x0_mode)
    status, st, got = _solve(inst, x0_mode=x0_mode)
    d = rel(got, ref["u"])
    say(f"   x0_mode {x0_mode}: rel diff {d:.3e}, cycles {st['cycles']}")
    assert status == R.RSFDE_OK and st["cycles"] > 3
    assert d <= 1e-10


def _rows(name):
    out = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                out.append([float(v) for v in line.split()])
    return out


def _table_cases():
    cases = []
    for a, M, Np1, it in _rows("table2_example1_tpgm_iter.txt"):
        cases.append((1, (a,), int(M), int(Np1), it))
    for a1, a2, M, Np1, it in _rows("table3_example2_tpgm_iter.txt"):
        cases.append((2, (a1, a2), int(M), int(Np1), it))
    for a1, a2, a3, M, Np1, it in _rows("table4_example3_tpgm_iter.txt"):
        cases.append((3, (a1, a2, a3), int(M), int(Np1), it))
    return cases


def test_tables_2_3_4_two_sided_iterations_on_gpu():
    # the oracle's bound: 0.35 of an iteration, 1.0 on the one row the oracle also
    # misses (Table 3, alpha = (1.3, 1.5), N+1 = 16)
    for d, al, M, np1, it_ref in _table_cases():
        status, st, _ = _solve(paper_example(d, al, np1, M))
        it = st["iters"] / M
        say(f"   d={d} alpha {al} N+1 {np1}: iter {it:.3f} (paper {it_ref})")
        assert status == R.RSFDE_OK
        tol = 1.0 if (d, al, np1) == (2, (1.3, 1.5), 16) else 0.35
        assert abs(it - it_ref) <= tol
