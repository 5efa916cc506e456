"""Pins of the oracle's remaining open parts (CPU only).

* Fourth order in space of the whole scheme in two and three dimensions
  (Section 4 ties M to N^2, so halving h divides the error by about 16), which
  pins the d = 3 discretisation independently of Table 4's Error column.
* The synthetic field families, point by point, against the workload formulas
  written out here as literals (not through the oracle's evaluators).
* The manufactured sources against the Riesz derivative obtained as the limit of
  the fractional centred difference operator (Section 2), independent of the
  closed-form Riemann-Liouville power rule the oracle uses.
* ebar (eqs. dhat, bard) against a brute-force scan and, for the sin-product
  coefficient, its closed form.
"""
import math

import numpy as np
import pytest

import oracle as O
from oracle import rsfde_oracle as OR
from rsfde_workloads import FieldSpec, Instance, config, paper_example, with_grid


# --- order of the whole scheme (Section 4: M = N^2) -------------------------

@pytest.mark.parametrize("d,alpha,grids", [
    (2, (1.3, 1.7), (8, 16, 32)),
    (3, (1.2, 1.5, 1.8), (8, 16)),
])
def test_T14b_fourth_order_in_space_two_and_three_dimensions(d, alpha, grids):
    """Examples 2 and 3 of Section 4 with M = (N+1)^2 steps: the L2 error (max over
    the steps) falls by about 2^4 each time h halves.  A dropped or mis-signed term
    anywhere in the d-dimensional operator, the source F or the time stepping
    breaks the ratio."""
    errs = []
    for Np1 in grids:
        inst = paper_example(d, alpha, Np1, M=Np1 * Np1)
        errs.append(O.run(inst, track_error=True)["err_l2"])
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    for r in ratios:
        assert 13.0 < r < 20.0, (errs, ratios)


# --- field families against the workload formulas ---------------------------

def _pts(d, rng, k=7):
    return [rng.uniform(0.0, 1.0, size=k) for _ in range(d)]


def test_e_families_against_the_workload_formulas():
    rng = np.random.default_rng(11)
    t = 0.37
    # C1: e = 1 + x^2 (1 + t)
    (x,) = _pts(1, rng)
    got = OR.eval_e(config("C1").e, [x], t)
    np.testing.assert_allclose(got, 1.0 + x * x * (1.0 + t), rtol=0, atol=1e-15)
    # C2: e = 2 + sin(pi x) sin(pi y) cos t
    x, y = _pts(2, rng)
    got = OR.eval_e(config("C2").e, [x, y], t)
    np.testing.assert_allclose(got, 2.0 + np.sin(np.pi * x) * np.sin(np.pi * y) * math.cos(t),
                               rtol=0, atol=1e-15)
    # C3: e = 1 + 0.5 x y z (1 + t)
    x, y, z = _pts(3, rng)
    got = OR.eval_e(config("C3").e, [x, y, z], t)
    np.testing.assert_allclose(got, 1.0 + 0.5 * x * y * z * (1.0 + t), rtol=0, atol=1e-15)
    # C5: e = 2 + sin(pi x) sin(pi y) sin(pi z) cos t
    got = OR.eval_e(config("C5").e, [x, y, z], t)
    np.testing.assert_allclose(
        got, 2.0 + np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z) * math.cos(t),
        rtol=0, atol=1e-15)
    # Examples 1-3: e = (sum x_i^2 + exp(-t)) / c with c = 50, 100, 100
    for d, c in ((1, 50.0), (2, 100.0), (3, 100.0)):
        X = _pts(d, rng)
        inst = paper_example(d, (1.5,) * d, 8, 4)
        got = OR.eval_e(inst.e, X, t)
        np.testing.assert_allclose(got, (sum(v * v for v in X) + math.exp(-t)) / c,
                                   rtol=0, atol=1e-15)


def _modes_loop(amp, K, X):
    """sum_{k_1..k_d = 1..K} a_K prod_i sin(k_i pi x_i), amplitude index
    k_1 - 1 + K (k_2 - 1) + K^2 (k_3 - 1): plain loops, one point at a time."""
    d = len(X)
    npt = len(X[0])
    out = np.zeros(npt)
    for p in range(npt):
        acc = 0.0
        for flat in range(K ** d):
            ks = [(flat // K ** i) % K + 1 for i in range(d)]
            term = amp[flat]
            for i in range(d):
                term *= math.sin(ks[i] * math.pi * X[i][p])
            acc += term
        out[p] = acc
    return out


def test_sine_mode_fields_against_plain_loops():
    """C2 and C5 sources (8^d seeded sine modes, mode numbers from 1, k_1 fastest)
    and C4's coefficient e = 1 + U (1 + g / sum|a|) / 2, which lies in [1, 1 + U]."""
    rng = np.random.default_rng(12)
    for name in ("C2", "C5"):
        inst = config(name)
        X = _pts(inst.d, rng, k=5)
        got = OR.eval_f(inst.f, inst.e, inst.alpha, inst.kappa, X, 0.3)
        np.testing.assert_allclose(got, _modes_loop(inst.f.amp, 8, X), rtol=1e-13, atol=1e-13)
    for inst in config("C4")[:3]:
        X = _pts(2, rng, k=5)
        U = inst.e.c[1]
        g = _modes_loop(inst.e.amp, 8, X)
        want = 1.0 + U * 0.5 * (1.0 + g / np.sum(np.abs(inst.e.amp)))
        got = OR.eval_e(inst.e, X, 0.0)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-14)
        assert np.all(got >= 1.0) and np.all(got <= 1.0 + U)
        # the source of the same instance: its own 8x8 modes
        got_f = OR.eval_f(inst.f, inst.e, inst.alpha, inst.kappa, X, 0.0)
        np.testing.assert_allclose(got_f, _modes_loop(inst.f.amp, 8, X), rtol=1e-13, atol=1e-13)


def _riesz_fcd_limit(alpha, a, x):
    """d^alpha / d|x|^alpha of x^a (1-x)^a (extended by zero) at grid-exact points x,
    as the limit h -> 0 of the fractional centred difference -h^-alpha sum_k s_|k| u(x-kh)
    (Section 2; second order in h), Richardson-extrapolated from h = 2^-12, 2^-13."""
    vals = []
    for p in (12, 13):
        N = 2 ** p - 1
        h = 1.0 / (N + 1)
        grid = h * np.arange(1, N + 1)
        u = grid ** a * (1.0 - grid) ** a
        s = O.fcd_weights(alpha, N)
        out = []
        for xv in x:
            j = int(round(xv / h)) - 1
            assert abs(grid[j] - xv) < 1e-15
            out.append(-(s[np.abs(np.arange(N) - j)] @ u) / h ** alpha)
        vals.append(np.array(out))
    return (4.0 * vals[1] - vals[0]) / 3.0


def test_manufactured_sources_against_the_fcd_limit():
    """f = e u_t - sum_i kappa_i d^{alpha_i} u / d|x_i|^{alpha_i} for the manufactured
    solutions of C1 (1-D, u = e^{-t} x^2 (1-x)^2) and C3 (3-D, product of the same
    factors), with the Riesz derivative taken from the discrete operator's limit."""
    t = 0.45
    pts = np.array([0.25, 0.375, 0.5, 0.8125])
    c1 = config("C1")
    a = 2
    ux = pts ** a * (1 - pts) ** a
    e = 1.0 + pts * pts * (1.0 + t)
    want = -e * math.exp(-t) * ux - c1.kappa[0] * math.exp(-t) * _riesz_fcd_limit(c1.alpha[0], a, pts)
    got = OR.eval_f(c1.f, c1.e, c1.alpha, c1.kappa, [pts], t)
    np.testing.assert_allclose(got, want, rtol=2e-8)

    c3 = config("C3")
    X = [pts, pts[::-1].copy(), np.array([0.5, 0.25, 0.8125, 0.375])]
    fac = [v ** a * (1 - v) ** a for v in X]
    der = [_riesz_fcd_limit(c3.alpha[i], a, X[i]) for i in range(3)]
    e = 1.0 + 0.5 * X[0] * X[1] * X[2] * (1.0 + t)
    u = math.exp(-t) * fac[0] * fac[1] * fac[2]
    want = -e * u
    for i in range(3):
        other = np.prod([fac[l] for l in range(3) if l != i], axis=0)
        want = want - c3.kappa[i] * math.exp(-t) * other * der[i]
    got = OR.eval_f(c3.f, c3.e, c3.alpha, c3.kappa, X, t)
    np.testing.assert_allclose(got, want, rtol=2e-8)


# --- ebar (eqs. dhat, bard) -------------------------------------------------

def test_compute_ebar_against_brute_force_and_closed_form():
    """ebar = (max + min)/2 of e over the interior grid and every midpoint
    t_{m+1/2} = (m + 1/2) dt.  For e = 2 + sin(pi x) sin(pi y) cos t on (0,1)^2 with
    N odd (so x = 1/2 is a grid point) and t in [0, 1] (cos t > 0), the extremes are
    2 + cos t_{1/2} at the centre and 2 + sin(pi h)^2 cos t_{M-1/2} at a corner."""
    inst = with_grid(config("C2"), (15, 15), M=6)
    P = O.OracleProblem(inst)
    h = 1.0 / 16
    dt = 1.0 / 6
    hi = 2.0 + math.cos(0.5 * dt)
    lo = 2.0 + math.sin(math.pi * h) ** 2 * math.cos(5.5 * dt)
    assert abs(P.ebar - 0.5 * (hi + lo)) < 1e-15

    # brute force: one point and one midpoint at a time, for a time-dependent e
    inst3 = with_grid(config("C3"), (5, 4, 3), M=5)
    P3 = O.OracleProblem(inst3)
    vals = []
    for m in range(5):
        t = (m + 0.5) / 5
        for k in range(1, 4):
            for j in range(1, 5):
                for i in range(1, 6):
                    x, y, z = i / 6, j / 5, k / 4
                    vals.append(1.0 + 0.5 * x * y * z * (1.0 + t))
    assert abs(P3.ebar - 0.5 * (max(vals) + min(vals))) < 1e-15
