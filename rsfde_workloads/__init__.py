"""Seeded, synthetic workload descriptions shared by the oracle and the GPU path.

This module only *describes* problems: grid sizes, fractional orders, diffusion
coefficients, time span, solver settings, and the analytic families that the
coefficient e(x,t), the source f(x,t) and the initial value psi(x) belong to,
together with any random amplitudes those families need (drawn here, from a
stated seed).  It holds none of the method's arithmetic: evaluating a field,
building a matrix or solving anything is left to each side on its own.

Problem statement followed: the d-dimensional variable-coefficient Riesz space
fractional diffusion equation of Section 1 (eq. RSFDE) on prod_i (lo_i, hi_i),
with homogeneous Dirichlet data, discretised on N_i interior points per axis and
M Crank-Nicolson steps over [0, T] (Section 2).

Field families (each side evaluates them itself):

  e-kinds
    "const"        e = c0
    "sumsq_exp"    e = (sum_i x_i^2 + exp(-t)) / c0           (paper Examples 1-3)
    "poly_t"       e = c0 + c1 * (1 + c2 t) * prod_i x_i^p     (p = c3)
    "sinprod_cos"  e = c0 + c1 * prod_i sin(pi x_i) * cos(t)
    "sine_field"   e = c0 + c1 * (1 + g(x)/sum|a|)/2,  g = sum_K a_K prod_i sin(k_i pi x_i)
  f-kinds
    "zero"         f = 0
    "manufactured" f = e u_t - sum_i kappa_i d^{alpha_i}_{x_i} u  for
                   u = A exp(-t) prod_i x_i^a (1 - x_i)^a on the unit cube
                   (A = c0, a = integer c1)
    "sine_modes"   f = sum_K a_K prod_i sin(k_i pi x_i)   (time independent)
  psi-kinds
    "zero"         psi = 0
    "manufactured" psi = u(x, 0) of the manufactured family above

Mode amplitudes a_K are stored in a flat array of length K^d indexed
k_1 + K (k_2 + K k_3) (mode numbers k_i = index + 1), axis 1 fastest.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field, replace
from typing import Dict, List, Optional, Tuple

import numpy as np

__all__ = ["Instance", "config", "paper_example", "CONFIG_NAMES", "with_grid"]


@dataclass
class FieldSpec:
    kind: str
    c: Tuple[float, ...] = ()
    modes: int = 0
    amp: Optional[np.ndarray] = None  # flat K^d array (float64) for mode families
    time_dependent: bool = True


@dataclass
class Instance:
    name: str
    d: int
    n: Tuple[int, ...]
    alpha: Tuple[float, ...]
    kappa: Tuple[float, ...]
    T: float
    M: int
    e: FieldSpec
    f: FieldSpec
    psi: FieldSpec
    restart: int = 20
    rtol: float = 1e-10
    max_cycles: int = 10
    lo: Tuple[float, ...] = ()
    hi: Tuple[float, ...] = ()

    def __post_init__(self):
        if not self.lo:
            self.lo = (0.0,) * self.d
        if not self.hi:
            self.hi = (1.0,) * self.d

    @property
    def dt(self) -> float:
        return self.T / self.M

    @property
    def size(self) -> int:
        return int(np.prod(self.n))


def _modes(rng: np.random.Generator, K: int, d: int) -> np.ndarray:
    return rng.standard_normal(K ** d).astype(np.float64)


def with_grid(inst: Instance, n, M: Optional[int] = None) -> Instance:
    """Same problem on another grid (and optionally another step count)."""
    if isinstance(n, int):
        n = (n,) * inst.d
    return replace(inst, n=tuple(int(v) for v in n), M=inst.M if M is None else int(M))


def _c1() -> Instance:
    # d=1 plain FP64: n=511 on (0,1), alpha=1.5, kappa=1, e = 1 + x^2 (1+t),
    # T=1, 64 steps, manufactured u = e^{-t} x^2 (1-x)^2, GMRES(20) rtol 1e-12.
    return Instance(
        name="C1", d=1, n=(511,), alpha=(1.5,), kappa=(1.0,), T=1.0, M=64,
        e=FieldSpec("poly_t", (1.0, 1.0, 1.0, 2.0)),
        f=FieldSpec("manufactured", (1.0, 2.0)),
        psi=FieldSpec("manufactured", (1.0, 2.0), time_dependent=False),
        restart=20, rtol=1e-12)


def _c2() -> Instance:
    # d=2: n=1023 per axis, alpha=(1.3,1.7), kappa=(1,0.5),
    # e = 2 + sin(pi x) sin(pi y) cos(t), 32 steps, f = 8x8 sine modes with
    # N(0,1) amplitudes (seed 0), psi = 0, GMRES(30) rtol 1e-10.
    rng = np.random.default_rng(0)
    return Instance(
        name="C2", d=2, n=(1023, 1023), alpha=(1.3, 1.7), kappa=(1.0, 0.5), T=1.0, M=32,
        e=FieldSpec("sinprod_cos", (2.0, 1.0)),
        f=FieldSpec("sine_modes", (), modes=8, amp=_modes(rng, 8, 2), time_dependent=False),
        psi=FieldSpec("zero", time_dependent=False),
        restart=30, rtol=1e-10)


def _c3() -> Instance:
    # d=3: n=255 per axis, alpha=(1.2,1.5,1.8), kappa=(1,1,1),
    # e = 1 + 0.5 xyz (1+t), 16 steps, manufactured u = e^{-t} prod x_i^2 (1-x_i)^2.
    return Instance(
        name="C3", d=3, n=(255, 255, 255), alpha=(1.2, 1.5, 1.8), kappa=(1.0, 1.0, 1.0),
        T=1.0, M=16,
        e=FieldSpec("poly_t", (1.0, 0.5, 1.0, 1.0)),
        f=FieldSpec("manufactured", (1.0, 2.0)),
        psi=FieldSpec("manufactured", (1.0, 2.0), time_dependent=False),
        restart=30, rtol=1e-10)


def _c4(count: int = 64) -> List[Instance]:
    # 64 independent 2-D instances; n_i drawn from {127,255,383,511} per axis,
    # alpha_i ~ U(1.1,1.9), kappa_i ~ U(0.2,2), e = 1 + U(0,1) * ghat (ghat a
    # smooth sine-mode field mapped into [0,1]), f = 8x8 sine modes, psi = 0,
    # 16 steps, GMRES(30) rtol 1e-10.  Seed 1 for the instance draws and
    # 1000+i for instance i's fields.
    rng = np.random.default_rng(1)
    sizes = np.array([127, 255, 383, 511])
    out = []
    for i in range(count):
        n = tuple(int(v) for v in rng.choice(sizes, size=2))
        alpha = tuple(float(v) for v in rng.uniform(1.1, 1.9, size=2))
        kappa = tuple(float(v) for v in rng.uniform(0.2, 2.0, size=2))
        u01 = float(rng.uniform(0.0, 1.0))
        frng = np.random.default_rng(1000 + i)
        eamp = _modes(frng, 8, 2)
        famp = _modes(frng, 8, 2)
        out.append(Instance(
            name=f"C4[{i}]", d=2, n=n, alpha=alpha, kappa=kappa, T=1.0, M=16,
            e=FieldSpec("sine_field", (1.0, u01), modes=8, amp=eamp, time_dependent=False),
            f=FieldSpec("sine_modes", (), modes=8, amp=famp, time_dependent=False),
            psi=FieldSpec("zero", time_dependent=False),
            restart=30, rtol=1e-10))
    return out


def _c5() -> Instance:
    # d=3 large: n=511 per axis, alpha=(1.4,1.6,1.9), kappa=(1,0.8,0.6),
    # e = 2 + prod sin(pi x_i) cos(t), f = 8x8x8 sine modes (seed 2), psi = 0,
    # 8 steps, GMRES(20) rtol 1e-10.
    rng = np.random.default_rng(2)
    return Instance(
        name="C5", d=3, n=(511, 511, 511), alpha=(1.4, 1.6, 1.9), kappa=(1.0, 0.8, 0.6),
        T=1.0, M=8,
        e=FieldSpec("sinprod_cos", (2.0, 1.0)),
        f=FieldSpec("sine_modes", (), modes=8, amp=_modes(rng, 8, 3), time_dependent=False),
        psi=FieldSpec("zero", time_dependent=False),
        restart=20, rtol=1e-10)


CONFIG_NAMES = ("C1", "C2", "C3", "C4", "C5")


def config(name: str):
    """The named synthetic workload: an Instance, or a list of them for C4."""
    name = name.upper()
    if name == "C1":
        return _c1()
    if name == "C2":
        return _c2()
    if name == "C3":
        return _c3()
    if name == "C4":
        return _c4()
    if name == "C5":
        return _c5()
    raise KeyError(name)


def paper_example(d: int, alpha, Np1: int, M: int, restart: int = 30) -> Instance:
    """Examples 1-3 of Section 4 (the paper's own analytic test problems).

    d=1: kappa=100,          e=(x^2+e^{-t})/50,        u=100 e^{-t} x^4(1-x)^4
    d=2: kappa=(100,100),     e=(x^2+y^2+e^{-t})/100,   u=1e4 e^{-t} prod x_i^4(1-x_i)^4
    d=3: kappa=(100,85,103),  e=(sum x_i^2+e^{-t})/100, u=1e8 e^{-t} prod x_i^4(1-x_i)^4
    The stopping tolerance is 1e-9 for d=1,2 and 1e-10 for d=3.
    """
    if isinstance(alpha, (int, float)):
        alpha = (float(alpha),)
    alpha = tuple(float(a) for a in alpha)
    assert len(alpha) == d
    kappa = {1: (100.0,), 2: (100.0, 100.0), 3: (100.0, 85.0, 103.0)}[d]
    escale = {1: 50.0, 2: 100.0, 3: 100.0}[d]
    amp = {1: 100.0, 2: 1e4, 3: 1e8}[d]
    rtol = 1e-9 if d < 3 else 1e-10
    return Instance(
        name=f"ex{d}", d=d, n=(Np1 - 1,) * d, alpha=alpha, kappa=kappa, T=1.0, M=M,
        e=FieldSpec("sumsq_exp", (escale,)),
        f=FieldSpec("manufactured", (amp, 4.0)),
        psi=FieldSpec("manufactured", (amp, 4.0), time_dependent=False),
        restart=restart, rtol=rtol)
