"""FP64 CPU oracle: quasi-compact Crank-Nicolson scheme for the variable-coefficient
Riesz space-fractional diffusion equation, solved at every step by GMRES(m) with
the sine-transform (tau) preconditioner: the one-sided form (eq. one-sided) and
the two-sided form (eq. Pls); and, as the paper's comparison solver, GMRES with
the Strang circulant preconditioner (Section 4).

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import or call this module.  It is written from
the paper alone, shares no code with the GPU library, and uses plain dense
matrices, an O(N^2) sine transform, an O(N^2) cosine sum for the tau eigenvalues
and textbook GMRES (modified Gram-Schmidt Arnoldi with Givens rotations).
Library primitives used as single steps: numpy matrix products (tensordot) and a
dense triangular solve.

Notation (Sections 2-3): N_i interior points on axis i, h_i = (hi_i-lo_i)/(N_i+1),
grid vectors ordered lexicographically with x_1 fastest, i.e. a numpy array of
shape (N_d, ..., N_1).

Readings of points the paper leaves open (each also listed in the design notes):
  * f in F^{(m+1/2)} is sampled at t_{m+1/2}; F is the tensor compact operator
    applied to f sampled on the closure grid, restricted to the interior
    (Appendix A written as one stencil).
  * e_hat, e_check are taken over the interior grid and all M midpoints (eq. dhat).
  * GMRES starts from x0 = u^{(m)} (x0 = 0 selectable), stops at the first k with
    ||z_k||_2 <= tol ||z_0||_2 for the left-preconditioned residual z, restarts
    every `restart` iterations keeping ||z_0|| of the step as the reference.
  * The L2 error of Table 1 is max_m sqrt(prod_i h_i * sum_J (u*-u)^2).
  * Two-sided form: GMRES with no further preconditioner on eq. Pls, started from
    utilde_0 = P^{1/2} u^{(m)} (the image of the one-sided start), with the same
    stopping rule on its own residual; u^{(m+1)} = P^{-1/2} utilde.
  * Strang form: left preconditioning of eq. tls by c(B) P_c = ebar c(B) + c(S)
    (the circulant counterpart of B P; c(B)^{1/2} P_c c(B)^{1/2} with commuting
    circulants), same start and stopping rule as the one-sided form.
"""
from __future__ import annotations

import math
from typing import Callable, Dict, List, Optional

import numpy as np

__all__ = [
    "fcd_weights", "fcd_weights_gamma", "toeplitz_dense", "B_dense", "sine_matrix",
    "hankel_dense", "tau_dense", "tau_eigs_cosine", "B_eigs", "riesz_poly_derivative",
    "strang_first_column", "circulant_dense", "strang_eigs",
    "OracleProblem", "PointOracle", "gmres_left", "run",
]


# ----------------------------------------------------------------------------
# Section 2: FCD weights s_k^{(alpha)}, the Toeplitz matrix S_{alpha_i} and B_{alpha_i}
# ----------------------------------------------------------------------------

def fcd_weights(alpha: float, N: int) -> np.ndarray:
    """s_0..s_{N-1} by the recurrence stated under eq. (eq0):
    s_0 = Gamma(alpha+1)/Gamma(alpha/2+1)^2, s_k = (1-(alpha+1)/(alpha/2+k)) s_{k-1}."""
    s = np.empty(N, dtype=np.float64)
    s[0] = math.gamma(alpha + 1.0) / math.gamma(alpha / 2.0 + 1.0) ** 2
    for k in range(1, N):
        s[k] = (1.0 - (alpha + 1.0) / (alpha / 2.0 + k)) * s[k - 1]
    return s


def fcd_weights_gamma(alpha: float, N: int) -> np.ndarray:
    """The same weights from their closed form (Section 2, FCD weights):
    s_j = (-1)^j Gamma(alpha+1) / (Gamma(alpha/2-j+1) Gamma(alpha/2+j+1)).
    For z = alpha/2-j+1 <= 0 the reflection formula 1/Gamma(z) = sin(pi z) Gamma(1-z)/pi
    keeps large j finite; 1/Gamma vanishes at the non-positive integers."""
    out = np.empty(N, dtype=np.float64)
    for j in range(N):
        z = alpha / 2.0 - j + 1.0
        if z > 0:
            out[j] = ((-1) ** j) * math.gamma(alpha + 1.0) / (math.gamma(z) * math.gamma(alpha / 2.0 + j + 1.0))
        elif z == math.floor(z):
            out[j] = 0.0
        else:
            sgn = math.copysign(1.0, math.sin(math.pi * z))
            lg = (math.lgamma(alpha + 1.0) + math.log(abs(math.sin(math.pi * z))) - math.log(math.pi)
                  + math.lgamma(1.0 - z) - math.lgamma(alpha / 2.0 + j + 1.0))
            out[j] = ((-1) ** j) * sgn * math.exp(lg)
    return out


def toeplitz_dense(t: np.ndarray) -> np.ndarray:
    """Symmetric Toeplitz matrix [t_{|p-q|}] (eq. eq0)."""
    N = len(t)
    idx = np.abs(np.arange(N)[:, None] - np.arange(N)[None, :])
    return t[idx].copy()


def B_dense(alpha: float, N: int) -> np.ndarray:
    """B_{alpha_i} = I + (alpha/24) tridiag(1,-2,1) (eq. Ha)."""
    Bm = np.eye(N) * (1.0 - alpha / 12.0)
    off = alpha / 24.0
    i = np.arange(N - 1)
    Bm[i, i + 1] = off
    Bm[i + 1, i] = off
    return Bm


# ----------------------------------------------------------------------------
# Section 3: tau algebra, the sine transform, eigenvalues
# ----------------------------------------------------------------------------

def sine_matrix(N: int) -> np.ndarray:
    """S = sqrt(2/(N+1)) [sin(pi j k/(N+1))]_{j,k=1..N} (Section 3)."""
    j = np.arange(1, N + 1)
    return math.sqrt(2.0 / (N + 1)) * np.sin(np.pi * np.outer(j, j) / (N + 1))


def hankel_dense(t: np.ndarray) -> np.ndarray:
    """H(T) of eq. (tau): first row (t_2, ..., t_{N-1}, 0, 0), last row
    (0, 0, t_{N-1}, ..., t_2), constant along anti-diagonals.  Written with
    1-based (j,k): H_{jk} = t_{j+k} + t_{2N+2-j-k}, with t_m = 0 for m >= N
    (the printed display is garbled; this is the reading that makes
    T - H(T) a tau matrix)."""
    N = len(t)
    tt = np.zeros(2 * N + 3)
    tt[:N] = t
    H = np.zeros((N, N))
    for j in range(1, N + 1):
        for k in range(1, N + 1):
            H[j - 1, k - 1] = tt[j + k] + tt[2 * N + 2 - j - k]
    return H


def tau_dense(t: np.ndarray) -> np.ndarray:
    """tau(T) = T - H(T) (eq. tau)."""
    return toeplitz_dense(t) - hankel_dense(t)


def tau_eigs_cosine(t: np.ndarray) -> np.ndarray:
    """q_i = t_0 + 2 sum_{j=1}^{N-1} t_j cos(pi j (i+1)/(N+1)), i=0..N-1 (eq. q),
    evaluated as the plain O(N^2) sum."""
    N = len(t)
    i = np.arange(N)[:, None]
    j = np.arange(1, N)[None, :]
    return t[0] + 2.0 * (np.cos(np.pi * j * (i + 1) / (N + 1)) * t[1:][None, :]).sum(axis=1)


def B_eigs(alpha: float, N: int) -> np.ndarray:
    """Eigenvalues of B_{alpha_i} (Lemma Heig): 1 + (alpha/24)(-4 sin^2(k pi/(2N+2))),
    k = 1..N, in the order of the sine modes."""
    k = np.arange(1, N + 1)
    return 1.0 - (alpha / 6.0) * np.sin(k * np.pi / (2.0 * N + 2.0)) ** 2


# ----------------------------------------------------------------------------
# Section 1: Riesz derivative of the polynomial x^a (1-x)^a on [0,1]
# ----------------------------------------------------------------------------

# ----------------------------------------------------------------------------
# Section 4: the Strang circulant s(T) of a symmetric Toeplitz matrix
# ----------------------------------------------------------------------------

def strang_first_column(t: np.ndarray) -> np.ndarray:
    """First column of s(T): the central diagonals of T (first column t) copied and
    wrapped around, c_k = t_k for k <= N/2 and c_k = t_{N-k} above."""
    N = len(t)
    return np.array([t[k] if k <= N // 2 else t[N - k] for k in range(N)], dtype=np.float64)


def circulant_dense(c: np.ndarray) -> np.ndarray:
    """The N x N circulant matrix with first column c."""
    N = len(c)
    i = np.arange(N)
    return c[(i[:, None] - i[None, :]) % N]


def strang_eigs(t: np.ndarray) -> np.ndarray:
    """Eigenvalues of s(T) in discrete-Fourier order (mode j at [j]): the DFT of its
    first column, real because the column is symmetric."""
    return np.fft.fft(strang_first_column(t)).real


def _poly_coeffs(a: int) -> np.ndarray:
    """Coefficients c_k of x^a (1-x)^a = sum_k c_k x^k."""
    c = np.zeros(2 * a + 1)
    for j in range(a + 1):
        c[a + j] = math.comb(a, j) * (-1) ** j
    return c


def riesz_poly_derivative(alpha: float, a: int, x: np.ndarray) -> np.ndarray:
    """d^alpha p / d|x|^alpha for p(x) = x^a (1-x)^a on [0,1] (Section 1):
    sigma_alpha (0D_x^alpha p + xD_1^alpha p), sigma_alpha = -1/(2 cos(alpha pi/2)),
    using the Riemann-Liouville power rule 0D_x^alpha x^k = Gamma(k+1)/Gamma(k+1-alpha) x^{k-alpha}
    and its mirror image for powers of (1-x).  p(1-y) expanded in y gives the
    right-sided coefficients."""
    c = _poly_coeffs(a)
    # p(1-y) = sum_k d_k y^k
    pc = np.polynomial.Polynomial(c)
    d_coef = pc(np.polynomial.Polynomial([1.0, -1.0])).coef
    d_full = np.zeros(len(c))
    d_full[:len(d_coef)] = d_coef
    x = np.asarray(x, dtype=np.float64)
    left = np.zeros_like(x)
    right = np.zeros_like(x)
    for k in range(len(c)):
        if c[k] == 0.0 and d_full[k] == 0.0:
            continue
        g = math.gamma(k + 1.0) / math.gamma(k + 1.0 - alpha)
        left += c[k] * g * np.power(x, k - alpha)
        right += d_full[k] * g * np.power(1.0 - x, k - alpha)
    sigma = -1.0 / (2.0 * math.cos(alpha * math.pi / 2.0))
    return sigma * (left + right)


# ----------------------------------------------------------------------------
# Field families (problem data, Section 4 examples and synthetic workloads)
# ----------------------------------------------------------------------------

def _mesh(coords: List[np.ndarray]) -> List[np.ndarray]:
    """Broadcastable coordinate arrays for a grid of shape (len(c_d), ..., len(c_1))."""
    d = len(coords)
    out = []
    for i in range(d):
        shape = [1] * d
        shape[d - 1 - i] = len(coords[i])
        out.append(coords[i].reshape(shape))
    return out


def _modes_field(amp: np.ndarray, K: int, X: List[np.ndarray]) -> np.ndarray:
    d = len(X)
    g = 0.0
    for flat in range(K ** d):
        ks = []
        r = flat
        for _ in range(d):
            ks.append(r % K + 1)
            r //= K
        term = amp[flat]
        prod = 1.0
        for i in range(d):
            prod = prod * np.sin(ks[i] * np.pi * X[i])
        g = g + term * prod
    return g


def eval_e(spec, X: List[np.ndarray], t: float) -> np.ndarray:
    d = len(X)
    k = spec.kind
    c = spec.c
    shape = np.broadcast_shapes(*[x.shape for x in X])
    if k == "const":
        return np.full(shape, c[0])
    if k == "sumsq_exp":
        s = sum(x ** 2 for x in X)
        return np.broadcast_to((s + math.exp(-t)) / c[0], shape).copy()
    if k == "poly_t":
        p = np.ones(shape)
        for x in X:
            p = p * x ** c[3]
        return c[0] + c[1] * (1.0 + c[2] * t) * p
    if k == "sinprod_cos":
        p = np.ones(shape)
        for x in X:
            p = p * np.sin(np.pi * x)
        return c[0] + c[1] * p * math.cos(t)
    if k == "sine_field":
        g = _modes_field(spec.amp, spec.modes, X)
        return np.broadcast_to(c[0] + c[1] * 0.5 * (1.0 + g / np.abs(spec.amp).sum()), shape).copy()
    raise ValueError(k)


def eval_u_manufactured(spec, X: List[np.ndarray], t: float) -> np.ndarray:
    A, a = spec.c[0], int(spec.c[1])
    p = 1.0
    for x in X:
        p = p * x ** a * (1.0 - x) ** a
    return A * math.exp(-t) * p


def eval_f(spec, espec, alpha, kappa, X: List[np.ndarray], t: float) -> np.ndarray:
    shape = np.broadcast_shapes(*[x.shape for x in X])
    k = spec.kind
    if k == "zero":
        return np.zeros(shape)
    if k == "sine_modes":
        return np.broadcast_to(_modes_field(spec.amp, spec.modes, X), shape).copy()
    if k == "manufactured":
        A, a = spec.c[0], int(spec.c[1])
        d = len(X)
        u = eval_u_manufactured(spec, X, t)
        e = eval_e(espec, X, t)
        f = e * (-u)  # e u_t with u_t = -u
        for i in range(d):
            other = 1.0
            for l in range(d):
                if l != i:
                    other = other * X[l] ** a * (1.0 - X[l]) ** a
            f = f - kappa[i] * A * math.exp(-t) * other * riesz_poly_derivative(alpha[i], a, X[i])
        return np.broadcast_to(f, shape).copy()
    raise ValueError(k)


def eval_psi(spec, X: List[np.ndarray]) -> np.ndarray:
    shape = np.broadcast_shapes(*[x.shape for x in X])
    if spec.kind == "zero":
        return np.zeros(shape)
    if spec.kind == "manufactured":
        return np.broadcast_to(eval_u_manufactured(spec, X, 0.0), shape).copy()
    raise ValueError(spec.kind)


# ----------------------------------------------------------------------------
# The discrete problem (Section 2, eqs. tls/Salpha/Ha/eq0; Section 3, eqs. Pa/tauSalpha/bard)
# ----------------------------------------------------------------------------

def _along(Mx: np.ndarray, X: np.ndarray, i: int) -> np.ndarray:
    """Apply the N_i x N_i matrix Mx along paper axis i (0-based) of X, shape (N_d..N_1)."""
    d = X.ndim
    ax = d - 1 - i
    Y = np.tensordot(Mx, X, axes=([1], [ax]))
    return np.moveaxis(Y, 0, ax)


class OracleProblem:
    """Dense-matrix model of one instance."""

    def __init__(self, inst, ebar: Optional[float] = None):
        self.inst = inst
        self.d = inst.d
        self.N = tuple(int(v) for v in inst.n)
        self.shape = tuple(reversed(self.N))
        self.dt = inst.T / inst.M
        self.h = [(inst.hi[i] - inst.lo[i]) / (self.N[i] + 1) for i in range(self.d)]
        # eq. Salpha: eta_i = kappa_i dt / (2 h_i^alpha_i)
        self.eta = [inst.kappa[i] * self.dt / (2.0 * self.h[i] ** inst.alpha[i]) for i in range(self.d)]
        self.s = [fcd_weights(inst.alpha[i], self.N[i]) for i in range(self.d)]
        self.T = [toeplitz_dense(self.s[i]) for i in range(self.d)]
        self.B = [B_dense(inst.alpha[i], self.N[i]) for i in range(self.d)]
        self.S = [sine_matrix(self.N[i]) for i in range(self.d)]
        self.q = [tau_eigs_cosine(self.s[i]) for i in range(self.d)]
        self.lam = [B_eigs(inst.alpha[i], self.N[i]) for i in range(self.d)]
        self.x_int = [inst.lo[i] + self.h[i] * np.arange(1, self.N[i] + 1) for i in range(self.d)]
        self.x_clo = [inst.lo[i] + self.h[i] * np.arange(0, self.N[i] + 2) for i in range(self.d)]
        self.X_int = _mesh(self.x_int)
        self.X_clo = _mesh(self.x_clo)
        self.ebar = self.compute_ebar() if ebar is None else float(ebar)
        self._mu = None

    # -- data at t_{m+1/2}
    def t_half(self, m: int) -> float:
        return (m + 0.5) * self.dt

    def e_at(self, t: float) -> np.ndarray:
        return eval_e(self.inst.e, self.X_int, t)

    def f_closure_at(self, t: float) -> np.ndarray:
        return eval_f(self.inst.f, self.inst.e, self.inst.alpha, self.inst.kappa, self.X_clo, t)

    def psi(self) -> np.ndarray:
        return eval_psi(self.inst.psi, self.X_int)

    def exact(self, t: float) -> np.ndarray:
        return eval_u_manufactured(self.inst.f, self.X_int, t) * np.ones(self.shape)

    def compute_ebar(self) -> float:
        """eq. bard/dhat: (max + min)/2 of e over the grid and all midpoints t_{m+1/2}."""
        lo, hi = math.inf, -math.inf
        steps = range(self.inst.M) if self.inst.e.time_dependent else range(1)
        for m in steps:
            e = self.e_at(self.t_half(m))
            lo = min(lo, float(e.min()))
            hi = max(hi, float(e.max()))
        return 0.5 * (lo + hi)

    # -- operators
    def apply_B(self, X: np.ndarray) -> np.ndarray:
        """B_alpha = B_{alpha_d} x ... x B_{alpha_1}."""
        Y = X
        for i in range(self.d):
            Y = _along(self.B[i], Y, i)
        return Y

    def apply_S(self, X: np.ndarray) -> np.ndarray:
        """S_alpha = sum_i eta_i (B_d x .. x S_{alpha_i} x .. x B_1) (eq. Salpha)."""
        out = np.zeros(self.shape)
        for i in range(self.d):
            Y = X
            for l in range(self.d):
                Y = _along(self.T[l] if l == i else self.B[l], Y, l)
            out = out + self.eta[i] * Y
        return out

    def apply_A(self, e: np.ndarray, X: np.ndarray) -> np.ndarray:
        """A = B_alpha E + S_alpha (eq. tls)."""
        return self.apply_B(e * X) + self.apply_S(X)

    def F_from_closure(self, fc: np.ndarray) -> np.ndarray:
        """F = (prod_l H_{alpha_l}) f on the closure grid, restricted to the interior
        (eq. eq2.2 and Appendix A).  Each H acts as the (alpha/24, 1-alpha/12, alpha/24)
        stencil on interior indices and as the identity on boundary indices."""
        Y = fc.copy()
        for i in range(self.d):
            a = self.inst.alpha[i]
            Np2 = self.N[i] + 2
            Hm = np.eye(Np2)
            for j in range(1, Np2 - 1):
                Hm[j, j - 1] = a / 24.0
                Hm[j, j] = 1.0 - a / 12.0
                Hm[j, j + 1] = a / 24.0
            Y = _along(Hm, Y, i)
        sl = tuple(slice(1, -1) for _ in range(self.d))
        return Y[sl].copy()

    def rhs(self, e: np.ndarray, F: np.ndarray, u: np.ndarray) -> np.ndarray:
        """b^{(m)} = (B_alpha E - S_alpha) u^{(m)} + dt F^{(m+1/2)} (eq. tls)."""
        return self.apply_B(e * u) - self.apply_S(u) + self.dt * F

    def mu(self) -> np.ndarray:
        """Eigenvalues of B_alpha P_alpha = ebar B_alpha + tau(S_alpha) in the sine basis
        (eqs. Pa, tauSalpha; Lemma le:eig; Lemma Heig; eq. q)."""
        if self._mu is None:
            lamK = np.ones(self.shape)
            for i in range(self.d):
                lamK = lamK * self.lam[i].reshape([-1 if a == self.d - 1 - i else 1 for a in range(self.d)])
            mu = self.ebar * lamK
            for i in range(self.d):
                term = np.ones(self.shape) * self.eta[i]
                for l in range(self.d):
                    v = self.q[l] if l == i else self.lam[l]
                    term = term * v.reshape([-1 if a == self.d - 1 - l else 1 for a in range(self.d)])
                mu = mu + term
            self._mu = mu
        return self._mu

    # -- two-sided form (eqs. equi, Pa, Pls)
    def lam_K(self) -> np.ndarray:
        """Eigenvalues of B_alpha = B_{alpha_d} x ... x B_{alpha_1} in the sine basis
        (Lemma Heig; products of the per-axis eigenvalues)."""
        lamK = np.ones(self.shape)
        for i in range(self.d):
            lamK = lamK * self.lam[i].reshape([-1 if a == self.d - 1 - i else 1 for a in range(self.d)])
        return lamK

    def tauS_eigs(self) -> np.ndarray:
        """Eigenvalues of tau(S_alpha) (eq. tauSalpha) in the sine basis: each Kronecker
        term contributes eta_i q_i times the B eigenvalues of the other axes."""
        out = np.zeros(self.shape)
        for i in range(self.d):
            term = np.ones(self.shape) * self.eta[i]
            for l in range(self.d):
                v = self.q[l] if l == i else self.lam[l]
                term = term * v.reshape([-1 if a == self.d - 1 - l else 1 for a in range(self.d)])
            out = out + term
        return out

    def P_eigs(self) -> np.ndarray:
        """Eigenvalues of P_alpha = ebar I + B^{-1/2} tau(S_alpha) B^{-1/2} (eq. Pa): the
        sine transform diagonalises B_alpha and tau(S_alpha) together (eq. diag)."""
        return self.ebar + self.tauS_eigs() / self.lam_K()

    def apply_B_inv(self, X: np.ndarray) -> np.ndarray:
        """B_alpha^{-1} x through its sine diagonalisation (eq. diag)."""
        return self.apply_sine(self.apply_sine(X) / self.lam_K())

    def apply_P_power(self, X: np.ndarray, power: float) -> np.ndarray:
        """P_alpha^{power} x = S diag(p_K^{power}) S x (eq. Pa, eq. diag)."""
        return self.apply_sine(self.apply_sine(X) * self.P_eigs() ** power)

    def apply_Atilde(self, e: np.ndarray, X: np.ndarray) -> np.ndarray:
        """Atilde = E + B_alpha^{-1} S_alpha (eq. equi)."""
        return e * X + self.apply_B_inv(self.apply_S(X))

    # -- Strang circulant preconditioner (Section 4)
    def strang_m(self) -> np.ndarray:
        """Eigenvalues of ebar c(B_alpha) + c(S_alpha) (the Strang circulants of each
        factor, eqs. Pcir/cirSalpha), in discrete-Fourier order on every axis."""
        def along(v, i):
            return v.reshape([-1 if a == self.d - 1 - i else 1 for a in range(self.d)])
        bB, bS = [], []
        for i in range(self.d):
            N, al = self.N[i], self.inst.alpha[i]
            tb = np.zeros(N)
            tb[0] = 1.0 - al / 12.0
            if N > 1:
                tb[1] = al / 24.0
            bB.append(strang_eigs(tb))
            bS.append(strang_eigs(self.s[i]))
        lamK = np.ones(self.shape)
        for i in range(self.d):
            lamK = lamK * along(bB[i], i)
        m = self.ebar * lamK
        for i in range(self.d):
            term = np.ones(self.shape) * self.eta[i]
            for l in range(self.d):
                term = term * along(bS[l] if l == i else bB[l], l)
            m = m + term
        return m

    def apply_strang_prec_inv(self, R: np.ndarray) -> np.ndarray:
        """(ebar c(B) + c(S))^{-1} r by the d-dimensional DFT."""
        return np.real(np.fft.ifftn(np.fft.fftn(R) / self.strang_m()))

    def apply_sine(self, X: np.ndarray) -> np.ndarray:
        Y = X
        for i in range(self.d):
            Y = _along(self.S[i], Y, i)
        return Y

    def apply_prec_inv(self, R: np.ndarray) -> np.ndarray:
        """(B_alpha P_alpha)^{-1} r = S diag(1/mu) S r with S = S_d x ... x S_1 (eq. diag)."""
        return self.apply_sine(self.apply_sine(R) / self.mu())

    # -- dense forms for tiny grids
    def dense_kron(self, mats: List[np.ndarray]) -> np.ndarray:
        """M_d x ... x M_1 for per-axis matrices mats[i] (axis i = 0..d-1)."""
        K = np.ones((1, 1))
        for i in reversed(range(self.d)):
            K = np.kron(K, mats[i])
        return K

    def dense_A(self, e: np.ndarray) -> np.ndarray:
        Bk = self.dense_kron(self.B)
        Sa = np.zeros_like(Bk)
        for i in range(self.d):
            Sa += self.eta[i] * self.dense_kron([self.T[l] if l == i else self.B[l] for l in range(self.d)])
        return Bk @ np.diag(e.ravel()) + Sa

    def dense_BP(self) -> np.ndarray:
        """ebar B_alpha + tau(S_alpha), built from tau(T) = T - H(T) (eqs. tau, Pa, tauSalpha)."""
        Bk = self.dense_kron(self.B)
        tS = np.zeros_like(Bk)
        for i in range(self.d):
            tS += self.eta[i] * self.dense_kron(
                [tau_dense(self.s[l]) if l == i else self.B[l] for l in range(self.d)])
        return self.ebar * Bk + tS

    # -- one Crank-Nicolson step
    def step(self, u: np.ndarray, m: int, x0_mode: int = 0, restart: Optional[int] = None,
             rtol: Optional[float] = None, max_cycles: Optional[int] = None,
             progress: Optional[Callable] = None):
        th = self.t_half(m)
        e = self.e_at(th)
        F = self.F_from_closure(self.f_closure_at(th))
        b = self.rhs(e, F, u)
        x0 = u.copy() if x0_mode == 0 else np.zeros_like(u)
        x, st = gmres_left(lambda v: self.apply_A(e, v), self.apply_prec_inv, b, x0,
                           restart=self.inst.restart if restart is None else restart,
                           rtol=self.inst.rtol if rtol is None else rtol,
                           max_cycles=self.inst.max_cycles if max_cycles is None else max_cycles,
                           progress=progress)
        return x, st


    def step_strang(self, u: np.ndarray, m: int, x0_mode: int = 0, restart: Optional[int] = None,
                    rtol: Optional[float] = None, max_cycles: Optional[int] = None):
        """One step of eq. tls by GMRES left-preconditioned with ebar c(B) + c(S)."""
        th = self.t_half(m)
        e = self.e_at(th)
        F = self.F_from_closure(self.f_closure_at(th))
        b = self.rhs(e, F, u)
        x0 = u.copy() if x0_mode == 0 else np.zeros_like(u)
        return gmres_left(lambda v: self.apply_A(e, v), self.apply_strang_prec_inv, b, x0,
                          restart=self.inst.restart if restart is None else restart,
                          rtol=self.inst.rtol if rtol is None else rtol,
                          max_cycles=self.inst.max_cycles if max_cycles is None else max_cycles)

    def step_two_sided(self, u: np.ndarray, m: int, x0_mode: int = 0,
                       restart: Optional[int] = None, rtol: Optional[float] = None,
                       max_cycles: Optional[int] = None):
        """One step through the two-sided system (eq. Pls): GMRES on
        P^{-1/2} Atilde P^{-1/2} utilde = P^{-1/2} btilde with btilde = B^{-1} b
        (eq. equi) and utilde = P^{1/2} u; then u^{(m+1)} = P^{-1/2} utilde."""
        th = self.t_half(m)
        e = self.e_at(th)
        F = self.F_from_closure(self.f_closure_at(th))
        b = self.rhs(e, F, u)
        rhs = self.apply_P_power(self.apply_B_inv(b), -0.5)

        def op(v):
            return self.apply_P_power(self.apply_Atilde(e, self.apply_P_power(v, -0.5)), -0.5)

        x0 = self.apply_P_power(u, 0.5) if x0_mode == 0 else np.zeros_like(u)
        xt, st = gmres_left(op, lambda r: r, rhs, x0,
                            restart=self.inst.restart if restart is None else restart,
                            rtol=self.inst.rtol if rtol is None else rtol,
                            max_cycles=self.inst.max_cycles if max_cycles is None else max_cycles)
        return self.apply_P_power(xt, -0.5), st


# ----------------------------------------------------------------------------
# Single entries of the operators on grids too large for the dense model
# ----------------------------------------------------------------------------

class PointOracle:
    """One output entry at a time of A = B_alpha E + S_alpha (eq. tls, Salpha, Ha),
    of B P = ebar B_alpha + tau(S_alpha) (eqs. Pa, tauSalpha, tau) and of the source
    operator F (eq. eq2.2), by their definitions.  Only per-axis data is held
    (FCD weights, stencil weights); a Toeplitz or Hankel row is formed when used.
    Grid points J = (j_1, ..., j_d) are 0-based interior indices; arrays have shape
    (N_d, ..., N_1) as in OracleProblem."""

    def __init__(self, inst, ebar: float):
        self.inst = inst
        self.d = inst.d
        self.N = tuple(int(v) for v in inst.n)
        self.dt = inst.T / inst.M
        self.h = [(inst.hi[i] - inst.lo[i]) / (self.N[i] + 1) for i in range(self.d)]
        self.eta = [inst.kappa[i] * self.dt / (2.0 * self.h[i] ** inst.alpha[i]) for i in range(self.d)]
        self.s = [fcd_weights(inst.alpha[i], self.N[i]) for i in range(self.d)]
        self.ebar = float(ebar)

    def _ix(self, J):
        return tuple(reversed(J))

    def _w(self, i, o):
        a = self.inst.alpha[i]
        return 1.0 - a / 12.0 if o == 0 else a / 24.0

    def _neighbours(self, J, axes):
        """(weight, J') of the tridiagonal stencils along `axes` (zero outside)."""
        out = [(1.0, list(J))]
        for i in axes:
            nxt = []
            for w, Jn in out:
                for o in (-1, 0, 1):
                    k = Jn[i] + o
                    if 0 <= k < self.N[i]:
                        J2 = list(Jn)
                        J2[i] = k
                        nxt.append((w * self._w(i, o), J2))
            out = nxt
        return out

    def _line(self, X, J, i):
        idx = list(self._ix(J))
        idx[self.d - 1 - i] = slice(None)
        return X[tuple(idx)]

    def toeplitz_row(self, i, j):
        """Row j of S_{alpha_i}: s_{|j-k|} (eq. eq0)."""
        return self.s[i][np.abs(j - np.arange(self.N[i]))]

    def hankel_row(self, i, j):
        """Row j of H(S_{alpha_i}) (eq. tau; the reading of hankel_dense, 0-based)."""
        N = self.N[i]
        tt = np.zeros(2 * N + 3)
        tt[:N] = self.s[i]
        k = np.arange(N)
        return tt[j + k + 2] + tt[2 * N - j - k]

    def apply_A_at(self, e, X, J) -> float:
        allx = list(range(self.d))
        val = sum(w * e[self._ix(Jn)] * X[self._ix(Jn)] for w, Jn in self._neighbours(J, allx))
        for i in range(self.d):
            row = self.toeplitz_row(i, J[i])
            for w, Jn in self._neighbours(J, [l for l in allx if l != i]):
                val += self.eta[i] * w * float(row @ self._line(X, Jn, i))
        return float(val)

    def apply_BP_at(self, X, J) -> float:
        allx = list(range(self.d))
        val = self.ebar * sum(w * X[self._ix(Jn)] for w, Jn in self._neighbours(J, allx))
        for i in range(self.d):
            row = self.toeplitz_row(i, J[i]) - self.hankel_row(i, J[i])
            for w, Jn in self._neighbours(J, [l for l in allx if l != i]):
                val += self.eta[i] * w * float(row @ self._line(X, Jn, i))
        return float(val)

    def rhs_at(self, e, U, F_J: float, J) -> float:
        """b_J = (B E u)_J - (S u)_J + dt F_J (eq. tls)."""
        allx = list(range(self.d))
        val = sum(w * e[self._ix(Jn)] * U[self._ix(Jn)] for w, Jn in self._neighbours(J, allx))
        for i in range(self.d):
            row = self.toeplitz_row(i, J[i])
            for w, Jn in self._neighbours(J, [l for l in allx if l != i]):
                val -= self.eta[i] * w * float(row @ self._line(U, Jn, i))
        return float(val) + self.dt * F_J

    def F_at(self, f_closure_at, J) -> float:
        """F_J = (prod_l H_{alpha_l}) f at interior J, from f on the closure grid;
        f_closure_at(K) gives f at closure index K (interior j <-> closure j+1)."""
        val = 0.0
        for w, Jn in self._closure_neighbours(J):
            val += w * f_closure_at(Jn)
        return float(val)

    def _closure_neighbours(self, J):
        out = [(1.0, [j + 1 for j in J])]
        for i in range(self.d):
            nxt = []
            for w, Kn in out:
                for o in (-1, 0, 1):
                    K2 = list(Kn)
                    K2[i] += o
                    nxt.append((w * self._w(i, o), K2))
            out = nxt
        return out

    def mu_bounds(self):
        """Bounds mu_min <= mu_K <= mu_max of the eigenvalues of B P (eq. q, Lemma
        Heig): products and sums of the per-axis extremes."""
        lo_l, hi_l, lo_w, hi_w = 1.0, 1.0, self.ebar, self.ebar
        for i in range(self.d):
            lam = B_eigs(self.inst.alpha[i], self.N[i])
            w = self.eta[i] * tau_eigs_cosine(self.s[i]) / lam
            lo_l *= lam.min()
            hi_l *= lam.max()
            lo_w += w.min()
            hi_w += w.max()
        return lo_l * lo_w, hi_l * hi_w


# ----------------------------------------------------------------------------
# GMRES(m), left preconditioned (Section 3, eq. one-sided; Lemma Krylov; Section 4 stop rule)
# ----------------------------------------------------------------------------

def gmres_left(apply_A: Callable, apply_Minv: Callable, b: np.ndarray, x0: np.ndarray,
               restart: int, rtol: float, max_cycles: int = 10,
               progress: Optional[Callable] = None):
    """Textbook restarted GMRES on M^{-1} A x = M^{-1} b (Saad-Schultz): modified
    Gram-Schmidt Arnoldi, Givens rotations on the Hessenberg matrix.  Stops at the
    first iteration k with ||M^{-1}(b - A x_k)||_2 <= rtol ||M^{-1}(b - A x_0)||_2, the
    residual norm being the least-squares value |g_{k+1}|.  progress(iteration,
    relative residual), when given, is called after every iteration (reporting only)."""
    x = x0.copy()
    z = apply_Minv(b - apply_A(x))
    beta0 = float(np.linalg.norm(z))
    stats = dict(iters=0, cycles=0, converged=False, beta0=beta0, rel_pres=0.0)
    if beta0 == 0.0:
        stats["converged"] = True
        return x, stats
    beta = beta0
    for cycle in range(max_cycles):
        stats["cycles"] = cycle + 1
        V = [z / beta]
        Hm = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        k = 0
        done = False
        for j in range(restart):
            w = apply_Minv(apply_A(V[j]))
            for i in range(j + 1):
                Hm[i, j] = float(np.vdot(V[i], w))
                w = w - Hm[i, j] * V[i]
            Hm[j + 1, j] = float(np.linalg.norm(w))
            for i in range(j):
                a, c = Hm[i, j], Hm[i + 1, j]
                Hm[i, j] = cs[i] * a + sn[i] * c
                Hm[i + 1, j] = -sn[i] * a + cs[i] * c
            a, c = Hm[j, j], Hm[j + 1, j]
            r = math.hypot(a, c)
            cs[j] = a / r
            sn[j] = c / r
            Hm[j, j] = r
            Hm[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            stats["iters"] += 1
            k = j + 1
            stats["rel_pres"] = abs(g[j + 1]) / beta0
            if progress is not None:
                progress(stats["iters"], stats["rel_pres"])
            if abs(g[j + 1]) <= rtol * beta0:
                done = True
                break
            hn = np.linalg.norm(w)
            if hn == 0.0:
                done = True
                break
            V.append(w / hn)
        y = np.linalg.solve(np.triu(Hm[:k, :k]), g[:k])
        for i in range(k):
            x = x + y[i] * V[i]
        if done:
            stats["converged"] = abs(g[k]) <= rtol * beta0
            break
        z = apply_Minv(b - apply_A(x))
        beta = float(np.linalg.norm(z))
        if beta <= rtol * beta0:
            stats["converged"] = True
            break
    return x, stats


# ----------------------------------------------------------------------------
# Time loop
# ----------------------------------------------------------------------------

def run(inst, steps: Optional[int] = None, ebar: Optional[float] = None, x0_mode: int = 0,
        u0: Optional[np.ndarray] = None, m0: int = 0, track_error: bool = False,
        callback: Optional[Callable] = None, two_sided: bool = False, strang: bool = False) -> Dict:
    """Run `steps` Crank-Nicolson steps (default: all M) from u0 (default psi) starting
    at step index m0, each solved in the one-sided form (eq. one-sided) or, with
    two_sided, in the two-sided form (eq. Pls), or with strang, with the Strang
    circulant preconditioner.  Returns the final u (flat, x_1 fastest) and per-step
    stats."""
    P = OracleProblem(inst, ebar=ebar)
    u = P.psi() if u0 is None else np.asarray(u0, dtype=np.float64).reshape(P.shape).copy()
    steps = inst.M - m0 if steps is None else steps
    iters = []
    err = 0.0
    for m in range(m0, m0 + steps):
        if two_sided:
            u, st = P.step_two_sided(u, m, x0_mode=x0_mode)
        elif strang:
            u, st = P.step_strang(u, m, x0_mode=x0_mode)
        else:
            u, st = P.step(u, m, x0_mode=x0_mode)
        iters.append(st["iters"])
        if callback is not None:
            callback(m, u, st)
        if track_error:
            ex = P.exact((m + 1) * P.dt)
            err = max(err, math.sqrt(float(np.prod(P.h)) * float(((ex - u) ** 2).sum())))
    return dict(u=u.ravel().copy(), iters=iters, mean_iters=float(np.mean(iters)) if iters else 0.0,
                err_l2=err, ebar=P.ebar)
