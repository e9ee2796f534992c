"""FP64 numpy oracle of the semi-Lagrangian (SL) Gauss--Newton--Krylov path.

TEST INFRASTRUCTURE ONLY (see the package docstring): the product path never
imports this module.

Conventions (stated once, used everywhere below)
------------------------------------------------
* Periodic grid on [0, 2*pi)^d, d = 2 or 3, with n1 x n2 (x n3) nodes,
  x_i = 2*pi*i/n (the paper's (-pi, pi)^2 is the same torus, shifted; the
  method has nothing specific to d = 2, section 1 "Limitations and Unresolved
  Issues").  Arrays are indexed [i1, i2(, i3)] with the last index the fastest
  axis; a velocity is an array of shape (d, n1, n2(, n3)).
* Pseudospectral calculus (section 3.2): unnormalised forward DFT, 1/N on the
  inverse; odd-order symbols (gradient, divergence) drop the Nyquist mode,
  even-order symbols (the regulariser) keep it.
* Interpolation (section 3.3.2, "Interpolation"; section 3.5): the C^2 periodic
  cubic spline, i.e. the tensor-product cubic B-spline whose coefficients solve
  the periodic system (c[i-1] + 4 c[i] + c[i+1]) / 6 = f[i] along each axis.
* Time grid t^j = j*ht, ht = 1/nt (section 3.2).  Time integrals over [0, 1]
  use the composite trapezoid rule on t^0..t^nt.
* Parity status: every function here is pinned by a test in
  ``tests/test_oracle_*.py`` (closed forms, library routines, invariants,
  finite differences, brute force on tiny grids).
"""

from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field, replace

import numpy as np

__all__ = [
    "Grid", "Params", "Level", "Linearization",
    "fft_grad", "fft_div", "reg_symbol", "apply_reg", "apply_proj", "leray",
    "spline_coefficients", "bspline_weights", "interpolate",
    "trace", "adjoint_factor", "solve_state", "transport_state", "solve_adjoint",
    "trapezoid_weights", "linearize", "objective", "gradient",
    "incremental_state", "gn_transport_part", "fn_transport_part", "transport_part", "hessian_matvec",
    "prec_reg", "split_scale", "lowpass", "restrict", "prolong",
    "split_matvec", "chebyshev", "lanczos_max", "splitmix64", "splitmix64_uniform",
    "TwoLevel", "setup_two_level", "apply_two_level",
    "pcg", "pcg_reestimating", "reestimate_emax", "newton_solve", "inner_l2",
    "rk2a_forward_op", "rk2a_adjoint_op", "rk2a_state_source", "rk2a_adjoint_source", "rk2a_integrand",
    "rk2a_heun", "rk2a_solve_state", "rk2a_solve_adjoint", "rk2a_incremental_state", "rk2a_transport_part",
]


# ---------------------------------------------------------------------------
# Grid and parameters
# ---------------------------------------------------------------------------

class Grid:
    """Regular periodic grid in d = 2 or 3 dimensions, cell size h_i = 2*pi/n_i (section 3.2).

    K[i]: wave numbers along axis i (Nyquist -n_i/2); Ko[i]: the same with the
    Nyquist mode zeroed (odd-order symbols); X: node coordinates, shape (d,) + shape.
    """

    def __init__(self, *n: int):
        if len(n) not in (2, 3):
            raise ValueError("a grid has 2 or 3 axes")
        if any(int(ni) % 2 for ni in n):
            raise ValueError("grid sizes must be even")
        self.n = tuple(int(ni) for ni in n)
        self.d = len(self.n)
        self.n1, self.n2 = self.n[0], self.n[1]
        if self.d == 3:
            self.n3 = self.n[2]
        self.shape = self.n
        self.N = int(np.prod(self.n))
        self.h = tuple(2.0 * math.pi / ni for ni in self.n)
        self.cell = float(np.prod(self.h))
        k = [np.fft.fftfreq(ni, 1.0 / ni) for ni in self.n]
        ko = []
        for ni, ki in zip(self.n, k):
            ki = ki.copy()
            ki[ni // 2] = 0.0
            ko.append(ki)
        self.K = np.meshgrid(*k, indexing="ij")
        self.Ko = np.meshgrid(*ko, indexing="ij")
        self.K1, self.K2 = self.K[0], self.K[1]
        self.K1o, self.K2o = self.Ko[0], self.Ko[1]
        idx = np.meshgrid(*[np.arange(ni, dtype=np.float64) for ni in self.n], indexing="ij")
        self.X = np.stack([I * hi for I, hi in zip(idx, self.h)])

    def coarse(self) -> "Grid":
        return Grid(*(ni // 2 for ni in self.n))


@dataclass
class Params:
    """Problem parameters (section 3.5 lists the paper's settings).

    reg: 1, 2, 3 for the H1, H2, H3 seminorm (eq. e:varopt:regv).
    proj: 0 for the compressible case (K = identity), 1 for the Leray
          projection (the incompressible case, w = 0).
    hessian: "gn" for the Gauss--Newton matvec, "fn" for the full-Newton one
          (eq. e:hessian-matvec with every lambda term kept).
    transport: "sl" for the semi-Lagrangian scheme (section 3.3.2), "rk2a" for
          the stabilised RK2 scheme (section 3.3.1 and the appendix "Stabilized
          RK2 Scheme"): the transport equations in antisymmetric form,
          pseudospectral in space, Heun's method in time.
    """
    nt: int
    beta: float
    reg: int = 2
    proj: int = 0
    hessian: str = "gn"
    transport: str = "sl"


# ---------------------------------------------------------------------------
# Pseudospectral operators (section 3.2; eq. e:diffopregv; Leray operator)
# ---------------------------------------------------------------------------

def _fft(u):
    return np.fft.fftn(u)


def _ifft_real(U):
    return np.fft.ifftn(U).real


def _dot(a, b):
    """sum_i a[i] b[i] over the d components, in axis order."""
    out = a[0] * b[0]
    for i in range(1, len(a)):
        out = out + a[i] * b[i]
    return out


def fft_grad(g: Grid, u):
    """Spectral gradient of a scalar field: (d1 u, ..., dd u)."""
    U = _fft(u)
    return np.stack([_ifft_real(1j * Ki * U) for Ki in g.Ko])


def fft_div(g: Grid, v):
    """Spectral divergence of a vector field."""
    S = 1j * g.Ko[0] * _fft(v[0])
    for i in range(1, g.d):
        S = S + 1j * g.Ko[i] * _fft(v[i])
    return _ifft_real(S)


def reg_symbol(g: Grid, reg: int):
    """Symbol a(k) of the regularisation operator A (eq. e:diffopregv).

    A = -Laplacian (H1), Laplacian^2 (H2), -Laplacian^3 (H3): a(k) = |k|^(2 reg)
    (the H3 sign is the one that makes A the positive semidefinite first
    variation of the seminorm).
    """
    return _dot(g.K, g.K) ** reg


def apply_reg(g: Grid, v, reg: int):
    a = reg_symbol(g, reg)
    return np.stack([_ifft_real(a * _fft(v[c])) for c in range(g.d)])


def leray(g: Grid, b):
    """Leray projection K[b] = b - grad Laplacian^{-1} div b (section 3.1)."""
    Bs = [_fft(b[c]) for c in range(g.d)]
    k2 = _dot(g.Ko, g.Ko)
    safe = np.where(k2 > 0, k2, 1.0)
    kb = _dot(g.Ko, Bs) / safe
    kb = np.where(k2 > 0, kb, 0.0)
    return np.stack([_ifft_real(Bs[c] - g.Ko[c] * kb) for c in range(g.d)])


def apply_proj(g: Grid, b, proj: int):
    return b if proj == 0 else leray(g, b)


def inner_l2(g: Grid, a, b) -> float:
    """Discrete L2 inner product: cell area times the Euclidean product."""
    return g.cell * float(np.sum(a * b))


# ---------------------------------------------------------------------------
# Periodic cubic spline (section 3.3.2, "Interpolation"; section 3.5)
# ---------------------------------------------------------------------------

def spline_coefficients(g: Grid, f):
    """B-spline coefficients c of the periodic cubic spline through f.

    Along each axis the coefficients solve the circulant system
    (c[i-1] + 4 c[i] + c[i+1]) / 6 = f[i]; a circulant system is diagonal in
    Fourier space, with eigenvalue (2 + cos(2 pi k / n)) / 3 per axis.
    """
    b = (2.0 + np.cos(2.0 * np.pi * g.K[0] / g.n[0])) / 3.0
    for i in range(1, g.d):
        b = b * ((2.0 + np.cos(2.0 * np.pi * g.K[i] / g.n[i])) / 3.0)
    return _ifft_real(_fft(f) / b)


def bspline_weights(theta):
    """Uniform cubic B-spline weights for the offsets -1, 0, 1, 2 at fraction theta."""
    t = theta
    return (
        (1.0 - t) ** 3 / 6.0,
        (3.0 * t ** 3 - 6.0 * t ** 2 + 4.0) / 6.0,
        (-3.0 * t ** 3 + 3.0 * t ** 2 + 3.0 * t + 1.0) / 6.0,
        t ** 3 / 6.0,
    )


def _eval_coefficients(g: Grid, c, X):
    """Tensor-product cubic B-spline with coefficients c at the points X: the 4^d stencil
    nodes floor(s_i) - 1 .. floor(s_i) + 2 (periodic) per axis, s_i = X_i / h_i."""
    s = [X[i] / g.h[i] for i in range(g.d)]
    f = [np.floor(si) for si in s]
    w = [bspline_weights(si - fi) for si, fi in zip(s, f)]
    base = [fi.astype(np.int64) for fi in f]
    out = np.zeros(np.shape(s[0]))
    for offs in itertools.product(range(4), repeat=g.d):
        wt = w[0][offs[0]]
        for i in range(1, g.d):
            wt = wt * w[i][offs[i]]
        idx = tuple(np.mod(base[i] + offs[i] - 1, g.n[i]) for i in range(g.d))
        out += wt * c[idx]
    return out


def interpolate(g: Grid, f, X):
    """Value at the points X (shape (d, ...), radians) of the spline through f."""
    return _eval_coefficients(g, spline_coefficients(g, f), X)


# ---------------------------------------------------------------------------
# Characteristics and transport (section 3.3.2; eqs. e:characteristic,
# e:state-slm, e:adj-slm, e:inc-state-slm, e:inc-adj-slm)
# ---------------------------------------------------------------------------

def trace(g: Grid, v, ht: float, direction: int):
    """Departure points of one SL step by Heun's method (section 3.3.2).

    direction = -1: characteristic of the forward equations (dX/dt = v traced
    back over one step): X* = x - ht v(x), X = x - ht/2 (v(x) + v(X*)).
    direction = +1: characteristic of the backward (adjoint) equations, which
    are transported by -v in reversed time: the same formulas with +ht.
    """
    s = float(direction)
    Xs = g.X + s * ht * v
    vs = np.stack([interpolate(g, v[c], Xs) for c in range(g.d)])
    return g.X + s * 0.5 * ht * (v + vs)


def adjoint_factor(g: Grid, v, Xa, ht: float):
    """Heun step of d(lambda)/ds = lambda div v along the adjoint characteristic.

    The adjoint equation -d_t lambda - v.grad lambda - lambda div v = 0
    (eq. e:adj-slm) reads d(lambda)/ds = lambda div v along dX/ds = -v in
    reversed time s = 1 - t; Heun's method over one step multiplies the
    departure value by 1 + ht/2 (d_D + d_x) + ht^2/2 d_D d_x, where d_x is
    div v at the arrival node and d_D at the departure point.
    """
    dx = fft_div(g, v)
    dD = interpolate(g, dx, Xa)
    return 1.0 + 0.5 * ht * (dD + dx) + 0.5 * ht * ht * dD * dx


def solve_state(g: Grid, Xf, m0, nt: int):
    """State equation (eq. e:state-slm): m^j = m^{j-1} at the departure points."""
    m = [np.array(m0, dtype=np.float64)]
    for _ in range(nt):
        m.append(interpolate(g, m[-1], Xf))
    return m


def transport_state(g: Grid, v, m0, nt: int):
    """m at t = 1 for the initial value m0 transported by the stationary v."""
    Xf = trace(g, v, 1.0 / nt, -1)
    return solve_state(g, Xf, m0, nt)[-1]


def solve_adjoint(g: Grid, Xa, gamma, lam_final, nt: int):
    """Adjoint equation (eq. e:adj-slm), backward from t = 1: list lambda^0..lambda^nt."""
    lam = [None] * (nt + 1)
    lam[nt] = np.array(lam_final, dtype=np.float64)
    for j in range(nt, 0, -1):
        lam[j - 1] = gamma * interpolate(g, lam[j], Xa)
    return lam


def trapezoid_weights(nt: int):
    """Weights of the composite trapezoid rule on t^0..t^nt (sum to 1)."""
    w = np.full(nt + 1, 1.0 / nt)
    w[0] *= 0.5
    w[-1] *= 0.5
    return w


@dataclass
class Level:
    """One grid level of a registration problem (images and parameters)."""
    grid: Grid
    mT: np.ndarray
    mR: np.ndarray
    prm: Params


@dataclass
class Linearization:
    """Quantities fixed for a given v (traced once per Newton iterate)."""
    level: Level
    v: np.ndarray
    Xf: np.ndarray
    Xa: np.ndarray
    gamma: np.ndarray
    m: list
    gradm: list
    Av: np.ndarray
    J: float
    lam: list = field(default=None)
    g: np.ndarray = field(default=None)


# ---------------------------------------------------------------------------
# Stabilised RK2 transport (section 3.3.1; appendix "Stabilized RK2 Scheme")
# ---------------------------------------------------------------------------
# The state equation in antisymmetric form, d_t m + L m = 0 with
#   L u = 1/2 (grad u . v + div(u v) - u div v),
# its first and second variations (adjoint, incremental state, incremental
# adjoint) and the b / b~ integrands of the gradient and the Hessian matvec, as
# the appendix derives them.  Derivatives are spectral (odd orders with the
# Nyquist mode zeroed), products pointwise; every equation is integrated with
# Heun's method on the nt uniform steps (the adjoint ones backward in time).

def rk2a_forward_op(g: Grid, v, divv, u):
    """L u = 1/2 (grad u . v + div(u v) - u div v)."""
    gu = fft_grad(g, u)
    return 0.5 * (_dot(gu, v) + fft_div(g, u * v) - u * divv)


def rk2a_adjoint_op(g: Grid, v, divv, lam):
    """A lam = 1/2 (div(lam v) + grad lam . v + lam div v); the adjoint equation is
    -d_t lam - A lam = 0 (A = -L^T for the discrete operators)."""
    gl = fft_grad(g, lam)
    return 0.5 * (fft_div(g, lam * v) + _dot(gl, v) + lam * divv)


def rk2a_state_source(g: Grid, m, vt):
    """S(m) vt = 1/2 (div(m vt) + grad m . vt - m div vt): the terms of the incremental state
    equation that carry vt (d_t m~ + L m~ + S(m) vt = 0)."""
    gm = fft_grad(g, m)
    return 0.5 * (fft_div(g, m * vt) + _dot(gm, vt) - m * fft_div(g, vt))


def rk2a_adjoint_source(g: Grid, lam, vt):
    """1/2 (div(lam vt) + grad lam . vt + lam div vt): the lambda terms of the full-Newton
    incremental adjoint equation (-d_t lam~ - A lam~ - this = 0)."""
    gl = fft_grad(g, lam)
    return 0.5 * (fft_div(g, lam * vt) + _dot(gl, vt) + lam * fft_div(g, vt))


def rk2a_integrand(g: Grid, lam, m):
    """1/2 (lam grad m - m grad lam + grad(lam m)): the antisymmetric form of lam grad m in b
    (and, with lam~ or m~ in place of lam or m, in b~)."""
    gm, gl, glm = fft_grad(g, m), fft_grad(g, lam), fft_grad(g, lam * m)
    return 0.5 * (lam * gm - m * gl + glm)


def rk2a_heun(op, y, ht, src0=None, src1=None):
    """One step of Heun's method for dy/dt = op(y) + src(t): predictor with the source at the
    start of the step, corrector with the source at its end (src None: no source)."""
    k1 = op(y) + (0.0 if src0 is None else src0)
    k2 = op(y + ht * k1) + (0.0 if src1 is None else src1)
    return y + 0.5 * ht * (k1 + k2)


def rk2a_solve_state(g: Grid, v, m0, nt: int):
    """m^0 = m0, m^j from m^{j-1} by Heun on d_t m = -L m (forward in time)."""
    ht = 1.0 / nt
    divv = fft_div(g, v)
    m = [np.array(m0, dtype=np.float64)]
    for _ in range(nt):
        m.append(rk2a_heun(lambda u: -rk2a_forward_op(g, v, divv, u), m[-1], ht))
    return m


def rk2a_solve_adjoint(g: Grid, v, lam1, nt: int, sources=None):
    """lam^nt = lam1, lam^{j-1} from lam^j by Heun on d_s lam = A lam (+ sources[j]), s = 1 - t
    the backward time; sources (optional, nt + 1 levels) is the known right-hand side."""
    ht = 1.0 / nt
    divv = fft_div(g, v)
    lam = [None] * (nt + 1)
    lam[nt] = np.array(lam1, dtype=np.float64)
    for j in range(nt, 0, -1):
        s0 = None if sources is None else sources[j]
        s1 = None if sources is None else sources[j - 1]
        lam[j - 1] = rk2a_heun(lambda u: rk2a_adjoint_op(g, v, divv, u), lam[j], ht, s0, s1)
    return lam


def rk2a_incremental_state(g: Grid, v, m, vt, nt: int):
    """m~^0 = 0, Heun on d_t m~ = -L m~ - S(m) vt with the source at both ends of each step."""
    ht = 1.0 / nt
    divv = fft_div(g, v)
    src = [-rk2a_state_source(g, mj, vt) for mj in m]
    mt = [np.zeros(g.shape)]
    for j in range(1, nt + 1):
        mt.append(rk2a_heun(lambda u: -rk2a_forward_op(g, v, divv, u), mt[-1], ht, src[j - 1], src[j]))
    return mt


def linearize(L: Level, v) -> Linearization:
    """Trace both characteristics, solve the state equation, evaluate J (RK2A: no
    characteristics, the state by Heun's method)."""
    g, p = L.grid, L.prm
    ht = 1.0 / p.nt
    v = np.array(v, dtype=np.float64)
    if p.transport == "rk2a":
        m = rk2a_solve_state(g, v, L.mT, p.nt)
        gradm = [fft_grad(g, mj) for mj in m]
        Av = apply_reg(g, v, p.reg)
        J = 0.5 * inner_l2(g, m[-1] - L.mR, m[-1] - L.mR) + 0.5 * p.beta * inner_l2(g, v, Av)
        return Linearization(L, v, None, None, None, m, gradm, Av, J)
    Xf = trace(g, v, ht, -1)
    Xa = trace(g, v, ht, +1)
    gamma = adjoint_factor(g, v, Xa, ht)
    m = solve_state(g, Xf, L.mT, p.nt)
    gradm = [fft_grad(g, mj) for mj in m]
    Av = apply_reg(g, v, p.reg)
    J = 0.5 * inner_l2(g, m[-1] - L.mR, m[-1] - L.mR) + 0.5 * p.beta * inner_l2(g, v, Av)
    return Linearization(L, v, Xf, Xa, gamma, m, gradm, Av, J)


def objective(L: Level, v) -> float:
    """J[v] = 1/2 ||m_1 - m_R||^2 + beta/2 <v, A v> (eq. e:varopt:objective, w-term absent)."""
    return linearize(L, v).J


def gradient(lin: Linearization):
    """Reduced gradient g = beta A v + K int_0^1 lambda grad m dt (eq. e:control-elim)."""
    L = lin.level
    g, p = L.grid, L.prm
    w = trapezoid_weights(p.nt)
    if p.transport == "rk2a":
        lam = rk2a_solve_adjoint(g, lin.v, L.mR - lin.m[-1], p.nt)
        b = sum(w[j] * rk2a_integrand(g, lam[j], lin.m[j]) for j in range(p.nt + 1))
    else:
        lam = solve_adjoint(g, lin.Xa, lin.gamma, L.mR - lin.m[-1], p.nt)
        b = sum(w[j] * lam[j] * lin.gradm[j] for j in range(p.nt + 1))
    lin.lam = lam
    lin.g = p.beta * lin.Av + apply_proj(g, b, p.proj)
    return lin.g


def incremental_state(lin: Linearization, vt):
    """Incremental state (eq. e:inc-state-slm), list m~^0..m~^nt.

    Along the forward characteristic d(m~)/dt = f with f = -vt . grad m, a
    source that does not depend on m~, so Heun's step is the trapezoid rule:
    m~^j = I[m~^{j-1} + ht/2 f^{j-1}](X_f) + ht/2 f^j.
    """
    L = lin.level
    g, p = L.grid, L.prm
    ht = 1.0 / p.nt
    f = [-_dot(vt, gm) for gm in lin.gradm]
    mt = [np.zeros(g.shape)]
    for j in range(1, p.nt + 1):
        mt.append(interpolate(g, mt[-1] + 0.5 * ht * f[j - 1], lin.Xf) + 0.5 * ht * f[j])
    return mt


def gn_transport_part(lin: Linearization, vt):
    """Q[vt] = K int_0^1 lam~ grad m dt of the GN matvec (eqs. e:hessian-matvec, e:inc-adj-slm).

    Gauss--Newton drops every term with lambda (section 3.4.1): the incremental
    adjoint solves the adjoint equation with final value -m~(1).
    """
    L = lin.level
    g, p = L.grid, L.prm
    mt = incremental_state(lin, vt)
    lt = solve_adjoint(g, lin.Xa, lin.gamma, -mt[-1], p.nt)
    w = trapezoid_weights(p.nt)
    bt = sum(w[j] * lt[j] * lin.gradm[j] for j in range(p.nt + 1))
    return apply_proj(g, bt, p.proj)


def fn_transport_part(lin: Linearization, vt):
    """Q[vt] = K int_0^1 (lam~ grad m + lam grad m~) dt of the full-Newton matvec
    (eqs. e:hessian-matvec, e:inc-adj-slm; table t:computational-complexity-theoretical, FN rows).

    The incremental adjoint keeps its source: -d_t lam~ - v.grad lam~ - lam~ div v
    = div(lam vt), i.e. along the adjoint characteristic (dX/ds = -v, s = 1 - t)
    d(lam~)/ds = lam~ div v + sigma with sigma = div(lam vt) known on every time
    level.  Heun's step from the departure point (value y_D, source sigma_D) to
    the node (div v = d_x, source sigma_x) gives
    gamma y_D + ht/2 (1 + ht d_x) sigma_D + ht/2 sigma_x, so
    lam~^{j-1} = gamma I[lam~^j](X_a) + ht/2 (1 + ht div v) I[sigma^j](X_a) + ht/2 sigma^{j-1}
    from lam~^nt = -m~^nt.  lam^j is the adjoint of the linearisation point
    (computed here when the gradient has not been evaluated yet).
    """
    L = lin.level
    g, p = L.grid, L.prm
    ht = 1.0 / p.nt
    if lin.lam is None:
        gradient(lin)
    mt = incremental_state(lin, vt)
    sigma = [fft_div(g, lam_j * vt) for lam_j in lin.lam]
    dx = fft_div(g, lin.v)
    lt = [None] * (p.nt + 1)
    lt[p.nt] = -mt[-1]
    for j in range(p.nt, 0, -1):
        lt[j - 1] = (lin.gamma * interpolate(g, lt[j], lin.Xa)
                     + 0.5 * ht * (1.0 + ht * dx) * interpolate(g, sigma[j], lin.Xa)
                     + 0.5 * ht * sigma[j - 1])
    w = trapezoid_weights(p.nt)
    bt = sum(w[j] * (lt[j] * lin.gradm[j] + lin.lam[j] * fft_grad(g, mt[j])) for j in range(p.nt + 1))
    return apply_proj(g, bt, p.proj)


def rk2a_transport_part(lin: Linearization, vt):
    """Q[vt] = K b~ with RK2A transport (appendix "Stabilized RK2 Scheme"): the incremental
    state, the incremental adjoint from -m~(1) (full Newton: with its lambda source terms) and
    b~ = int 1/2 (lam~ grad m - m grad lam~ + grad(lam~ m)) dt (full Newton: plus the same
    form in lam and m~)."""
    L = lin.level
    g, p = L.grid, L.prm
    mt = rk2a_incremental_state(g, lin.v, lin.m, vt, p.nt)
    fn = p.hessian == "fn"
    if fn and lin.lam is None:
        gradient(lin)
    src = [rk2a_adjoint_source(g, lam_j, vt) for lam_j in lin.lam] if fn else None
    lt = rk2a_solve_adjoint(g, lin.v, -mt[-1], p.nt, src)
    w = trapezoid_weights(p.nt)
    bt = sum(w[j] * rk2a_integrand(g, lt[j], lin.m[j]) for j in range(p.nt + 1))
    if fn:
        bt = bt + sum(w[j] * rk2a_integrand(g, lin.lam[j], mt[j]) for j in range(p.nt + 1))
    return apply_proj(g, bt, p.proj)


def transport_part(lin: Linearization, vt):
    """Q[vt] of the matvec the parameters select (Gauss--Newton or full Newton; SL or RK2A)."""
    if lin.level.prm.transport == "rk2a":
        return rk2a_transport_part(lin, vt)
    return fn_transport_part(lin, vt) if lin.level.prm.hessian == "fn" else gn_transport_part(lin, vt)


def hessian_matvec(lin: Linearization, vt):
    """Reduced Hessian matvec H vt = beta A vt + Q[vt] (eq. e:hessian-matvec), GN unless
    the level's parameters ask for the full-Newton form."""
    L = lin.level
    return L.prm.beta * apply_reg(L.grid, vt, L.prm.reg) + transport_part(lin, vt)


# ---------------------------------------------------------------------------
# Preconditioners (section 3.4.2)
# ---------------------------------------------------------------------------

def _reg_symbol_nonzero(g: Grid, reg: int):
    a = reg_symbol(g, reg)
    return np.where(a == 0.0, 1.0, a)


def prec_reg(g: Grid, r, beta: float, reg: int):
    """P_REG^{-1} r: spectral inverse of beta A with the zero symbol replaced by 1 (eq. e:reg-precond)."""
    a = beta * _reg_symbol_nonzero(g, reg)
    return np.stack([_ifft_real(_fft(r[c]) / a) for c in range(g.d)])


def split_scale(g: Grid, r, beta: float, reg: int):
    """S r = (beta A')^{-1/2} r, the split spectral preconditioner's half step."""
    a = beta * _reg_symbol_nonzero(g, reg)
    return np.stack([_ifft_real(_fft(r[c]) / np.sqrt(a)) for c in range(g.d)])


def _low_mask(g: Grid):
    """Ideal low-pass: |k_i| < n_i/4, i.e. the modes a grid of half the size keeps (its Nyquist dropped)."""
    m = np.abs(g.K[0]) < g.n[0] / 4
    for i in range(1, g.d):
        m = m & (np.abs(g.K[i]) < g.n[i] / 4)
    return m


def lowpass(g: Grid, r):
    m = _low_mask(g)
    return np.stack([_ifft_real(_fft(r[c]) * m) for c in range(g.d)])


def _coarse_index(fine: Grid, coarse: Grid):
    """Fine-grid positions of the coarse modes (np.ix_ index) and the mask of the coarse modes
    kept (|k_i| < n_i/2 of the coarse grid along every axis: its Nyquist dropped)."""
    kc = [np.fft.fftfreq(nc, 1.0 / nc).astype(np.int64) for nc in coarse.n]
    ix = np.ix_(*[np.mod(k, nf) for k, nf in zip(kc, fine.n)])
    mask = np.ones(coarse.shape, dtype=bool)
    for i, (k, nc) in enumerate(zip(kc, coarse.n)):
        shape = [1] * coarse.d
        shape[i] = nc
        mask = mask & (np.abs(k) < nc // 2).reshape(shape)
    return ix, mask


def restrict(fine: Grid, coarse: Grid, u):
    """Spectral restriction: keep the modes |k_i| < n_i/4, rescale for the DFT size."""
    ix, mask = _coarse_index(fine, coarse)
    U = _fft(u)
    Uc = U[ix] * (coarse.N / fine.N)
    Uc = Uc * mask
    return _ifft_real(Uc)


def prolong(fine: Grid, coarse: Grid, uc):
    """Spectral prolongation: zero padding of the coarse modes (coarse Nyquist dropped)."""
    ix, mask = _coarse_index(fine, coarse)
    Uc = _fft(uc) * mask * (fine.N / coarse.N)
    U = np.zeros(fine.shape, dtype=np.complex128)
    U[ix] = Uc
    return _ifft_real(U)


def split_matvec(lin: Linearization, s):
    """M s = s + S Q S s: the split spectrally preconditioned Hessian (section 3.4.2)."""
    L = lin.level
    g, p = L.grid, L.prm
    w = split_scale(g, s, p.beta, p.reg)
    return s + split_scale(g, transport_part(lin, w), p.beta, p.reg)


def chebyshev(op, b, emin: float, emax: float, k: int):
    """k steps of the Chebyshev iteration for op x = b from x = 0.

    Textbook Chebyshev acceleration with spectral bounds [emin, emax] (centre
    theta, half width delta); after k steps the residual is
    T_k((theta - A)/delta) / T_k(theta/delta) applied to b.  The k-th update
    needs no new residual, so k steps apply the operator k - 1 times.
    """
    theta = 0.5 * (emax + emin)
    delta = 0.5 * (emax - emin)
    sigma = theta / delta
    rho = 1.0 / sigma
    x = np.zeros_like(b)
    r = np.array(b, dtype=np.float64)
    d = r / theta
    for i in range(k):
        x = x + d
        if i == k - 1:
            break
        r = r - op(d)
        rho_next = 1.0 / (2.0 * sigma - rho)
        d = rho_next * rho * d + (2.0 * rho_next / delta) * r
        rho = rho_next
    return x


def splitmix64(seed: int, count: int):
    """'count' outputs of the SplitMix64 generator (Steele, Lea, Flood 2014) started at 'seed'.

    State update: add the Weyl increment 0x9E3779B97F4A7C15 (mod 2^64); output:
    the state mixed by two xor-shift-multiply rounds and a final xor-shift.
    """
    M = (1 << 64) - 1
    state = seed & M
    out = []
    for _ in range(count):
        state = (state + 0x9E3779B97F4A7C15) & M
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
        out.append(z ^ (z >> 31))
    return out


def splitmix64_uniform(seed: int, count: int):
    """Uniform numbers in [-0.5, 0.5): the top 53 bits of each SplitMix64 output as a fraction, minus 1/2."""
    return np.array([(z >> 11) * (1.0 / (1 << 53)) - 0.5 for z in splitmix64(seed, count)])


def lanczos_max(op, q0, steps: int) -> float:
    """Largest Ritz value of 'steps' Lanczos steps (no re-orthogonalisation) from q0."""
    q = q0 / np.sqrt(np.sum(q0 * q0))
    q_prev = np.zeros_like(q)
    beta = 0.0
    alphas, betas = [], []
    for j in range(steps):
        w = op(q) - beta * q_prev
        alpha = float(np.sum(q * w))
        w = w - alpha * q
        alphas.append(alpha)
        beta = float(np.sqrt(np.sum(w * w)))
        if j == steps - 1 or beta <= 1e-14 * abs(alpha):
            break
        betas.append(beta)
        q_prev, q = q, w / beta
    T = np.diag(alphas) + np.diag(betas, 1) + np.diag(betas, -1)
    return float(np.max(np.linalg.eigvalsh(T)))


@dataclass
class TwoLevel:
    """Data of the nested two-level preconditioner P_2L fixed for one solve.

    solver: "cheb" for CHEB(k) on the coarse split operator, "pcg" for the nested
    PCG(eps) solve (section 3.4.2): CG on the coarse split operator, itself already
    spectrally preconditioned, to the relative residual eps times the tolerance of
    the outer solve."""
    coarse: Level
    emin: float
    emax: float
    cheb_iters: int
    lin_c: Linearization = None
    solver: str = "cheb"
    eps: float = 0.1
    max_inner: int = 200


def setup_two_level(L: Level, cheb_iters=10, lanczos_steps=30, safety=1.05, seed=0x5EED, solver="cheb",
                    eps=0.1):
    """Coarse problem and Chebyshev bounds (section 3.4.2, "Nested Preconditioner").

    The coarse problem restricts m_T and m_R spectrally and keeps nt and beta;
    its operator is the Gauss--Newton one also when the fine solve uses the
    full-Newton matvec (the Chebyshev iteration needs a positive definite
    operator, which the full-Newton Hessian need not be away from the minimiser).
    e_max is the largest Ritz value of Lanczos on the coarse split operator at
    v = 0 (times a safety factor), computed once per solve; e_min is the
    analytic estimate min(1 + 1/(beta a'(k))) over the coarse modes.
    """
    fg = L.grid
    cg = fg.coarse()
    Lc = Level(cg, restrict(fg, cg, L.mT), restrict(fg, cg, L.mR), replace(L.prm, hessian="gn"))
    lin0 = linearize(Lc, np.zeros((cg.d,) + cg.shape))
    q0 = splitmix64_uniform(seed, cg.d * cg.N).reshape((cg.d,) + cg.shape)
    emax = safety * lanczos_max(lambda s: split_matvec(lin0, s), q0, lanczos_steps)
    emin = float(np.min(1.0 + 1.0 / (L.prm.beta * _reg_symbol_nonzero(cg, L.prm.reg))))
    return TwoLevel(Lc, emin, emax, cheb_iters, solver=solver, eps=eps)


def apply_two_level(L: Level, tl: TwoLevel, r, outer_tol: float = 1.0):
    """P_2L^{-1} r = (I - L) r + Pro C(M_c) Res r (section 3.4.2, nested preconditioner), C the
    coarse solver: CHEB(k), or CG on M_c to the relative residual eps * outer_tol (PCG(eps)).
    Returns z, or (z, inner iterations) for PCG(eps)."""
    fg, cg = L.grid, tl.coarse.grid
    high = r - lowpass(fg, r)
    rc = np.stack([restrict(fg, cg, r[c]) for c in range(fg.d)])
    op = lambda s: split_matvec(tl.lin_c, s)
    if tl.solver == "pcg":
        zc, its, _ = pcg(op, rc, lambda x: x, tl.eps * outer_tol, tl.max_inner)
        return high + np.stack([prolong(fg, cg, zc[c]) for c in range(fg.d)]), its
    zc = chebyshev(op, rc, tl.emin, tl.emax, tl.cheb_iters)
    return high + np.stack([prolong(fg, cg, zc[c]) for c in range(fg.d)])


# ---------------------------------------------------------------------------
# Newton--Krylov solver (sections 3.4.1 and 3.5)
# ---------------------------------------------------------------------------

def pcg(op, b, prec, tol: float, maxit: int):
    """Preconditioned CG from x = 0 (Hestenes--Stiefel), Euclidean products.

    Stops when ||r|| <= tol ||b||, at maxit, on non-positive curvature p.Ap <= 0
    (then the current iterate, or P^{-1} b at the first step, is returned), or
    when the preconditioned residual product r.z that gave the step was not
    positive: the preconditioner is then not positive definite (an e_max below
    the spectrum makes CHEB(k) indefinite), the iterate is of no use and the
    status says so.  Returns (x, iterations, status) with status 'ok', 'maxit',
    'negcurv' or 'indefprec'.
    """
    x = np.zeros_like(b)
    r = np.array(b, dtype=np.float64)
    bnorm = float(np.sqrt(np.sum(b * b)))
    if bnorm == 0.0:
        return x, 0, "ok"
    z = prec(r)
    p = z.copy()
    rz = float(np.sum(r * z))
    for it in range(1, maxit + 1):
        q = op(p)
        pq = float(np.sum(p * q))
        if pq <= 0.0:
            return (z if it == 1 else x), it, "negcurv"
        alpha = rz / pq
        x = x + alpha * p
        r = r - alpha * q
        if float(np.sqrt(np.sum(r * r))) <= tol * bnorm:
            return x, it, "ok"
        if not rz > 0.0:
            return x, it, "indefprec"
        z = prec(r)
        rz_next = float(np.sum(r * z))
        p = z + (rz_next / rz) * p
        rz = rz_next
    return x, maxit, "maxit"


def pcg_reestimating(op, b, prec, tol: float, maxit: int, reestimate=None):
    """pcg; when it finds the preconditioner indefinite and reestimate is given, call it (new
    Chebyshev bounds) and run PCG once more from zero.  Returns (x, iterations of both runs,
    status of the last)."""
    x, its, st = pcg(op, b, prec, tol, maxit)
    if st == "indefprec" and reestimate is not None:
        reestimate()
        x, its2, st = pcg(op, b, prec, tol, maxit)
        its += its2
    return x, its, st


def reestimate_emax(tl: TwoLevel, lanczos_steps=30, safety=1.05, seed=0x5EED) -> float:
    """New e_max of CHEB(k) when the preconditioner has turned out indefinite (section 4.2.1:
    re-estimate the eigenvalues once the preconditioner deteriorates): the Lanczos estimate of
    setup_two_level, now on the coarse split operator at the coarse problem's current
    linearisation point."""
    cg = tl.coarse.grid
    q0 = splitmix64_uniform(seed, cg.d * cg.N).reshape((cg.d,) + cg.shape)
    return safety * lanczos_max(lambda s: split_matvec(tl.lin_c, s), q0, lanczos_steps)


def newton_solve(L: Level, v0=None, pc: str = "reg", max_newton=10, gtol_rel=1e-2, gtol_abs=1e-5,
                 max_pcg=500, armijo_c1=1e-4, max_halvings=10, cheb_iters=10, lanczos_steps=30,
                 emax_safety=1.05, seed=0x5EED, g0_norms=None, coarse_solver="cheb", coarse_eps=0.1,
                 emax=None):
    """Globalised inexact GN--Krylov solve (sections 3.4.1, 3.5).

    Newton step H vt = -g by PCG with the forcing term
    eta_k = min(0.5, ||g_k|| / ||g_0||); Armijo backtracking (alpha halved from
    1, sufficient decrease 1e-4 alpha <g, vt>_L2); stop when
    ||g_k||_inf / ||g_0||_inf <= gtol_rel or ||g_k||_inf <= gtol_abs; a solve that reaches
    max_newton iterations first reports status 'maxit' ('linesearch' when backtracking fails).
    pc = 'reg' runs PCG on H with P_REG; pc = '2l' runs PCG on the split system
    M s = -S g with P_2L and takes vt = S s; coarse_solver 'cheb' inverts the coarse
    operator by CHEB(cheb_iters), 'pcg' by PCG(coarse_eps) to coarse_eps * eta_k.  g_0 is the gradient at v = 0;
    g0_norms = (||g_0||_inf, ||g_0||_2) may be passed in to skip computing it.  emax, if given, replaces
    the Lanczos estimate of the Chebyshev bound (a bound known from elsewhere, e.g. rescaled from a
    solve with another beta).  A PCG solve that finds CHEB(k) indefinite ('indefprec') re-estimates
    e_max by Lanczos at the current coarse linearisation and runs again from zero; if that fails too,
    the solve stops with status 'cheb_diverged'.
    """
    g, p = L.grid, L.prm
    v = np.zeros((g.d,) + g.shape) if v0 is None else np.array(v0, dtype=np.float64)
    rep = {"newton_iters": 0, "pcg_iters": 0, "matvecs": 0, "coarse_matvecs": 0,
           "grel": [], "J": [], "status": "ok", "alphas": []}
    tl = setup_two_level(L, cheb_iters, lanczos_steps, emax_safety, seed, coarse_solver, coarse_eps) \
        if pc == "2l" else None
    if tl is not None:
        if emax is not None:
            tl.emax = float(emax)
        rep["emin"], rep["emax"] = tl.emin, tl.emax
    rep["cheb_reestimates"] = 0
    lin = linearize(L, v)
    grad = gradient(lin)
    if g0_norms is None:
        if v0 is None:
            g0 = grad
        else:
            lin0 = linearize(L, np.zeros_like(v))
            g0 = gradient(lin0)
        g0_inf = float(np.max(np.abs(g0)))
        g0_two = float(np.sqrt(np.sum(g0 * g0)))
    else:
        g0_inf, g0_two = g0_norms
    for k in range(max_newton + 1):
        ginf = float(np.max(np.abs(grad)))
        gtwo = float(np.sqrt(np.sum(grad * grad)))
        rep["grel"].append(ginf / g0_inf)
        rep["J"].append(lin.J)
        if ginf / g0_inf <= gtol_rel or ginf <= gtol_abs:
            break
        if k == max_newton:
            rep["status"] = "maxit"      # the Newton limit ended the solve before convergence
            break
        eta = min(0.5, gtwo / g0_two)
        if tl is None:
            def op(x):
                rep["matvecs"] += 1
                return hessian_matvec(lin, x)
            vt, its, st = pcg(op, -grad, lambda r: prec_reg(g, r, p.beta, p.reg), eta, max_pcg)
        else:
            fg, cg = g, tl.coarse.grid
            vc = np.stack([restrict(fg, cg, v[c]) for c in range(fg.d)])
            tl.lin_c = linearize(tl.coarse, vc)

            def op(x):
                rep["matvecs"] += 1
                return split_matvec(lin, x)

            def prec(r):
                if tl.solver == "pcg":
                    z, its_c = apply_two_level(L, tl, r, eta)
                    rep["coarse_matvecs"] += its_c
                    return z
                rep["coarse_matvecs"] += max(tl.cheb_iters - 1, 0)
                return apply_two_level(L, tl, r)
            def reestimate():
                tl.emax = reestimate_emax(tl, lanczos_steps, emax_safety, seed)
                rep["cheb_reestimates"] += 1
            s, its, st = pcg_reestimating(op, -split_scale(g, grad, p.beta, p.reg), prec, eta, max_pcg,
                                          reestimate if tl.solver == "cheb" else None)
            if st == "indefprec":
                rep["pcg_iters"] += its
                rep["status"] = "cheb_diverged"
                break
            vt = split_scale(g, s, p.beta, p.reg)
        rep["pcg_iters"] += its
        slope = inner_l2(g, grad, vt)
        alpha, accepted = 1.0, False
        for _ in range(max_halvings + 1):
            trial = linearize(L, v + alpha * vt)
            if trial.J <= lin.J + armijo_c1 * alpha * slope:
                accepted = True
                break
            alpha *= 0.5
        if not accepted:
            rep["status"] = "linesearch"
            break
        rep["alphas"].append(alpha)
        v = v + alpha * vt
        lin = trial
        grad = gradient(lin)
        rep["newton_iters"] = k + 1
    rep["g0_inf"] = g0_inf
    rep["g0_two"] = g0_two
    return v, rep
