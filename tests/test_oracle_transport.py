"""Pins of the oracle's semi-Lagrangian transport (section 3.3.2; eqs. e:characteristic,
e:state-slm, e:adj-slm; the adjoint-error study of section 4.1.3)."""

import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.interpolate import CubicSpline

import oracle as O
import synth


def test_zero_velocity_is_identity():
    g = O.Grid(32, 32)
    rng = np.random.default_rng(0)
    m0 = rng.standard_normal(g.shape)
    v = np.zeros((2,) + g.shape)
    for d in (-1, 1):
        assert np.array_equal(O.trace(g, v, 0.25, d), g.X)
    assert np.abs(O.transport_state(g, v, m0, 4) - m0).max() < 1e-13
    Xa = O.trace(g, v, 0.25, 1)
    assert np.abs(O.adjoint_factor(g, v, Xa, 0.25) - 1.0).max() < 1e-15


def test_constant_velocity_trace_and_integer_shift():
    g = O.Grid(32, 40)
    nt = 4
    ht = 1.0 / nt
    # per step the displacement is exactly (2 cells, -1 cell)
    c = np.array([2 * g.h[0] / ht, -1 * g.h[1] / ht])
    v = np.broadcast_to(c[:, None, None], (2,) + g.shape).copy()
    Xf = O.trace(g, v, ht, -1)
    assert np.abs(Xf - (g.X - ht * c[:, None, None])).max() < 1e-13
    rng = np.random.default_rng(1)
    m0 = rng.standard_normal(g.shape)
    m1 = O.transport_state(g, v, m0, nt)
    exact = np.roll(np.roll(m0, 2 * nt, 0), -1 * nt, 1)
    assert np.abs(m1 - exact).max() < 1e-12


def test_constant_velocity_general_shift_fourth_order():
    """A constant velocity shifts exactly; the only error is the spline's, O(h^4).

    The per-step displacement is held at (2.37, -1.61) cells on every grid so
    that the interpolation fractions, and with them the error constants, agree.
    """
    errs = []
    nt = 3
    for n in (32, 64, 128):
        g = O.Grid(n, n)
        c = np.array([2.37 * g.h[0], -1.61 * g.h[1]]) * nt
        v = np.broadcast_to(c[:, None, None], (2,) + g.shape).copy()
        m0 = np.sin(g.X[0]) * np.cos(2 * g.X[1]) + 0.3 * np.cos(3 * g.X[0] + g.X[1])
        m1 = O.transport_state(g, v, m0, nt)
        Y = g.X - c[:, None, None]
        exact = np.sin(Y[0]) * np.cos(2 * Y[1]) + 0.3 * np.cos(3 * Y[0] + Y[1])
        errs.append(np.abs(m1 - exact).max())
    assert 13 < errs[0] / errs[1] < 19 and 14 < errs[1] / errs[2] < 18


def _departure_exact(x, ht, sign):
    """Accurate solution of dX/dt = sign * v*(X) over ht, analytic v*."""
    def rhs(_, y):
        return sign * 0.5 * np.array([np.sin(y[1]) * np.cos(y[0]), -np.sin(y[0]) * np.cos(y[1])])
    return solve_ivp(rhs, (0, ht), x, rtol=1e-12, atol=1e-13).y[:, -1]


@pytest.mark.parametrize("direction", [-1, 1])
def test_heun_trace_third_order_local_error(direction):
    """Heun departure points converge to the exact characteristic like ht^3 per step."""
    g = O.Grid(128, 128)
    v = synth.smooth_a_velocity(128, 128)
    pts = [(5, 17), (40, 90), (101, 63)]
    errs = []
    for ht in (0.8, 0.4, 0.2):
        X = O.trace(g, v, ht, direction)
        e = 0.0
        for (i, j) in pts:
            ex = _departure_exact(g.X[:, i, j], ht, direction)
            e = max(e, np.abs(X[:, i, j] - ex).max())
        errs.append(e)
    assert 6.0 < errs[0] / errs[1] < 10.0
    assert 6.0 < errs[1] / errs[2] < 10.0


def _compressive_velocity(g):
    return np.stack([0.3 * np.sin(g.X[0]) + 0.1 * np.cos(g.X[1]), 0.2 * np.sin(g.X[1] + g.X[0])])


def _adjoint_map(g, v, lam1, nt):
    ht = 1.0 / nt
    Xa = O.trace(g, v, ht, +1)
    gam = O.adjoint_factor(g, v, Xa, ht)
    return O.solve_adjoint(g, Xa, gam, lam1, nt)[0]


def test_adjoint_conserves_mass_second_order():
    """-d_t lam - div(lam v) = 0 conserves int lam; the SL scheme does so to O(ht^2)."""
    g = O.Grid(64, 64)
    v = _compressive_velocity(g)
    lam1 = 1.0 + 0.5 * np.cos(g.X[0]) * np.sin(2 * g.X[1])
    mass1 = lam1.sum()
    errs = []
    for nt in (4, 8, 16):
        errs.append(abs(_adjoint_map(g, v, lam1, nt).sum() - mass1) / mass1)
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0
    assert errs[2] < 1e-3


def test_state_and_adjoint_are_transposes_up_to_discretisation():
    """<C m, lam> = <m, C^T lam> (the continuous identity); the gap shrinks with nt."""
    g = O.Grid(48, 48)
    v = _compressive_velocity(g)
    rng = np.random.default_rng(5)
    m0 = np.cos(g.X[0] + 2 * g.X[1]) + 0.2 * np.sin(3 * g.X[0])
    lam1 = np.sin(g.X[0]) * np.cos(g.X[1]) + 0.5
    gaps = []
    for nt in (4, 8, 16, 32):
        Cm = O.transport_state(g, v, m0, nt)
        CTl = _adjoint_map(g, v, lam1, nt)
        a, b = float(np.sum(Cm * lam1)), float(np.sum(m0 * CTl))
        gaps.append(abs(a - b) / abs(a))
    assert all(gaps[i + 1] < gaps[i] for i in range(3))
    del rng


def test_adjoint_error_decreases_with_nt():
    """delta_ADJ = |<Cm,Cm> - <C^T C m, m>| / |<Cm,Cm>| (section 4.1.3) decreases with nt."""
    g = O.Grid(64, 64)
    v = synth.smooth_a_velocity(64, 64, 1.0)
    m0 = synth.smooth_a_template(64, 64)
    vals = []
    for nt in (2, 4, 8):
        Cm = O.transport_state(g, v, m0, nt)
        CTCm = _adjoint_map(g, v, Cm, nt)
        vals.append(abs(np.sum(Cm * Cm) - np.sum(CTCm * m0)) / abs(np.sum(Cm * Cm)))
    assert vals[0] > 4 * vals[1] > 0 and vals[1] > 2 * vals[2] > 0


def _scipy_interp(g, f, pts):
    """Tensor-product periodic cubic spline from scipy: along x2 per row, then along x1."""
    x1 = np.arange(g.n1 + 1) * g.h[0]
    x2 = np.arange(g.n2 + 1) * g.h[1]
    flat = pts.reshape(2, -1)
    rows = CubicSpline(x2, np.concatenate([f, f[:, :1]], axis=1), axis=1, bc_type="periodic")
    along2 = rows(np.mod(flat[1], 2 * np.pi))          # (n1, P): row splines at each point's x2
    out = np.empty(flat.shape[1])
    for p in range(flat.shape[1]):
        col = np.append(along2[:, p], along2[0, p])
        out[p] = CubicSpline(x1, col, bc_type="periodic")(np.mod(flat[0, p], 2 * np.pi))
    return out.reshape(pts.shape[1:])


def test_brute_force_state_and_adjoint_with_scipy_splines():
    """SL state and adjoint on a 12x16 grid rebuilt from scipy's periodic splines and the
    analytic divergence, step by step (Heun trace; transport; Heun factor)."""
    g = O.Grid(12, 16)
    X1, X2 = g.X
    v = np.stack([0.6 * np.sin(X2) * np.cos(X1) + 0.2 * np.sin(X1), -0.6 * np.sin(X1) * np.cos(X2)])
    div = 0.2 * np.cos(X1)
    m0 = np.cos(X1 + 2 * X2) + 0.5 * np.sin(3 * X1)
    lam1 = np.sin(X1) * np.cos(X2) + 0.3
    nt = 3
    ht = 1.0 / nt

    def heun(sign):
        Xs = g.X + sign * ht * v
        vs = np.stack([_scipy_interp(g, v[0], Xs), _scipy_interp(g, v[1], Xs)])
        return g.X + sign * 0.5 * ht * (v + vs)

    Xf, Xa = heun(-1.0), heun(+1.0)
    m = m0
    for _ in range(nt):
        m = _scipy_interp(g, m, Xf)
    dD = _scipy_interp(g, div, Xa)
    gam = 1 + 0.5 * ht * (dD + div) + 0.5 * ht * ht * dD * div
    lam = lam1
    for _ in range(nt):
        lam = gam * _scipy_interp(g, lam, Xa)
    assert np.abs(O.transport_state(g, v, m0, nt) - m).max() < 1e-12
    assert np.abs(_adjoint_map(g, v, lam1, nt) - lam).max() < 1e-12
