"""Pins of the oracle's periodic C^2 cubic spline (section 3.3.2, "Interpolation"; section 3.5)."""

import numpy as np
import pytest
from scipy.interpolate import BSpline, CubicSpline

import oracle as O


def _field(g, seed=0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(g.shape)


def test_bspline_weights_are_the_cubic_bspline_basis():
    # scipy's cardinal cubic B-spline on knots -2..2, sampled at the offsets
    b = BSpline.basis_element(np.arange(-2.0, 3.0), extrapolate=False)
    th = np.linspace(0.0, 0.999, 37)
    w = O.bspline_weights(th)
    # weight of offset a is the basis centred at node a evaluated at distance theta - a
    for a, wa in zip((-1, 0, 1, 2), w):
        assert np.allclose(wa, b(th - a), atol=1e-15)
    assert np.allclose(sum(w), 1.0, atol=1e-15)


def test_coefficients_solve_the_circulant_system():
    g = O.Grid(16, 24)
    f = _field(g)
    c = O.spline_coefficients(g, f)
    # apply the tensor product of (1, 4, 1)/6 along both axes
    r1 = (np.roll(c, 1, 0) + 4 * c + np.roll(c, -1, 0)) / 6.0
    r = (np.roll(r1, 1, 1) + 4 * r1 + np.roll(r1, -1, 1)) / 6.0
    assert np.abs(r - f).max() < 1e-13


def test_node_reproduction():
    g = O.Grid(20, 12)
    f = _field(g, 1)
    assert np.abs(O.interpolate(g, f, g.X) - f).max() < 1e-13
    # integer shifts are exact cyclic shifts
    Xs = g.X + np.array([3 * g.h[0], -2 * g.h[1]])[:, None, None]
    assert np.abs(O.interpolate(g, f, Xs) - np.roll(np.roll(f, -3, 0), 2, 1)).max() < 1e-13


def test_against_scipy_periodic_cubic_spline():
    """Tensor-product periodic spline: interpolate along x2 per row, then along x1."""
    g = O.Grid(16, 20)
    f = _field(g, 2)
    rng = np.random.default_rng(3)
    pts = rng.uniform(-2.0, 8.0, size=(2, 25))   # includes points outside [0, 2 pi)
    ours = O.interpolate(g, f, pts)
    x1 = np.arange(g.n1 + 1) * g.h[0]
    x2 = np.arange(g.n2 + 1) * g.h[1]
    ref = np.empty(pts.shape[1])
    for p in range(pts.shape[1]):
        col = np.empty(g.n1)
        for i in range(g.n1):
            row = np.append(f[i], f[i, 0])
            col[i] = CubicSpline(x2, row, bc_type="periodic")(np.mod(pts[1, p], 2 * np.pi))
        ref[p] = CubicSpline(x1, np.append(col, col[0]), bc_type="periodic")(np.mod(pts[0, p], 2 * np.pi))
    assert np.abs(ours - ref).max() < 1e-12


@pytest.mark.parametrize("k1,k2", [(1, 0), (3, -2), (7, 5)])
def test_fourier_mode_closed_form(k1, k2):
    """Spline of exp(i k x) at x_j + theta h: exp(i k x_j) sum_a w_a(theta) exp(i k a h) / ((2 + cos kh)/3), per axis."""
    g = O.Grid(32, 32)
    rng = np.random.default_rng(4)
    th = rng.uniform(0, 1, size=(2,) + g.shape)
    X = g.X + th * np.array(g.h)[:, None, None]
    re = np.cos(k1 * g.X[0] + k2 * g.X[1])
    im = np.sin(k1 * g.X[0] + k2 * g.X[1])
    got = O.interpolate(g, re, X) + 1j * O.interpolate(g, im, X)

    def axis(k, h, t):
        w = O.bspline_weights(t)
        s = sum(wa * np.exp(1j * k * a * h) for a, wa in zip((-1, 0, 1, 2), w))
        return s / ((2 + np.cos(k * h)) / 3)

    exact = np.exp(1j * (k1 * g.X[0] + k2 * g.X[1])) * axis(k1, g.h[0], th[0]) * axis(k2, g.h[1], th[1])
    assert np.abs(got - exact).max() < 1e-12


def test_fourth_order_accuracy():
    """Interpolation error of a smooth field decays like h^4."""
    errs = []
    for n in (32, 64, 128):
        g = O.Grid(n, n)
        f = np.sin(g.X[0]) * np.cos(2 * g.X[1])
        X = g.X + 0.37 * np.array(g.h)[:, None, None]
        ex = np.sin(X[0]) * np.cos(2 * X[1])
        errs.append(np.abs(O.interpolate(g, f, X) - ex).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12 < r1 < 20 and 12 < r2 < 20
