"""Pins of the oracle's pseudospectral operators (section 3.2; eq. e:diffopregv; Leray operator).

Each check compares against a closed form of a trigonometric field, which the
pseudospectral discretisation differentiates exactly (up to rounding).
"""

import math

import numpy as np
import pytest

import oracle as O
import synth


@pytest.fixture(scope="module")
def g():
    return O.Grid(32, 48)


def _xy(g):
    return g.X[0], g.X[1]


def test_gradient_of_smooth_template_closed_form():
    g = O.Grid(64, 64)
    mT = synth.smooth_a_template(64, 64)
    gm = O.fft_grad(g, mT)
    x1, x2 = _xy(g)
    assert np.abs(gm[0] - 0.5 * np.sin(2 * x1)).max() < 1e-13
    assert np.abs(gm[1] - 0.5 * np.sin(2 * x2)).max() < 1e-13


def test_divergence_and_laplacian_of_smooth_velocity():
    g = O.Grid(64, 64)
    v = synth.smooth_a_velocity(64, 64)
    assert np.abs(O.fft_div(g, v)).max() < 1e-13
    # H1: A = -Laplacian; every mode of v* has |k|^2 = 2
    assert np.abs(O.apply_reg(g, v, 1) - 2 * v).max() < 1e-12


@pytest.mark.parametrize("reg", [1, 2, 3])
def test_regulariser_symbol_on_single_mode(g, reg):
    x1, x2 = _xy(g)
    k1, k2 = 3, -5
    u = np.cos(k1 * x1 + k2 * x2)
    v = np.stack([u, 2 * u])
    Av = O.apply_reg(g, v, reg)
    lam = float(k1 * k1 + k2 * k2) ** reg
    assert np.allclose(Av, lam * v, rtol=0, atol=1e-10 * lam)


def test_divergence_of_trig_field(g):
    x1, x2 = _xy(g)
    v = np.stack([np.sin(2 * x1) * np.cos(x2), np.cos(3 * x1) * np.sin(4 * x2)])
    d = O.fft_div(g, v)
    exact = 2 * np.cos(2 * x1) * np.cos(x2) + 4 * np.cos(3 * x1) * np.cos(4 * x2)
    assert np.abs(d - exact).max() < 1e-12


def test_nyquist_convention(g):
    x1, _ = _xy(g)
    u = np.cos(g.n1 / 2 * x1)
    # odd-order operators drop the Nyquist mode
    assert np.abs(O.fft_grad(g, u)).max() < 1e-13
    # the regulariser keeps it with |k| = n/2
    Au = O.apply_reg(g, np.stack([u, u]), 1)
    assert np.allclose(Au[0], (g.n1 / 2) ** 2 * u, atol=1e-10)


def test_leray_projection(g):
    x1, x2 = _xy(g)
    phi = np.sin(x1) * np.cos(2 * x2) + np.cos(3 * x1 - x2)
    grad_phi = O.fft_grad(g, phi)
    assert np.abs(O.leray(g, grad_phi)).max() < 1e-12
    w = synth.smooth_a_velocity(g.n1, g.n2)
    assert np.abs(O.leray(g, w) - w).max() < 1e-13
    b = np.stack([np.sin(x1 + 2 * x2), np.cos(2 * x1) * np.sin(x2)])
    Kb = O.leray(g, b)
    assert np.abs(O.fft_div(g, Kb)).max() < 1e-12
    assert np.abs(O.leray(g, Kb) - Kb).max() < 1e-13
    # K = I for the compressible case
    assert O.apply_proj(g, b, 0) is b


def test_discrete_l2_inner_product(g):
    one = np.ones(g.shape)
    assert abs(O.inner_l2(g, one, one) - 4 * math.pi ** 2) < 1e-12
    x1, x2 = _xy(g)
    s = np.sin(x1) * np.sin(x2)
    assert abs(O.inner_l2(g, s, s) - math.pi ** 2) < 1e-12
