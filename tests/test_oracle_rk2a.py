"""Pins of the oracle's stabilised RK2 transport (section 3.3.1; appendix "Stabilized RK2 Scheme":
the transport equations in antisymmetric form, pseudospectral in space, Heun's method in time).

- The discrete adjoint operator is exactly minus the transpose of the forward one, so the
  adjoint solve is the transpose of the state solve: the paper's delta_ADJ (table
  t:adjoint-error) is at machine precision for RK2A, while the SL scheme's is not.
- Constant velocity: the exact solution is the shifted template; Heun is second order in time.
- v = 0 closed forms: g(0) = (m_R - m_T) grad m_T and H(0) vt = beta A vt + (vt . grad m_T) grad m_T
  for trigonometric fields whose products the grid resolves; Q(0) exactly symmetric for any field.
- Finite differences of J: the gradient's error decreases at second order in ht.
- The RK2A and SL state solves converge to each other under refinement (the comparison of
  table t:convergence-SL-to-RK2A-transporteqs).
"""

import numpy as np
import pytest

import oracle as O
import synth


def _dense(op, g):
    n = g.N
    M = np.empty((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        M[:, k] = op(e.reshape(g.shape)).ravel()
    return M


def test_adjoint_operator_is_minus_transpose():
    g = O.Grid(6, 8)
    X1, X2 = g.X
    v = np.stack([0.4 * np.sin(X2) + 0.1 * np.cos(2 * X1), 0.3 * np.cos(X1 + X2)])
    divv = O.fft_div(g, v)
    L = _dense(lambda u: O.rk2a_forward_op(g, v, divv, u), g)
    A = _dense(lambda u: O.rk2a_adjoint_op(g, v, divv, u), g)
    assert np.abs(A + L.T).max() < 1e-13 * np.abs(L).max()
    # the b-form integrand is the transpose of the state source: <S(m) vt, lam> = <vt, T(lam, m)>
    rng = np.random.default_rng(0)
    m, lam, vt = rng.standard_normal(g.shape), rng.standard_normal(g.shape), rng.standard_normal((2,) + g.shape)
    lhs = np.sum(O.rk2a_state_source(g, m, vt) * lam)
    rhs = np.sum(vt * O.rk2a_integrand(g, lam, m))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def _delta_adj(g, v, m0, nt, transport):
    """delta_ADJ = |<C m0, C m0> - <C^T C m0, m0>| / |<C m0, C m0>| (section 4.1, adjoint error)."""
    if transport == "rk2a":
        m1 = O.rk2a_solve_state(g, v, m0, nt)[-1]
        lam0 = O.rk2a_solve_adjoint(g, v, m1, nt)[0]
    else:
        ht = 1.0 / nt
        Xf, Xa = O.trace(g, v, ht, -1), O.trace(g, v, ht, +1)
        m1 = O.solve_state(g, Xf, m0, nt)[-1]
        lam0 = O.solve_adjoint(g, Xa, O.adjoint_factor(g, v, Xa, ht), m1, nt)[0]
    a = np.sum(m1 * m1)
    return abs(a - np.sum(lam0 * m0)) / abs(a)


def test_adjoint_error_at_machine_precision():
    """RK2A's adjoint error is rounding (the paper: 1.2e-16 at 256^2); the SL scheme's is not."""
    n = 64
    g = O.Grid(n, n)
    m0 = synth.smooth_a_template(n, n)
    v = synth.smooth_a_velocity(n, n)
    for nt in (4, 16):
        assert _delta_adj(g, v, m0, nt, "rk2a") < 1e-14
    assert _delta_adj(g, v, m0, 4, "sl") > 1e-8


def test_constant_velocity_second_order_in_time():
    n = 32
    g = O.Grid(n, n)
    X1, X2 = g.X
    m0 = np.sin(X1) * np.cos(2 * X2) + 0.5 * np.cos(3 * X1 - X2)
    c = (0.7, -0.4)
    v = np.stack([np.full(g.shape, c[0]), np.full(g.shape, c[1])])
    exact = np.sin(X1 - c[0]) * np.cos(2 * (X2 - c[1])) + 0.5 * np.cos(3 * (X1 - c[0]) - (X2 - c[1]))
    errs = [np.linalg.norm(O.rk2a_solve_state(g, v, m0, nt)[-1] - exact) / np.linalg.norm(exact)
            for nt in (8, 16, 32, 64)]
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 1.9) and np.all(rates < 2.1), (errs, rates)
    # v = 0 is the identity
    assert np.array_equal(O.rk2a_solve_state(g, np.zeros((2,) + g.shape), m0, 4)[-1], m0)


def _trig_level(n, beta, reg, transport="rk2a", nt=4):
    g = O.Grid(n, n)
    X1, X2 = g.X
    mT = 0.5 + 0.2 * np.sin(X1) * np.cos(X2) + 0.1 * np.cos(2 * X2)
    mR = 0.5 + 0.2 * np.sin(X1 + 0.3) * np.cos(X2) + 0.1 * np.cos(2 * X2 - 0.2)
    return O.Level(g, mT, mR, O.Params(nt=nt, beta=beta, reg=reg, transport=transport))


def test_closed_forms_at_zero_velocity():
    L = _trig_level(32, 1e-2, 2)
    g = L.grid
    zero = np.zeros((2,) + g.shape)
    lin = O.linearize(L, zero)
    gm = O.fft_grad(g, L.mT)
    assert np.abs(O.gradient(lin) - (L.mR - L.mT) * gm).max() < 1e-14
    X1, X2 = g.X
    vt = np.stack([0.2 * np.cos(X2), 0.1 * np.sin(X1 - X2)])
    h = O.hessian_matvec(lin, vt)
    ref = L.prm.beta * O.apply_reg(g, vt, 2) + (vt[0] * gm[0] + vt[1] * gm[1]) * gm
    assert np.abs(h - ref).max() < 1e-13 * np.abs(ref).max()
    # Q(0) is exactly symmetric for any pair of directions (S^T S with the b-form as S^T)
    rng = np.random.default_rng(3)
    w1, w2 = rng.standard_normal((2,) + g.shape), rng.standard_normal((2,) + g.shape)
    q1, q2 = O.transport_part(lin, w1), O.transport_part(lin, w2)
    assert abs(np.sum(w2 * q1) - np.sum(w1 * q2)) < 1e-12 * abs(np.sum(w2 * q1))
    assert np.sum(w1 * q1) > 0


def test_gradient_finite_differences_converge_in_time():
    n = 32
    g = O.Grid(n, n)
    rng = np.random.default_rng(4)
    mT = synth.gaussian_sum_isotropic(n, n, rng, count=6)
    v = synth.random_velocity(n, n, rng, modes=6, kmax=2, amplitude=0.3)
    w = synth.random_velocity(n, n, rng, modes=6, kmax=2, amplitude=0.2)
    errs = []
    for nt in (4, 8, 16):
        L = O.Level(g, mT, 0.9 * mT + 0.05, O.Params(nt=nt, beta=1e-3, reg=2, transport="rk2a"))
        gr = O.gradient(O.linearize(L, v))
        d = O.inner_l2(g, gr, w)
        eps = 1e-4
        fd = (O.objective(L, v + eps * w) - O.objective(L, v - eps * w)) / (2 * eps)
        errs.append(abs(fd - d) / abs(d))
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] / errs[2] > 3.0, errs


def test_full_newton_matches_gradient_differences():
    """The full-Newton RK2A matvec against the central difference of the RK2A gradient: the
    discrepancy falls at second order in ht (the Gauss--Newton one does not)."""
    n = 32
    g = O.Grid(n, n)
    rng = np.random.default_rng(6)
    mT = synth.gaussian_sum_isotropic(n, n, rng, count=6)
    mR = synth.gaussian_sum_isotropic(n, n, rng, count=6)
    v = synth.random_velocity(n, n, rng, modes=6, kmax=2, amplitude=0.3)
    vt = synth.random_velocity(n, n, rng, modes=6, kmax=2, amplitude=0.2)
    errs, gn_errs = [], []
    for nt in (4, 8, 16):
        L = O.Level(g, mT, mR, O.Params(nt=nt, beta=1e-3, reg=2, transport="rk2a", hessian="fn"))
        eps = 1e-4
        fd = (O.gradient(O.linearize(L, v + eps * vt)) - O.gradient(O.linearize(L, v - eps * vt))) / (2 * eps)
        h = O.hessian_matvec(O.linearize(L, v), vt)
        errs.append(np.linalg.norm(h - fd) / np.linalg.norm(fd))
        Lg = O.Level(g, mT, mR, O.Params(nt=nt, beta=1e-3, reg=2, transport="rk2a", hessian="gn"))
        gn_errs.append(np.linalg.norm(O.hessian_matvec(O.linearize(Lg, v), vt) - fd) / np.linalg.norm(fd))
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs
    assert gn_errs[-1] > 10 * errs[-1], (errs, gn_errs)


@pytest.mark.slow
def test_sl_and_rk2a_states_converge_to_each_other():
    """The SL and RK2A state solutions of the smooth problem approach each other as the grid and
    the number of time steps grow (table t:convergence-SL-to-RK2A-transporteqs)."""
    diffs = []
    for n, nt in ((32, 8), (64, 16), (128, 32)):
        g = O.Grid(n, n)
        m0 = synth.smooth_a_template(n, n)
        v = synth.smooth_a_velocity(n, n)
        a = O.transport_state(g, v, m0, nt)
        b = O.rk2a_solve_state(g, v, m0, nt)[-1]
        diffs.append(np.linalg.norm(a - b) / np.linalg.norm(b))
    assert diffs[0] > diffs[1] > diffs[2]
    assert diffs[-1] < 1e-4, diffs


def test_newton_solve_with_rk2a_transport():
    """P_REG + RK2A (the paper's earlier solver) reaches the stop rule on the smooth problem."""
    n = 32
    g = O.Grid(n, n)
    mT = synth.smooth_a_template(n, n)
    vstar = synth.smooth_a_velocity(n, n)
    mR = O.rk2a_solve_state(g, vstar, mT, 8)[-1]
    L = O.Level(g, mT, mR, O.Params(nt=8, beta=1e-2, reg=1, transport="rk2a"))
    v, rep = O.newton_solve(L, pc="reg", max_newton=10)
    assert rep["status"] == "ok" and rep["grel"][-1] <= 1e-2
    assert all(np.diff(rep["J"]) < 0)
