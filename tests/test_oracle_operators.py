"""Pins of the oracle's objective, reduced gradient and GN Hessian matvec
(section 3.1: eqs. e:varopt:objective, e:control-elim, e:hessian-matvec; section 3.4.1)."""

import math

import numpy as np
import pytest

import oracle as O
import synth


def _smooth_problem(n=64, nt=4, beta=1e-2, reg=1):
    g = O.Grid(n, n)
    mT = synth.smooth_a_template(n, n)
    vstar = synth.smooth_a_velocity(n, n)
    mR = O.transport_state(g, vstar, mT, nt)
    return O.Level(g, mT, mR, O.Params(nt=nt, beta=beta, reg=reg)), vstar


def _direction(n, seed=11, amp=0.1):
    return synth.random_velocity(n, n, np.random.default_rng(seed), modes=8, kmax=3, amplitude=amp)


def test_objective_closed_forms():
    L, vstar = _smooth_problem()
    g = L.grid
    J0 = O.objective(L, np.zeros((2,) + g.shape))
    assert abs(J0 - 0.5 * g.cell * np.sum((L.mT - L.mR) ** 2)) < 1e-14
    # at v*: zero residual; beta/2 <v*, -Lap v*> = beta/2 * 2 * int |v*|^2 = beta * pi^2 / 2
    Jv = O.objective(L, vstar)
    assert abs(Jv - L.prm.beta * math.pi ** 2 / 2) < 1e-13


def test_gradient_at_zero_closed_form():
    """v = 0: X = x, gamma = 1, m^j = m_T, lambda^j = m_R - m_T, so g(0) = (m_R - m_T) grad m_T."""
    L, _ = _smooth_problem(nt=4, beta=1e-2)
    g = L.grid
    lin = O.linearize(L, np.zeros((2,) + g.shape))
    g0 = O.gradient(lin)
    gm = O.fft_grad(g, L.mT)
    assert np.abs(g0 - (L.mR - L.mT) * gm).max() < 1e-14


def test_gradient_at_zero_residual_point():
    """m_R was made by the same transport with v*, so lambda = 0 and g(v*) = beta A v* = 2 beta v*."""
    L, vstar = _smooth_problem()
    lin = O.linearize(L, vstar)
    assert np.abs(O.gradient(lin) - 2 * L.prm.beta * vstar).max() < 1e-14


def test_hessian_at_zero_closed_form():
    """v = 0: H_GN vt = beta A vt + (vt . grad m_T) grad m_T (Heun and trapezoid exact for constant f)."""
    L, _ = _smooth_problem(nt=4)
    g = L.grid
    lin = O.linearize(L, np.zeros((2,) + g.shape))
    vt = _direction(64)
    gm = O.fft_grad(g, L.mT)
    ref = L.prm.beta * O.apply_reg(g, vt, 1) + (vt[0] * gm[0] + vt[1] * gm[1]) * gm
    assert np.abs(O.hessian_matvec(lin, vt) - ref).max() < 1e-14


def _fd_gradient_error(L, v, w):
    g = L.grid
    lin = O.linearize(L, v)
    an = O.inner_l2(g, O.gradient(lin), w)
    best = np.inf
    for eps in (1e-2, 1e-3, 1e-4):
        fd = (O.objective(L, v + eps * w) - O.objective(L, v - eps * w)) / (2 * eps)
        best = min(best, abs(fd - an) / abs(an))
    return best


def test_gradient_matches_finite_differences_and_converges_in_nt():
    """Optimize-then-discretize: the FD check holds to discretisation error, shrinking with nt."""
    n = 64
    g = O.Grid(n, n)
    mT = synth.smooth_a_template(n, n)
    vstar = synth.smooth_a_velocity(n, n)
    mR = O.transport_state(g, vstar, mT, 16)
    w = _direction(n)
    errs = []
    for nt in (2, 4, 8):
        L = O.Level(g, mT, mR, O.Params(nt=nt, beta=1e-2, reg=1))
        errs.append(_fd_gradient_error(L, 0.5 * vstar, w))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-3


def test_gradient_finite_differences_at_zero_velocity():
    L, _ = _smooth_problem(nt=4)
    err = _fd_gradient_error(L, np.zeros((2,) + L.grid.shape), _direction(64))
    assert err < 1e-4


def test_incremental_state_is_derivative_of_state():
    """m~(1)[w] approximates d m_1 / dv [w]; the gap shrinks with nt."""
    n = 64
    g = O.Grid(n, n)
    mT = synth.smooth_a_template(n, n)
    v = 0.8 * synth.smooth_a_velocity(n, n)
    w = _direction(n)
    errs = []
    for nt in (2, 4, 8):
        L = O.Level(g, mT, mT, O.Params(nt=nt, beta=1e-2, reg=1))
        lin = O.linearize(L, v)
        mt = O.incremental_state(lin, w)[-1]
        eps = 1e-4
        fd = (O.transport_state(g, v + eps * w, mT, nt) - O.transport_state(g, v - eps * w, mT, nt)) / (2 * eps)
        errs.append(np.linalg.norm(mt - fd) / np.linalg.norm(fd))
    assert errs[0] > 2 * errs[1] > 0 and errs[1] > 2 * errs[2] > 0
    assert errs[2] < 1e-2


def test_hessian_matches_fd_of_gradient_at_zero_residual_point():
    """At v* (lambda = 0) GN equals full Newton, so (g(v*+eps w) - g(v*-eps w)) / 2 eps ~ H_GN w."""
    n = 64
    g = O.Grid(n, n)
    mT = synth.smooth_a_template(n, n)
    vstar = synth.smooth_a_velocity(n, n)
    w = _direction(n)
    errs = []
    for nt in (2, 4, 8):
        mR = O.transport_state(g, vstar, mT, nt)
        L = O.Level(g, mT, mR, O.Params(nt=nt, beta=1e-2, reg=1))
        Hw = O.hessian_matvec(O.linearize(L, vstar), w)
        eps = 1e-4
        gp = O.gradient(O.linearize(L, vstar + eps * w))
        gm = O.gradient(O.linearize(L, vstar - eps * w))
        fd = (gp - gm) / (2 * eps)
        errs.append(np.linalg.norm(Hw - fd) / np.linalg.norm(fd))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 2e-2


def test_hessian_symmetry_positivity_and_gn_identity():
    """<w1, H w2> = <H w1, w2>, <w, Q w> >= 0 and <w, Q w> = ||m~_1(w)||^2 hold up to the SL
    scheme's adjoint error, which shrinks as the grid is refined (nt = 16)."""
    sym, gn = [], []
    for n in (32, 64, 128):
        g = O.Grid(n, n)
        mT = synth.smooth_a_template(n, n)
        v = 0.8 * synth.smooth_a_velocity(n, n)
        w1, w2 = _direction(n, 1), _direction(n, 2)
        L = O.Level(g, mT, mT, O.Params(nt=16, beta=1e-2, reg=1))
        lin = O.linearize(L, v)
        a = O.inner_l2(g, w1, O.hessian_matvec(lin, w2))
        b = O.inner_l2(g, O.hessian_matvec(lin, w1), w2)
        sym.append(abs(a - b) / abs(a))
        q = O.inner_l2(g, w1, O.gn_transport_part(lin, w1))
        mt = O.incremental_state(lin, w1)[-1]
        assert q > 0
        gn.append(abs(q - O.inner_l2(g, mt, mt)) / q)
    assert sym[0] > sym[1] > sym[2] and sym[2] < 1e-4
    assert gn[0] > gn[1] > gn[2] and gn[2] < 1e-5
    # exact symmetry at v = 0
    g = O.Grid(64, 64)
    mT = synth.smooth_a_template(64, 64)
    w1, w2 = _direction(64, 1), _direction(64, 2)
    L = O.Level(g, mT, mT, O.Params(nt=4, beta=1e-2, reg=1))
    lin0 = O.linearize(L, np.zeros((2,) + g.shape))
    a = np.sum(w1 * O.hessian_matvec(lin0, w2)); b = np.sum(O.hessian_matvec(lin0, w1) * w2)
    assert abs(a - b) < 1e-13 * abs(a)


def test_hessian_is_linear():
    L, vstar = _smooth_problem()
    lin = O.linearize(L, 0.5 * vstar)
    w1, w2 = _direction(64, 3), _direction(64, 4)
    lhs = O.hessian_matvec(lin, 2 * w1 - 3 * w2)
    rhs = 2 * O.hessian_matvec(lin, w1) - 3 * O.hessian_matvec(lin, w2)
    assert np.abs(lhs - rhs).max() < 1e-13 * np.abs(rhs).max() * 10


def test_leray_gradient_is_divergence_free():
    L, vstar = _smooth_problem()
    L.prm.proj = 1
    lin = O.linearize(L, 0.3 * vstar)
    gr = O.gradient(lin)
    assert np.abs(O.fft_div(L.grid, gr)).max() < 1e-12
    Hw = O.hessian_matvec(lin, O.leray(L.grid, _direction(64)))
    assert np.abs(O.fft_div(L.grid, Hw)).max() < 1e-12


def test_full_newton_hessian_at_zero_closed_form():
    """v = 0, lambda = m_R - m_T constant in time: m~(t) = -t f0 with f0 = vt . grad m_T,
    lam~(t) = f0 + (1 - t) div(lambda vt) (Heun and trapezoid exact for these linear-in-t
    fields), so b~ = int lam~ grad m_T + lambda grad m~ dt
    = (f0 + div(lambda vt) / 2) grad m_T - (lambda / 2) grad f0."""
    n = 64
    g = O.Grid(n, n)
    mT = synth.smooth_a_template(n, n)
    mR = O.transport_state(g, synth.smooth_a_velocity(n, n), mT, 4)
    L = O.Level(g, mT, mR, O.Params(nt=4, beta=1e-2, reg=1, hessian="fn"))
    lin = O.linearize(L, np.zeros((2,) + g.shape))
    vt = _direction(n)
    gm = O.fft_grad(g, mT)
    lam = mR - mT
    f0 = vt[0] * gm[0] + vt[1] * gm[1]
    ref = (f0 + 0.5 * O.fft_div(g, lam * vt)) * gm - 0.5 * lam * O.fft_grad(g, f0)
    ref = L.prm.beta * O.apply_reg(g, vt, 1) + ref
    out = O.hessian_matvec(lin, vt)
    assert np.abs(out - ref).max() < 1e-13 * np.abs(ref).max()


def test_full_newton_hessian_is_derivative_of_gradient_second_order_in_nt():
    """Away from the minimiser (lambda != 0) and for a compressible v (div v != 0), the full-
    Newton matvec matches the central difference of the gradient up to the SL scheme's
    O(ht^2) error (ratio ~4 per doubling of nt), while Gauss--Newton stays O(1) away.  A
    dropped or first-order source term in the incremental adjoint shows as ratio ~2 or O(1)."""
    n = 64
    g = O.Grid(n, n)
    mT = synth.smooth_a_template(n, n)
    vstar = synth.smooth_a_velocity(n, n)
    mR = O.transport_state(g, vstar, mT, 16)
    v = 0.5 * vstar + synth.random_velocity(n, n, np.random.default_rng(5), modes=8, kmax=3, amplitude=0.3)
    w = _direction(n)
    errs = {}
    for hess in ("gn", "fn"):
        errs[hess] = []
        for nt in (2, 4, 8):
            L = O.Level(g, mT, mR, O.Params(nt=nt, beta=1e-2, reg=1, hessian=hess))
            Hw = O.hessian_matvec(O.linearize(L, v), w)
            eps = 1e-4
            fd = (O.gradient(O.linearize(L, v + eps * w)) - O.gradient(O.linearize(L, v - eps * w))) / (2 * eps)
            errs[hess].append(np.linalg.norm(Hw - fd) / np.linalg.norm(fd))
    fn, gn = errs["fn"], errs["gn"]
    assert fn[0] / fn[1] > 3.0 and fn[1] / fn[2] > 3.0, fn
    assert fn[2] < 2e-3, fn
    assert min(gn) > 0.1, gn


def test_full_newton_hessian_symmetric_up_to_discretisation():
    """<w1, H_FN w2> = <H_FN w1, w2> up to the time discretisation of the SL scheme: the gap
    shrinks at second order in ht for a compressible v away from the minimiser."""
    n = 64
    g = O.Grid(n, n)
    mT = synth.smooth_a_template(n, n)
    mR = O.transport_state(g, synth.smooth_a_velocity(n, n), mT, 16)
    v = synth.random_velocity(n, n, np.random.default_rng(5), modes=8, kmax=3, amplitude=0.3)
    w1, w2 = _direction(n, 1), _direction(n, 2)
    sym = []
    for nt in (4, 8, 16):
        L = O.Level(g, mT, mR, O.Params(nt=nt, beta=1e-2, reg=1, hessian="fn"))
        lin = O.linearize(L, v)
        a = O.inner_l2(g, w1, O.hessian_matvec(lin, w2))
        b = O.inner_l2(g, O.hessian_matvec(lin, w1), w2)
        sym.append(abs(a - b) / abs(a))
    assert sym[0] / sym[1] > 3.0 and sym[1] / sym[2] > 3.0 and sym[2] < 2e-3, sym


def test_leray_products_equal_compressible_ones_on_divergence_free_directions():
    """K is self-adjoint and fixes divergence-free fields, so for divergence-free w the directional
    derivatives of the incompressible problem are those of the compressible one:
    <g_K, w> = <g_I, w> and <H_K w1, w2> = <H_I w1, w2> (GN and FN), at a compressible v too."""
    L, vstar = _smooth_problem()
    g = L.grid
    v = 0.3 * vstar + synth.random_velocity(64, 64, np.random.default_rng(5), modes=8, kmax=3, amplitude=0.2)
    w1, w2 = O.leray(g, _direction(64, 1)), O.leray(g, _direction(64, 2))
    for hess in ("gn", "fn"):
        lins = [O.linearize(O.Level(g, L.mT, L.mR, O.Params(nt=4, beta=1e-2, reg=1, proj=p, hessian=hess)), v)
                for p in (0, 1)]
        gI, gK = O.gradient(lins[0]), O.gradient(lins[1])
        assert abs(O.inner_l2(g, gK, w1) - O.inner_l2(g, gI, w1)) < 1e-12 * abs(O.inner_l2(g, gI, w1))
        hI = O.inner_l2(g, O.hessian_matvec(lins[0], w1), w2)
        hK = O.inner_l2(g, O.hessian_matvec(lins[1], w1), w2)
        assert abs(hK - hI) < 1e-12 * abs(hI)
        # K b is divergence-free while b is not (g = beta A v + K b; v itself is compressible here)
        bAv = 1e-2 * O.apply_reg(g, v, 1)
        assert np.abs(O.fft_div(g, gI - bAv)).max() > 1e-3 and np.abs(O.fft_div(g, gK - bAv)).max() < 1e-12


@pytest.mark.parametrize("pc", ["reg", "2l"])
def test_leray_newton_keeps_velocity_divergence_free(pc):
    """The incompressible solve (K = Leray, H1) converges and every iterate stays divergence-free
    (the gradient, the preconditioners and the Hessian map divergence-free fields to themselves)."""
    n = 64
    g = O.Grid(n, n)
    rng = np.random.default_rng(2)
    mT = synth.smooth_a_template(n, n)
    vs = O.leray(g, synth.random_velocity(n, n, rng, modes=16, kmax=3, amplitude=0.3))
    L = O.Level(g, mT, O.transport_state(g, vs, mT, 4), O.Params(nt=4, beta=1e-2, reg=1, proj=1))
    v, rep = O.newton_solve(L, pc=pc, max_newton=10)
    assert rep["status"] == "ok" and rep["grel"][-1] <= 1e-2, rep["grel"]
    assert np.abs(O.fft_div(g, v)).max() < 1e-12 * np.abs(v).max()
    assert all(np.diff(rep["J"]) < 0)
