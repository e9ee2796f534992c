"""Pins of the oracle's Krylov and Newton layers (sections 3.4.1, 3.5; the KKT-solve
experiment of section 4.2.2 with true solution vt* = -0.5 v*)."""

import numpy as np
import pytest

import oracle as O
import synth


def _smooth_level(n=64, nt=4, beta=1e-2, reg=1):
    g = O.Grid(n, n)
    mT = synth.smooth_a_template(n, n)
    vstar = synth.smooth_a_velocity(n, n)
    return O.Level(g, mT, O.transport_state(g, vstar, mT, nt), O.Params(nt=nt, beta=beta, reg=reg)), vstar


def test_pcg_dense_tiny_system():
    """PCG on the GN Hessian of a 6x8 problem equals a dense solve of the assembled matrix."""
    g = O.Grid(6, 8)
    X1, X2 = g.X
    mT = 0.5 + 0.3 * np.sin(X1) * np.cos(X2)
    v = 0.3 * np.stack([np.sin(X2), np.cos(X1)])
    L = O.Level(g, mT, mT, O.Params(nt=2, beta=1e-1, reg=2))
    lin = O.linearize(L, np.zeros((2,) + g.shape))    # v = 0: H is exactly symmetric
    n = 2 * g.N
    H = np.empty((n, n))
    for k in range(n):
        e = np.zeros(n); e[k] = 1.0
        H[:, k] = O.hessian_matvec(lin, e.reshape((2,) + g.shape)).ravel()
    assert np.abs(H - H.T).max() < 1e-12 * np.abs(H).max()
    assert np.linalg.eigvalsh(H).min() > 0
    b = v.ravel()
    x, its, st = O.pcg(lambda s: O.hessian_matvec(lin, s), v,
                       lambda r: O.prec_reg(g, r, 1e-1, 2), 1e-13, 200)
    assert st == "ok"
    assert np.abs(x.ravel() - np.linalg.solve(H, b)).max() < 1e-9 * np.abs(x).max()


def test_pcg_negative_curvature_exit():
    b = np.ones((2, 2, 2))
    x, its, st = O.pcg(lambda s: -s, b, lambda r: r, 1e-8, 10)
    assert st == "negcurv" and its == 1 and np.array_equal(x, b)


@pytest.mark.parametrize("pc", ["reg", "2l"])
def test_kkt_true_solution_recovery(pc):
    """b = H vt*, vt* = -0.5 v*: PCG to 1e-12 recovers vt* (the paper reaches 1e-13 .. 1e-15)."""
    L, vstar = _smooth_level(n=64, nt=4, beta=1e-2, reg=2)
    g, p = L.grid, L.prm
    lin = O.linearize(L, vstar)
    vt_true = -0.5 * vstar
    if pc == "reg":
        b = O.hessian_matvec(lin, vt_true)
        x, its, st = O.pcg(lambda s: O.hessian_matvec(lin, s), b,
                           lambda r: O.prec_reg(g, r, p.beta, p.reg), 1e-12, 500)
    else:
        tl = O.setup_two_level(L)
        cg = tl.coarse.grid
        tl.lin_c = O.linearize(tl.coarse, np.stack([O.restrict(g, cg, vstar[c]) for c in range(2)]))
        # split system: M s = S H vt*, vt = S s
        b = O.split_scale(g, O.hessian_matvec(lin, vt_true), p.beta, p.reg)
        # at v* the CHEB(10) bounds estimated at v = 0 leave P_2L slightly indefinite on the last
        # residuals (r.z < 0 near 1e-8): the solve re-estimates e_max there and runs again
        s, its, st = O.pcg_reestimating(lambda s: O.split_matvec(lin, s), b, lambda r: O.apply_two_level(L, tl, r),
                                        1e-12, 500, lambda: setattr(tl, "emax", O.reestimate_emax(tl)))
        x = O.split_scale(g, s, p.beta, p.reg)
    assert st == "ok"
    assert np.linalg.norm(x - vt_true) / np.linalg.norm(vt_true) < 1e-10


@pytest.mark.parametrize("pc", ["reg", "2l"])
def test_newton_converges_on_smooth_problem(pc):
    L, vstar = _smooth_level(n=64, nt=4, beta=1e-2, reg=1)
    v, rep = O.newton_solve(L, pc=pc, max_newton=10)
    assert rep["status"] == "ok"
    assert rep["grel"][-1] <= 1e-2 and rep["newton_iters"] <= 10
    assert all(np.diff(rep["J"]) < 0)
    # the mismatch shrinks (beta = 1e-2 keeps the minimiser away from a perfect match)
    m1 = O.transport_state(L.grid, v, L.mT, 4)
    assert np.linalg.norm(m1 - L.mR) < 0.3 * np.linalg.norm(L.mT - L.mR)


def test_both_preconditioners_reach_the_same_minimiser():
    L, _ = _smooth_level(n=64, nt=4, beta=1e-2, reg=1)
    v1, r1 = O.newton_solve(L, pc="reg", gtol_rel=1e-3, max_newton=20)
    v2, r2 = O.newton_solve(L, pc="2l", gtol_rel=1e-3, max_newton=20)
    assert r1["grel"][-1] <= 1e-3 and r2["grel"][-1] <= 1e-3
    assert abs(r1["J"][-1] - r2["J"][-1]) < 1e-6 * r1["J"][-1]
    assert np.linalg.norm(v1 - v2) < 1e-2 * np.linalg.norm(v1)


def test_two_level_needs_fewer_pcg_iterations_at_small_beta():
    """At beta = 1e-3 (H2) P_2L takes fewer PCG steps than P_REG for the same KKT system."""
    n = 64
    g = O.Grid(n, n)
    rng = np.random.default_rng(2)
    mT = synth.gaussian_sum_isotropic(n, n, rng)
    vgen = synth.random_velocity(n, n, rng, modes=16, kmax=4, amplitude=0.3)
    L = O.Level(g, mT, O.transport_state(g, vgen, mT, 4), O.Params(nt=4, beta=1e-3, reg=2))
    lin = O.linearize(L, np.zeros((2,) + g.shape))
    grad = O.gradient(lin)
    p = L.prm
    _, it_reg, st1 = O.pcg(lambda s: O.hessian_matvec(lin, s), -grad,
                           lambda r: O.prec_reg(g, r, p.beta, p.reg), 1e-6, 500)
    tl = O.setup_two_level(L)
    tl.lin_c = O.linearize(tl.coarse, np.zeros((2,) + tl.coarse.grid.shape))
    _, it_2l, st2 = O.pcg(lambda s: O.split_matvec(lin, s), -O.split_scale(g, grad, p.beta, p.reg),
                          lambda r: O.apply_two_level(L, tl, r), 1e-6, 500)
    assert st1 == "ok" and st2 == "ok"
    assert it_2l < it_reg


@pytest.mark.parametrize("pc", ["reg", "2l"])
def test_full_newton_converges_superlinearly(pc):
    """With the full-Newton matvec the last Newton step contracts the gradient by more than
    two orders of magnitude (quadratic convergence near the minimiser), reaching
    ||g||rel <= 1e-5 within five iterations, where Gauss--Newton contracts linearly."""
    from dataclasses import replace
    L, _ = _smooth_level(n=64, nt=4, beta=1e-2, reg=1)
    Lfn = O.Level(L.grid, L.mT, L.mR, replace(L.prm, hessian="fn"))
    _, rep = O.newton_solve(Lfn, pc=pc, gtol_rel=1e-5, max_newton=8)
    assert rep["status"] == "ok" and rep["grel"][-1] <= 1e-5 and rep["newton_iters"] <= 5, rep["grel"]
    assert rep["grel"][-1] < 1e-2 * rep["grel"][-2]
    assert all(np.diff(rep["J"]) < 0)


def test_nested_pcg_coarse_solve_equals_dense_inverse():
    """PCG(eps) with a tiny tolerance applies (I - L) r + Pro M_c^{-1} Res r, M_c assembled densely
    from the coarse split operator on a 32^2 / 16^2 problem and inverted by numpy."""
    n = 32
    g = O.Grid(n, n)
    rng = np.random.default_rng(3)
    mT = synth.gaussian_sum_isotropic(n, n, rng, count=8, sigma=(0.3, 0.6))
    vgen = synth.random_velocity(n, n, rng, modes=8, kmax=3, amplitude=0.2)
    L = O.Level(g, mT, O.transport_state(g, vgen, mT, 4), O.Params(nt=4, beta=1e-2, reg=2))
    tl = O.setup_two_level(L, solver="pcg", eps=1e-13)
    cg = tl.coarse.grid
    tl.lin_c = O.linearize(tl.coarse, np.stack([O.restrict(g, cg, 0.5 * vgen[c]) for c in range(2)]))
    m = 2 * cg.N
    M = np.empty((m, m))
    for k in range(m):
        e = np.zeros(m); e[k] = 1.0
        M[:, k] = O.split_matvec(tl.lin_c, e.reshape((2,) + cg.shape)).ravel()
    r = synth.random_velocity(n, n, np.random.default_rng(9), modes=16, kmax=8, amplitude=1.0)
    z, its = O.apply_two_level(L, tl, r)
    rc = np.stack([O.restrict(g, cg, r[c]) for c in range(2)])
    zc = np.linalg.solve(M, rc.ravel()).reshape((2,) + cg.shape)
    ref = r - O.lowpass(g, r) + np.stack([O.prolong(g, cg, zc[c]) for c in range(2)])
    assert its > 1 and np.abs(z - ref).max() < 1e-10 * np.abs(ref).max()


def test_nested_pcg_preconditioner_is_nearly_ideal_at_small_beta():
    """Section 4.2.2: with PCG(1e-1) inverting the coarse operator, the outer PCG at beta = 1e-3
    needs no more iterations than with CHEB(10), and far fewer than P_REG."""
    n = 64
    g = O.Grid(n, n)
    rng = np.random.default_rng(2)
    mT = synth.gaussian_sum_isotropic(n, n, rng)
    vgen = synth.random_velocity(n, n, rng, modes=16, kmax=4, amplitude=0.3)
    L = O.Level(g, mT, O.transport_state(g, vgen, mT, 4), O.Params(nt=4, beta=1e-3, reg=2))
    lin = O.linearize(L, np.zeros((2,) + g.shape))
    grad = O.gradient(lin)
    p = L.prm
    rhs = -O.split_scale(g, grad, p.beta, p.reg)
    its = {}
    for solver in ("cheb", "pcg"):
        tl = O.setup_two_level(L, solver=solver, eps=0.1)
        tl.lin_c = O.linearize(tl.coarse, np.zeros((2,) + tl.coarse.grid.shape))
        prec = (lambda r: O.apply_two_level(L, tl, r, 1e-6)[0]) if solver == "pcg" else \
            (lambda r: O.apply_two_level(L, tl, r))
        _, its[solver], st = O.pcg(lambda s: O.split_matvec(lin, s), rhs, prec, 1e-6, 500)
        assert st == "ok"
    _, it_reg, _ = O.pcg(lambda s: O.hessian_matvec(lin, s), -grad, lambda r: O.prec_reg(g, r, p.beta, p.reg),
                         1e-6, 500)
    assert its["pcg"] <= its["cheb"] < it_reg, (its, it_reg)


def test_newton_with_nested_pcg_coarse_solve_converges():
    L, _ = _smooth_level(n=64, nt=4, beta=1e-2, reg=1)
    v, rep = O.newton_solve(L, pc="2l", max_newton=10, coarse_solver="pcg", coarse_eps=0.1)
    assert rep["status"] == "ok" and rep["grel"][-1] <= 1e-2
    v2, rep2 = O.newton_solve(L, pc="2l", max_newton=10)
    assert rep["pcg_iters"] <= rep2["pcg_iters"]
    assert np.linalg.norm(v - v2) < 2e-2 * np.linalg.norm(v2)


def test_newton_limit_is_reported():
    """A solve that the Newton limit ends before the stop test holds reports 'maxit' (section
    3.4.1 stops on the gradient; the limit is a safeguard, not convergence)."""
    L, _ = _smooth_level(n=32, nt=4, beta=1e-2, reg=1)
    _, full = O.newton_solve(L, pc="reg", max_newton=10, gtol_rel=1e-3)
    assert full["status"] == "ok" and full["newton_iters"] >= 2 and full["grel"][-1] <= 1e-3
    _, cut = O.newton_solve(L, pc="reg", max_newton=1, gtol_rel=1e-3)
    assert cut["status"] == "maxit" and cut["newton_iters"] == 1 and cut["grel"][-1] > 1e-3
    assert cut["grel"] == full["grel"][:2]


def test_pcg_reports_an_indefinite_preconditioner():
    """PCG on an SPD operator with a preconditioner that has a negative eigenvalue: the first step
    with r.z <= 0 ends the solve with status 'indefprec'; a positive definite one converges."""
    d = np.linspace(1.0, 4.0, 2 * 3 * 3).reshape(2, 3, 3)
    b = np.ones_like(d)
    pinv = 1.0 / d
    bad = pinv.copy()
    bad[0, 0, 0] = -50.0        # r.z = sum r^2 / d with one large negative weight: negative at once
    _, its, st = O.pcg(lambda s: d * s, b, lambda r: bad * r, 1e-12, 50)
    assert st == "indefprec" and its == 1
    x, _, st = O.pcg(lambda s: d * s, b, lambda r: pinv * r, 1e-12, 50)
    assert st == "ok" and np.abs(d * x - b).max() < 1e-10


def test_underestimated_emax_is_reestimated():
    """An e_max far below the coarse operator's spectrum makes CHEB(10) an indefinite preconditioner
    (its residual polynomial exceeds one above e_max); the solve detects it, re-estimates e_max by
    Lanczos at the current coarse linearisation (section 4.2.1) and still converges."""
    n = 64
    g = O.Grid(n, n)
    rng = np.random.default_rng(21)
    mT = synth.gaussian_sum_isotropic(n, n, rng)
    vgen = synth.random_velocity(n, n, rng, modes=16, kmax=4, amplitude=0.3)
    L = O.Level(g, mT, O.transport_state(g, vgen, mT, 4), O.Params(nt=4, beta=1e-3, reg=2))
    _, ref = O.newton_solve(L, pc="2l", max_newton=10)
    assert ref["cheb_reestimates"] == 0 and ref["status"] == "ok"
    low = 1.0 + 0.05 * (ref["emax"] - 1.0)
    _, rep = O.newton_solve(L, pc="2l", max_newton=10, emax=low)
    assert rep["emax"] == low
    assert rep["cheb_reestimates"] >= 1
    assert rep["status"] == "ok" and rep["grel"][-1] <= 1e-2
