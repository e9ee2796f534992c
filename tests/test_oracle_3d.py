"""Pins of the oracle in three dimensions (d = 3; section 1, "Limitations and Unresolved Issues":
nothing in the method is specific to d = 2).

Independent anchors: closed forms of the spectral operators on plane waves; scipy's periodic
cubic spline along each axis (the tensor-product spline of a separable field is the product of
the 1-D splines); exact integer-cell shifts under a constant velocity; the already pinned 2-D
oracle, which a 3-D problem that does not vary along one axis (and has no velocity along it)
must reproduce along each of the three axes; equivariance under permutations of the axes;
finite differences of the objective.
"""
import math

import numpy as np
import pytest
from scipy.interpolate import CubicSpline

import synth
from oracle import slnk_oracle as O


def _grid():
    return O.Grid(8, 12, 16)


def test_grid_is_three_dimensional():
    g = _grid()
    assert g.d == 3 and g.shape == (8, 12, 16) and g.N == 8 * 12 * 16
    assert abs(g.cell - (2 * math.pi) ** 3 / g.N) < 1e-15
    assert g.X.shape == (3, 8, 12, 16)
    assert g.coarse().shape == (4, 6, 8)
    with pytest.raises(ValueError):
        O.Grid(8, 12, 15)


def test_spectral_operators_on_plane_waves():
    g = _grid()
    X1, X2, X3 = g.X
    k = (1, 2, 3)
    ph = k[0] * X1 + k[1] * X2 + k[2] * X3
    u = np.sin(ph)
    gu = O.fft_grad(g, u)
    for i in range(3):
        assert np.abs(gu[i] - k[i] * np.cos(ph)).max() < 1e-12
    v = np.stack([np.sin(ph), 2 * np.cos(ph), -np.sin(2 * X3)])
    div = k[0] * np.cos(ph) - 2 * k[1] * np.sin(ph) - 2 * np.cos(2 * X3)
    assert np.abs(O.fft_div(g, v) - div).max() < 1e-12
    kk = k[0] ** 2 + k[1] ** 2 + k[2] ** 2
    for reg in (1, 2, 3):
        Au = O.apply_reg(g, np.stack([u, u, u]), reg)
        assert np.abs(Au[2] - kk ** reg * u).max() < 1e-9 * kk ** reg
    # Nyquist of an odd-order symbol is dropped along every axis; the regulariser keeps it
    for i, n in enumerate(g.n):
        w = np.cos(n / 2 * g.X[i])
        assert np.abs(O.fft_grad(g, w)).max() < 1e-12
        assert np.abs(O.apply_reg(g, np.stack([w] * 3), 1)[0] - (n / 2) ** 2 * w).max() < 1e-9


def test_leray_projection_in_three_dimensions():
    g = _grid()
    X1, X2, X3 = g.X
    phi = np.sin(X1 + 2 * X2) * np.cos(X3)
    grad_phi = O.fft_grad(g, phi)
    assert np.abs(O.leray(g, grad_phi)).max() < 1e-12
    # curl of a smooth potential: divergence free, left unchanged
    a = np.stack([np.sin(X2 + X3), np.cos(X1 - X3), np.sin(2 * X1 + X2)])
    ga = [O.fft_grad(g, a[c]) for c in range(3)]
    curl = np.stack([ga[2][1] - ga[1][2], ga[0][2] - ga[2][0], ga[1][0] - ga[0][1]])
    assert np.abs(O.fft_div(g, curl)).max() < 1e-12
    assert np.abs(O.leray(g, curl) - curl).max() < 1e-12
    rng = np.random.default_rng(0)
    b = rng.standard_normal((3,) + g.shape)
    kb = O.leray(g, b)
    assert np.abs(O.fft_div(g, kb)).max() < 1e-10
    assert np.abs(O.leray(g, kb) - kb).max() < 1e-12


def test_tensor_spline_matches_scipy_along_each_axis():
    g = _grid()
    rng = np.random.default_rng(1)
    f1, f2, f3 = (rng.standard_normal(n) for n in g.n)
    f = f1[:, None, None] * f2[None, :, None] * f3[None, None, :]
    pts = rng.uniform(-1.0, 2 * math.pi + 1.0, size=(3, 40))
    got = O.interpolate(g, f, pts)
    ref = np.ones(40)
    for i, fi in enumerate((f1, f2, f3)):
        x = np.arange(g.n[i] + 1) * g.h[i]
        cs = CubicSpline(x, np.append(fi, fi[0]), bc_type="periodic")
        ref = ref * cs(np.mod(pts[i], 2 * math.pi))
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    # nodes are reproduced
    assert np.abs(O.interpolate(g, f, g.X) - f).max() < 1e-12


def test_integer_cell_shift_is_exact():
    g = _grid()
    nt = 3
    c = (1, -2, 3)  # cells moved per time step along each axis
    v = np.stack([np.full(g.shape, c[i] * nt * g.h[i]) for i in range(3)])
    rng = np.random.default_rng(2)
    m0 = rng.standard_normal(g.shape)
    m1 = O.transport_state(g, v, m0, nt)
    ref = np.roll(m0, shift=tuple(nt * ci for ci in c), axis=(0, 1, 2))
    assert np.abs(m1 - ref).max() < 1e-12


def _problem3(g, seed=3, nt=4, reg=2, proj=0, beta=1e-2):
    rng = np.random.default_rng(seed)
    mT = synth.gaussian_sum_3d(*g.n, rng, count=6, sigma=(0.5, 0.9))
    v = synth.random_velocity_3d(*g.n, rng, modes=6, kmax=2, amplitude=0.4)
    mR = O.transport_state(g, v, mT, nt)
    return O.Level(g, mT, mR, O.Params(nt=nt, beta=beta, reg=reg, proj=proj)), v


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("reg,proj", [(2, 0), (3, 1)])
def test_reduces_to_the_two_dimensional_oracle(axis, reg, proj):
    """A problem constant along 'axis' with no velocity along it: objective, gradient, GN matvec,
    P_REG and the split operator equal the 2-D oracle's on the other two axes."""
    g3 = _grid()
    keep = [i for i in range(3) if i != axis]
    g2 = O.Grid(*(g3.n[i] for i in keep))
    rng = np.random.default_rng(4 + axis)
    mT2 = synth.gaussian_sum_isotropic(*g2.n, rng, count=5, sigma=(0.5, 0.9))
    v2 = synth.random_velocity(*g2.n, rng, modes=6, kmax=2, amplitude=0.5)
    vt2 = synth.random_velocity(*g2.n, rng, modes=6, kmax=3, amplitude=0.2)
    prm = O.Params(nt=4, beta=1e-2, reg=reg, proj=proj)
    mR2 = O.transport_state(g2, v2, mT2, 4)
    L2 = O.Level(g2, mT2, 0.8 * mR2 + 0.1, prm)

    def lift_scalar(u):
        return np.repeat(np.expand_dims(u, axis), g3.n[axis], axis=axis)

    def lift_vector(w):
        out = np.zeros((3,) + g3.shape)
        for j, i in enumerate(keep):
            out[i] = lift_scalar(w[j])
        return out

    def drop_vector(w):
        sl = [slice(None)] * 3
        sl[axis] = 0
        return np.stack([w[i][tuple(sl)] for i in keep]), w[axis]

    L3 = O.Level(g3, lift_scalar(L2.mT), lift_scalar(L2.mR), prm)
    lin2, lin3 = O.linearize(L2, 0.7 * v2), O.linearize(L3, lift_vector(0.7 * v2))
    assert abs(lin3.J - g3.n[axis] * g3.h[axis] * lin2.J) < 1e-12 * abs(lin3.J)
    for name, a3, a2 in (
            ("gradient", O.gradient(lin3), O.gradient(lin2)),
            ("matvec", O.hessian_matvec(lin3, lift_vector(vt2)), O.hessian_matvec(lin2, vt2)),
            ("prec_reg", O.prec_reg(g3, lift_vector(vt2), 1e-2, reg), O.prec_reg(g2, vt2, 1e-2, reg)),
            ("split", O.split_matvec(lin3, lift_vector(vt2)), O.split_matvec(lin2, vt2))):
        red, along = drop_vector(a3)
        scale = np.abs(a2).max()
        assert np.abs(red - a2).max() < 1e-11 * scale, name
        assert np.abs(along).max() < 1e-11 * scale, name
        # constant along the axis
        assert np.abs(a3 - np.take(a3, [0], axis=axis + 1)).max() < 1e-11 * scale, name


def test_axis_permutation_equivariance():
    """Relabelling the axes of a genuinely three-dimensional problem relabels the results."""
    g = O.Grid(8, 12, 16)
    L, v = _problem3(g)
    perm = (2, 0, 1)
    gp = O.Grid(*(g.n[i] for i in perm))

    def ps(u):
        return np.transpose(u, perm)

    def pv(w):
        return np.stack([ps(w[i]) for i in perm])

    Lp = O.Level(gp, ps(L.mT), ps(L.mR), L.prm)
    rng = np.random.default_rng(6)
    vt = synth.random_velocity_3d(*g.n, rng, modes=5, kmax=2, amplitude=0.2)
    lin, linp = O.linearize(L, 0.6 * v), O.linearize(Lp, pv(0.6 * v))
    assert abs(lin.J - linp.J) < 1e-13 * abs(lin.J)
    for a, b in ((O.gradient(lin), O.gradient(linp)),
                 (O.hessian_matvec(lin, vt), O.hessian_matvec(linp, pv(vt)))):
        assert np.abs(pv(a) - b).max() < 1e-12 * np.abs(a).max()


def test_closed_forms_at_zero_velocity():
    """v = 0: lambda is constant in time, so g = beta A 0 + (m_R - m_T) grad m_T, and the GN matvec
    is beta A vt + (vt . grad m_T) grad m_T."""
    g = O.Grid(8, 12, 16)
    L, _ = _problem3(g)
    lin = O.linearize(L, np.zeros((3,) + g.shape))
    gm = O.fft_grad(g, L.mT)
    assert np.abs(O.gradient(lin) - (L.mR - L.mT) * gm).max() < 1e-14
    rng = np.random.default_rng(7)
    vt = synth.random_velocity_3d(*g.n, rng, modes=5, kmax=2, amplitude=0.2)
    ref = L.prm.beta * O.apply_reg(g, vt, 2) + (vt[0] * gm[0] + vt[1] * gm[1] + vt[2] * gm[2]) * gm
    assert np.abs(O.hessian_matvec(lin, vt) - ref).max() < 1e-13 * np.abs(ref).max()


def test_gradient_finite_differences_converge_in_time():
    """<g, w> against the central difference of J along w, RK2A transport in 3-D: the mismatch
    falls with nt (the discrete gradient is consistent with the objective's derivative)."""
    n = 12
    g = O.Grid(n, n, n)
    rng = np.random.default_rng(8)
    mT = synth.gaussian_sum_3d(n, n, n, rng, count=4, sigma=(0.6, 1.0))
    v = synth.random_velocity_3d(n, n, n, rng, modes=5, kmax=2, amplitude=0.3)
    w = synth.random_velocity_3d(n, n, n, rng, modes=5, kmax=2, amplitude=0.2)
    errs = []
    for nt in (4, 8, 16):
        L = O.Level(g, mT, 0.9 * mT + 0.05, O.Params(nt=nt, beta=1e-3, reg=2, transport="rk2a"))
        d = O.inner_l2(g, O.gradient(O.linearize(L, v)), w)
        eps = 1e-4
        fd = (O.objective(L, v + eps * w) - O.objective(L, v - eps * w)) / (2 * eps)
        errs.append(abs(fd - d) / abs(d))
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[1] / errs[2] > 3.0, errs


def test_sl_gradient_agrees_with_finite_differences():
    """SL in 3-D: <g, w> against the central difference of J, within the discretisation error
    of the optimise-then-discretise gradient, which shrinks as nt grows."""
    n = 12
    g = O.Grid(n, n, n)
    rng = np.random.default_rng(9)
    mT = synth.gaussian_sum_3d(n, n, n, rng, count=4, sigma=(0.6, 1.0))
    v = synth.random_velocity_3d(n, n, n, rng, modes=5, kmax=2, amplitude=0.3)
    w = synth.random_velocity_3d(n, n, n, rng, modes=5, kmax=2, amplitude=0.2)
    errs = []
    for nt in (4, 16):
        L = O.Level(g, mT, 0.9 * mT + 0.05, O.Params(nt=nt, beta=1e-3, reg=2))
        d = O.inner_l2(g, O.gradient(O.linearize(L, v)), w)
        eps = 1e-4
        fd = (O.objective(L, v + eps * w) - O.objective(L, v - eps * w)) / (2 * eps)
        errs.append(abs(fd - d) / abs(d))
    assert errs[1] < 0.05 and errs[1] < errs[0], errs


@pytest.mark.parametrize("pc", ["reg", "2l"])
def test_newton_solve_in_three_dimensions(pc):
    g = O.Grid(16, 16, 16)
    L, v = _problem3(g, beta=1e-3)
    vs, rep = O.newton_solve(L, pc=pc, max_newton=6)
    assert rep["status"] == "ok" and rep["grel"][-1] <= 1e-2, rep
    assert rep["J"][-1] < 0.2 * rep["J"][0]


@pytest.mark.parametrize("axis", [0, 2])
def test_full_newton_reduces_to_the_two_dimensional_oracle(axis):
    """The full-Newton matvec of a problem constant along 'axis' with no velocity along it equals
    the (pinned) 2-D full-Newton matvec on the other two axes, with lambda != 0 and div v != 0."""
    g3 = _grid()
    keep = [i for i in range(3) if i != axis]
    g2 = O.Grid(*(g3.n[i] for i in keep))
    rng = np.random.default_rng(14 + axis)
    mT2 = synth.gaussian_sum_isotropic(*g2.n, rng, count=5, sigma=(0.5, 0.9))
    v2 = synth.random_velocity(*g2.n, rng, modes=6, kmax=2, amplitude=0.5)
    vt2 = synth.random_velocity(*g2.n, rng, modes=6, kmax=3, amplitude=0.2)
    prm = O.Params(nt=4, beta=1e-2, reg=2, hessian="fn")
    mR2 = 0.8 * O.transport_state(g2, v2, mT2, 4) + 0.1
    L2 = O.Level(g2, mT2, mR2, prm)

    def lift_scalar(u):
        return np.repeat(np.expand_dims(u, axis), g3.n[axis], axis=axis)

    def lift_vector(w):
        out = np.zeros((3,) + g3.shape)
        for j, i in enumerate(keep):
            out[i] = lift_scalar(w[j])
        return out

    L3 = O.Level(g3, lift_scalar(mT2), lift_scalar(mR2), prm)
    a2 = O.hessian_matvec(O.linearize(L2, 0.7 * v2), vt2)
    a3 = O.hessian_matvec(O.linearize(L3, lift_vector(0.7 * v2)), lift_vector(vt2))
    sl = [slice(None)] * 3
    sl[axis] = 0
    red = np.stack([a3[i][tuple(sl)] for i in keep])
    scale = np.abs(a2).max()
    assert np.abs(red - a2).max() < 1e-11 * scale
    assert np.abs(a3[axis]).max() < 1e-11 * scale
    L2gn = O.Level(g2, mT2, mR2, O.Params(nt=4, beta=1e-2, reg=2))
    assert np.abs(O.hessian_matvec(O.linearize(L2gn, 0.7 * v2), vt2) - a2).max() > 1e-3 * scale


def test_full_newton_matvec_is_derivative_of_gradient_in_three_dimensions():
    """SL in 3-D, away from the minimiser and with div v != 0: the full-Newton matvec matches the
    central difference of the gradient up to the scheme's time error, which falls at about second
    order in ht (band-limited images, so that the spatial error stays below it); Gauss--Newton stays
    O(1e-1) away.  A dropped or first-order source term in the incremental adjoint would stall the
    convergence."""
    n = 24
    g = O.Grid(n, n, n)
    X1, X2, X3 = g.X
    mT = 0.5 + 0.2 * np.sin(X1) * np.cos(X2) * np.sin(X3) + 0.1 * np.cos(X2 + X3)
    mR = 0.5 + 0.2 * np.sin(X1 + 0.3) * np.cos(X2) * np.sin(X3 - 0.2) + 0.1 * np.cos(X2 + X3 - 0.1)
    rng = np.random.default_rng(11)
    v = synth.random_velocity_3d(n, n, n, rng, modes=5, kmax=1, amplitude=0.3)
    w = synth.random_velocity_3d(n, n, n, rng, modes=5, kmax=1, amplitude=0.2)
    assert np.abs(O.fft_div(g, v)).max() > 0.1

    def fd_error(nt, hess):
        L = O.Level(g, mT, mR, O.Params(nt=nt, beta=1e-3, reg=2, hessian=hess))
        Hw = O.hessian_matvec(O.linearize(L, v), w)
        eps = 1e-4
        fd = (O.gradient(O.linearize(L, v + eps * w)) - O.gradient(O.linearize(L, v - eps * w))) / (2 * eps)
        return np.linalg.norm(Hw - fd) / np.linalg.norm(fd)

    fn = [fd_error(nt, "fn") for nt in (2, 4, 8)]
    gn = fd_error(8, "gn")
    assert fn[0] / fn[1] > 3.0 and fn[1] / fn[2] > 2.5 and fn[2] < 5e-4, fn
    assert gn > 100 * fn[2], (fn, gn)


def test_rk2a_adjoint_error_at_machine_precision_in_three_dimensions():
    """RK2A in 3-D: the discrete adjoint solve is the transpose of the state solve (the adjoint
    error of the paper's section 4.1 at rounding), A = -L^T on a dense operator of a small grid,
    and the b-form integrand is the transpose of the state source; the SL scheme's adjoint error
    is not at rounding."""
    g = O.Grid(4, 6, 8)
    X1, X2, X3 = g.X
    v = np.stack([0.4 * np.sin(X2) + 0.1 * np.cos(2 * X3), 0.3 * np.cos(X1 + X3), 0.2 * np.sin(X1 - X2)])
    divv = O.fft_div(g, v)
    n = g.N
    L = np.empty((n, n))
    A = np.empty((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        L[:, k] = O.rk2a_forward_op(g, v, divv, e.reshape(g.shape)).ravel()
        A[:, k] = O.rk2a_adjoint_op(g, v, divv, e.reshape(g.shape)).ravel()
    assert np.abs(A + L.T).max() < 1e-13 * np.abs(L).max()
    rng = np.random.default_rng(0)
    m, lam, vt = rng.standard_normal(g.shape), rng.standard_normal(g.shape), rng.standard_normal((3,) + g.shape)
    lhs = np.sum(O.rk2a_state_source(g, m, vt) * lam)
    assert abs(lhs - np.sum(vt * O.rk2a_integrand(g, lam, m))) < 1e-12 * abs(lhs)
    g = O.Grid(16, 16, 16)
    X1, X2, X3 = g.X
    m0 = 0.5 + 0.2 * np.sin(X1) * np.cos(X2) * np.sin(X3)
    v = np.stack([0.5 * np.sin(X2), 0.4 * np.cos(X3), 0.3 * np.sin(X1 + X2)])
    for nt in (4, 8):
        m1 = O.rk2a_solve_state(g, v, m0, nt)[-1]
        lam0 = O.rk2a_solve_adjoint(g, v, m1, nt)[0]
        a = np.sum(m1 * m1)
        assert abs(a - np.sum(lam0 * m0)) / a < 1e-14
    ht = 1.0 / 4
    Xf, Xa = O.trace(g, v, ht, -1), O.trace(g, v, ht, +1)
    m1 = O.solve_state(g, Xf, m0, 4)[-1]
    lam0 = O.solve_adjoint(g, Xa, O.adjoint_factor(g, v, Xa, ht), m1, 4)[0]
    assert abs(np.sum(m1 * m1) - np.sum(lam0 * m0)) / np.sum(m1 * m1) > 1e-9
