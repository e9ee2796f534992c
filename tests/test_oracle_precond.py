"""Pins of the oracle's preconditioners (section 3.4.2: P_REG, eq. e:reg-precond; the nested
two-level preconditioner with spectral restriction/prolongation, cut-off filters, CHEB(k)
and the Lanczos estimate of e_max; section 4.2.1)."""

import os

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

import oracle as O
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand(g, seed):
    return np.random.default_rng(seed).standard_normal((2,) + g.shape)


@pytest.mark.parametrize("reg", [1, 2, 3])
def test_prec_reg_inverts_beta_a(reg):
    g = O.Grid(32, 24)
    beta = 3e-3
    r = _rand(g, 0)
    r = r - r.mean(axis=(1, 2), keepdims=True)          # no constant mode (A kills it)
    z = O.prec_reg(g, beta * O.apply_reg(g, r, reg), beta, reg)
    cond = float(O.reg_symbol(g, reg).max())          # rounding is amplified by the symbol's range
    assert np.abs(z - r).max() < 1e-15 * cond * np.abs(r).max()
    # constant mode: zero symbol replaced by one, so P_REG^{-1} c = c / beta
    c = np.ones((2,) + g.shape)
    assert np.abs(O.prec_reg(g, c, beta, reg) - c / beta).max() < 1e-9
    # the split half step squares to P_REG^{-1}
    s2 = O.split_scale(g, O.split_scale(g, r, beta, reg), beta, reg)
    assert np.abs(s2 - O.prec_reg(g, r, beta, reg)).max() < 1e-9 * np.abs(s2).max()


def test_restriction_prolongation():
    fg = O.Grid(32, 48)
    cg = fg.coarse()
    # trigonometric polynomials resolved on the coarse grid keep their values
    f = lambda X: np.sin(3 * X[0]) * np.cos(5 * X[1]) + 0.2 * np.cos(X[0] - 7 * X[1])
    assert np.abs(O.restrict(fg, cg, f(fg.X)) - f(cg.X)).max() < 1e-13
    assert np.abs(O.prolong(fg, cg, f(cg.X)) - f(fg.X)).max() < 1e-13
    # Res o Pro = I on coarse fields without a coarse Nyquist component
    rng = np.random.default_rng(1)
    uc = O.lowpass(cg, np.stack([rng.standard_normal(cg.shape)] * 2))[0]
    uc = uc + 0.0
    u = O.restrict(fg, cg, O.prolong(fg, cg, uc))
    uc_nn = O.restrict(fg, cg, O.prolong(fg, cg, O.restrict(fg, cg, O.prolong(fg, cg, uc))))
    assert np.abs(u - uc_nn).max() < 1e-13
    # modes above the cut-off are removed by restriction
    hi = np.cos(cg.n1 // 2 * fg.X[0]) + np.sin((cg.n2 // 2 + 3) * fg.X[1])
    assert np.abs(O.restrict(fg, cg, hi)).max() < 1e-13


def test_filters_split_identity():
    g = O.Grid(32, 32)
    r = _rand(g, 2)
    lo = O.lowpass(g, r)
    assert np.abs(O.lowpass(g, lo) - lo).max() < 1e-13
    hi = r - lo
    assert np.abs(O.lowpass(g, hi)).max() < 1e-13
    # the low-pass keeps exactly the modes the coarse grid keeps
    cg = g.coarse()
    assert np.abs(O.prolong(g, cg, O.restrict(g, cg, r[0])) - lo[0]).max() < 1e-13


def test_chebyshev_residual_polynomial_diagonal_operator():
    """With op = diag(d), CHEB_k leaves the residual T_k((theta - d)/delta) / T_k(theta/delta) * b."""
    rng = np.random.default_rng(3)
    d = rng.uniform(1.0, 40.0, size=(2, 8, 8))
    b = rng.standard_normal((2, 8, 8))
    emin, emax = 0.9, 42.0
    theta, delta = 0.5 * (emax + emin), 0.5 * (emax - emin)
    for k in (1, 2, 5, 10):
        x = O.chebyshev(lambda s: d * s, b, emin, emax, k)
        Tk = np.zeros(k + 1); Tk[k] = 1.0
        p = npcheb.chebval((theta - d) / delta, Tk) / npcheb.chebval(theta / delta, Tk)
        assert np.abs((b - d * x) - p * b).max() < 1e-12 * np.abs(b).max()
    # with Q = 0 (op = I) the k-step result is [1 - T_k((theta-1)/delta)/T_k(theta/delta)] b
    x = O.chebyshev(lambda s: s, b, emin, emax, 10)
    T10 = np.zeros(11); T10[10] = 1.0
    fac = 1 - npcheb.chebval((theta - 1) / delta, T10) / npcheb.chebval(theta / delta, T10)
    assert np.abs(x - fac * b).max() < 1e-12


def test_lanczos_recovers_largest_eigenvalue():
    rng = np.random.default_rng(4)
    d = np.sort(rng.uniform(0.5, 10.0, size=2 * 10 * 10))
    d[-1] = 25.0
    d = d.reshape(2, 10, 10)
    q0 = O.splitmix64_uniform(7, d.size).reshape(d.shape)
    assert abs(O.lanczos_max(lambda s: d * s, q0, 30) - 25.0) < 1e-8
    # small symmetric matrix: Ritz value after n steps equals the largest eigenvalue
    A = rng.standard_normal((12, 12)); A = A @ A.T
    lam = O.lanczos_max(lambda s: (A @ s.ravel()).reshape(s.shape), rng.standard_normal((12,)), 12)
    assert abs(lam - np.linalg.eigvalsh(A).max()) < 1e-9 * lam


def test_splitmix64_reference_outputs():
    """First outputs of SplitMix64 from state 0, as published with the generator."""
    assert O.splitmix64(0, 4) == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                  0x06C45D188009454F, 0xF88BB8A8724C81EC]


def _paper_emax_table():
    rows = {}
    with open(os.path.join(GOLDEN, "emax_table.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, beta, e = line.split()
            rows.setdefault(name, []).append((float(beta), float(e)))
    return rows


def test_emax_scales_with_inverse_beta_as_in_the_paper():
    """(e_max,0 - 1) beta is beta-independent: true of the paper's printed estimates and of
    the oracle's coarse split operator at v = 0 (S Q S scales like 1/beta)."""
    for name, rows in _paper_emax_table().items():
        c = [(e - 1) * b for b, e in rows]
        assert max(c) - min(c) < 1e-4 * max(c), name
    n = 32
    g = O.Grid(n, n)
    rng = np.random.default_rng(5)
    mT = synth.gaussian_sum_isotropic(n, n, rng, count=8)
    mR = synth.gaussian_sum_isotropic(n, n, rng, count=8)
    q0 = O.splitmix64_uniform(11, 2 * g.N).reshape((2,) + g.shape)
    vals = []
    for beta in (1e-1, 1e-2, 1e-3):
        L = O.Level(g, mT, mR, O.Params(nt=4, beta=beta, reg=2))
        lin0 = O.linearize(L, np.zeros((2,) + g.shape))
        e = O.lanczos_max(lambda s: O.split_matvec(lin0, s), q0, 30)
        vals.append((e - 1) * beta)
    assert max(vals) - min(vals) < 1e-9 * max(vals)


def test_two_level_preconditioner_is_symmetric_positive():
    n = 32
    g = O.Grid(n, n)
    rng = np.random.default_rng(6)
    mT = synth.gaussian_sum_isotropic(n, n, rng, count=8)
    vgen = synth.random_velocity(n, n, rng, modes=6, kmax=3, amplitude=0.3)
    mR = O.transport_state(g, vgen, mT, 4)
    L = O.Level(g, mT, mR, O.Params(nt=4, beta=1e-3, reg=2))
    tl = O.setup_two_level(L)
    assert 1.0 <= tl.emin < tl.emax
    cg = tl.coarse.grid
    tl.lin_c = O.linearize(tl.coarse, np.zeros((2,) + cg.shape))
    r1, r2 = _rand(g, 7), _rand(g, 8)
    z1, z2 = O.apply_two_level(L, tl, r1), O.apply_two_level(L, tl, r2)
    # at v = 0 the coarse operator is exactly symmetric, so is P_2L^{-1}
    assert abs(np.sum(r1 * z2) - np.sum(z1 * r2)) < 1e-10 * abs(np.sum(r1 * z2))
    assert np.sum(r1 * z1) > 0 and np.sum(r2 * z2) > 0
    # high modes pass unchanged
    hi = r1 - O.lowpass(g, r1)
    assert np.abs(O.apply_two_level(L, tl, hi) - hi).max() < 1e-12


def _fourier_second_derivative(n):
    """Dense periodic Fourier second-derivative matrix on n (even) equispaced nodes, from its
    closed-form entries (differentiate the periodic sinc interpolant twice): -pi^2/(3h^2) - 1/6 on
    the diagonal, -(-1)^(i-j) / (2 sin^2((i-j)h/2)) off it.  Its eigenvalues are -k^2 for
    |k| <= n/2, the Nyquist mode included."""
    h = 2 * np.pi / n
    i = np.arange(n)
    d = (i[:, None] - i[None, :]) % n
    with np.errstate(divide="ignore"):
        D = -((-1.0) ** d) / (2.0 * np.sin(d * h / 2) ** 2)
    D[d == 0] = -np.pi ** 2 / (3 * h ** 2) - 1.0 / 6.0
    return D


@pytest.mark.parametrize("reg", [1, 2, 3])
def test_emin_is_smallest_eigenvalue_of_identity_plus_inverse_regulariser(reg):
    """e_min of P_2L is the smallest eigenvalue of I + (beta A')^{-1} on the coarse grid (section
    3.4.2, eigenvalue estimates: Q taken as a low-rank perturbation of the identity), A' = A with its
    zero eigenvalue (the constant) replaced by one.  The operator is assembled densely in real
    space from the sinc-interpolant differentiation matrices, not from FFT symbols; taking the fine
    grid's modes, or another regulariser power, changes the value."""
    fg = O.Grid(16, 24)
    cg = fg.coarse()
    beta = 2e-3
    lap = np.kron(_fourier_second_derivative(cg.n1), np.eye(cg.n2)) + \
        np.kron(np.eye(cg.n1), _fourier_second_derivative(cg.n2))
    A = np.linalg.matrix_power(-lap, reg)
    A = 0.5 * (A + A.T)
    A_prime = A + np.full(A.shape, 1.0 / cg.N)      # constant eigenvector: eigenvalue 0 -> 1
    M = np.eye(cg.N) + np.linalg.inv(beta * A_prime)
    e_dense = float(np.linalg.eigvalsh(0.5 * (M + M.T)).min())
    rng = np.random.default_rng(9)
    mT = synth.gaussian_sum_isotropic(fg.n1, fg.n2, rng, count=4)
    mR = synth.gaussian_sum_isotropic(fg.n1, fg.n2, rng, count=4)
    tl = O.setup_two_level(O.Level(fg, mT, mR, O.Params(nt=2, beta=beta, reg=reg)), lanczos_steps=5)
    assert abs(tl.emin - e_dense) < 1e-10 * e_dense
