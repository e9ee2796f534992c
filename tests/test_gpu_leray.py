"""GPU parity of the incompressible case (K = Leray projection applied to b and b~, section 3.1)
against the FP64 oracle, through the C ABI: gradient, Gauss--Newton and full-Newton matvecs, the
split operator, P_2L (Chebyshev bounds and application) and Newton solves.  Tolerances as for the
compressible path: FP64 1e-11, mixed 1e-4 (matvecs relative to the rounding floor of beta A vt)."""

from dataclasses import replace

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
import synth
from gpu_common import TOL, check_reg_op, problem, record, rel, same_inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slnk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1604_02153_amd as pkg
    pkg.load_library()
    return pkg


def _t(a, prec):
    dt = torch.float64 if prec == "fp64" else torch.float32
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dt)


def _np(t):
    return t.double().cpu().numpy()


def _ctx(slnk, L, prec, pc, **kw):
    p = L.prm
    reg = {1: "h1", 2: "h2", 3: "h3"}[p.reg]
    return slnk.Context(L.grid.n1, L.grid.n2, p.nt, reg=reg, beta=p.beta, prec=prec, pc=pc, proj="leray",
                        hessian=p.hessian, **kw)


def _check_reg_op(L, prec, got, ref, x, tol, what="operator"):
    """got ~ ref where ref contains beta A x (relative L2 and split-norm error, see check_reg_op)."""
    check_reg_op(L, got, ref, x, tol, f"Leray {what} {prec}")


CASES = [
    # kind, n1, n2, nt, beta, reg, prec, hessian, sl_path
    ("smooth", 64, 64, 4, 1e-2, 1, "fp64", "gn", 0),
    ("gauss", 96, 80, 4, 1e-3, 1, "fp64", "gn", 0),
    ("gauss", 96, 80, 4, 1e-3, 2, "fp64", "fn", 1),
    ("gauss", 96, 80, 4, 1e-3, 2, "mixed", "gn", 0),
    ("gauss", 60, 120, 3, 1e-3, 2, "mixed", "fn", 0),
    ("gauss", 256, 256, 4, 1e-3, 2, "mixed", "gn", 0),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}{c[1]}x{c[2]}_nt{c[3]}_{c[6]}_{c[7]}_path{c[8]}")
def test_leray_operators_match_oracle(slnk, case):
    kind, n1, n2, nt, beta, reg, prec, hess, path = case
    print(f"case {case}", flush=True)
    L, vgen, vt = problem(kind, n1, n2, nt=nt, beta=beta, reg=reg)
    L = O.Level(L.grid, L.mT, L.mR, replace(L.prm, proj=1, hessian=hess))
    L.mT, L.mR, vgen, vt = same_inputs(prec, L.mT, L.mR, vgen, vt)
    tol = TOL[prec]
    ctx = _ctx(slnk, L, prec, "2l", sl_path=path)
    ctx.set_images(_t(L.mR, prec), _t(L.mT, prec))
    tl = O.setup_two_level(L)
    emin, emax = ctx.cheb_bounds()
    assert abs(emin - tl.emin) < 1e-12 * tl.emin
    assert abs(emax - tl.emax) / tl.emax < (1e-9 if prec == "fp64" else 1e-5)
    v = same_inputs(prec, 0.6 * vgen)
    lin = O.linearize(L, v)
    g = torch.empty((2, n1, n2), dtype=ctx.dtype, device="cuda")
    J = ctx.gradient(_t(v, prec), g)
    assert abs(J - lin.J) / abs(lin.J) < tol["objective"]
    g_ref = O.gradient(lin)
    _check_reg_op(L, prec, _np(g), g_ref, v, tol["gradient"], "gradient")
    h = torch.empty_like(g)
    ctx.hessian_matvec(_t(vt, prec), h)
    _check_reg_op(L, prec, _np(h), O.hessian_matvec(lin, vt), vt, tol["matvec"], "matvec")
    ctx.split_matvec(_t(vt, prec), h)
    assert rel(_np(h), O.split_matvec(lin, vt)) < tol["matvec"]
    cg = tl.coarse.grid
    tl.lin_c = O.linearize(tl.coarse, np.stack([O.restrict(L.grid, cg, v[c]) for c in range(2)]))
    ctx.precond_apply(_t(vt, prec), h)
    assert rel(_np(h), O.apply_two_level(L, tl, vt)) < (1e-11 if prec == "fp64" else 1e-4)
    # the projected part of the gradient is divergence-free on the GPU too: div(g - beta A v) is a
    # rounding-level fraction of div b, b = int lambda grad m (the compressible b)
    bAv = L.prm.beta * O.apply_reg(L.grid, v, L.prm.reg)
    b = O.gradient(O.linearize(O.Level(L.grid, L.mT, L.mR, replace(L.prm, proj=0)), v)) - bAv
    div_b = np.abs(O.fft_div(L.grid, b)).max()
    assert np.abs(O.fft_div(L.grid, _np(g) - bAv)).max() < (1e-9 if prec == "fp64" else 1e-3) * div_b
    ctx.close()


@pytest.mark.parametrize("pc", ["reg", "2l"])
def test_leray_newton_solve_fp64_matches_oracle(slnk, pc):
    """Smooth 64^2 problem with a divergence-free generating velocity, H1, beta 1e-2, FP64: the GPU
    takes the oracle's incompressible Newton path and its iterate stays divergence-free."""
    n, nt = 64, 4
    g = O.Grid(n, n)
    mT = synth.smooth_a_template(n, n)
    vs = O.leray(g, synth.random_velocity(n, n, np.random.default_rng(2), modes=16, kmax=3, amplitude=0.3))
    L = O.Level(g, mT, O.transport_state(g, vs, mT, nt), O.Params(nt=nt, beta=1e-2, reg=1, proj=1))
    v_ref, rep_ref = O.newton_solve(L, pc=pc, max_newton=10)
    ctx = _ctx(slnk, L, "fp64", pc)
    ctx.set_images(_t(L.mR, "fp64"), _t(L.mT, "fp64"))
    v = torch.zeros((2, n, n), dtype=torch.float64, device="cuda")
    rep = ctx.newton_solve(v, max_newton=10)
    print(rep["grel"], rep_ref["grel"], flush=True)
    assert rep["status"] == "SLNK_OK"
    assert rep["newton_iters"] == rep_ref["newton_iters"]
    assert rep["pcg_iters"] == rep_ref["pcg_iters"]
    assert np.allclose(rep["grel"], rep_ref["grel"], rtol=1e-6, atol=0)
    vv = _np(v)
    assert rel(vv, v_ref) < 1e-9
    assert np.abs(O.fft_div(g, vv)).max() < 1e-10 * np.abs(vv).max()
    ctx.close()


def test_brain512ic_recipe_matches_oracle(slnk):
    """The incompressible 512^2 nt = 8 H1 workload (brain512 image, divergence-free 24-mode
    velocity of amplitude 0.5, K = Leray), mixed precision: gradient, GN matvec and P_2L bounds at
    0.7 v_gen against the oracle."""
    cfg = synth.config("brain512ic")
    n1, n2, nt = cfg["n1"], cfg["n2"], cfg["nt"]
    prec = "mixed"
    g = O.Grid(n1, n2)
    mT, vgen, vt = same_inputs(prec, cfg["mT"], cfg["v_gen"], cfg["vt"])
    mR = same_inputs(prec, O.transport_state(g, vgen, mT, nt))
    L = O.Level(g, mT, mR, O.Params(nt=nt, beta=cfg["beta"], reg=cfg["reg"], proj=1))
    v = same_inputs(prec, 0.7 * vgen)
    lin = O.linearize(L, v)
    ctx = _ctx(slnk, L, prec, "2l")
    ctx.set_images(_t(mR, prec), _t(mT, prec))
    gg = torch.empty((2, n1, n2), dtype=torch.float32, device="cuda")
    ctx.gradient(_t(v, prec), gg)
    _check_reg_op(L, prec, _np(gg), O.gradient(lin), v, TOL[prec]["gradient"], "gradient")
    h = torch.empty_like(gg)
    ctx.hessian_matvec(_t(vt, prec), h)
    _check_reg_op(L, prec, _np(h), O.hessian_matvec(lin, vt), vt, TOL[prec]["matvec"], "matvec")
    ctx.close()
