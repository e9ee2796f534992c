"""GPU parity of the full-Newton Hessian matvec (eq. e:hessian-matvec with the lambda terms; the
incremental adjoint of eq. e:inc-adj-slm with its source div(lambda vt)) against the FP64 oracle,
through the C ABI.  Same tolerances as the Gauss--Newton path: FP64 1e-11 relative L2, mixed
1e-4 on matvecs (relative to the rounding floor of beta A vt)."""

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


def _fn(L):
    return O.Level(L.grid, L.mT, L.mR, replace(L.prm, hessian="fn"))


def _ctx(slnk, L, prec, pc="reg", **kw):
    p = L.prm
    reg = {1: "h1", 2: "h2", 3: "h3"}[p.reg]
    return slnk.Context(L.grid.n1, L.grid.n2, p.nt, reg=reg, beta=p.beta, prec=prec, pc=pc, hessian="fn", **kw)


def _check_reg_op(L, prec, got, ref, x, tol, what="operator"):
    """got ~ ref where ref contains beta A x (relative L2 and split-norm error, see check_reg_op)."""
    check_reg_op(L, got, ref, x, tol, f"FN {what} {prec}")


def _point(L, vgen, n1, n2):
    """A compressible velocity away from the minimiser (lambda != 0, div v != 0)."""
    pert = synth.random_velocity(n1, n2, np.random.default_rng(77), modes=8, kmax=3, amplitude=0.1)
    return 0.6 * vgen + pert


CASES = [
    # kind, n1, n2, nt, beta, reg, prec, sl_path
    ("smooth", 64, 64, 4, 1e-2, 1, "fp64", 0),
    ("gauss", 96, 80, 4, 1e-3, 2, "fp64", 0),
    ("gauss", 96, 80, 4, 1e-3, 2, "fp64", 1),
    ("gauss", 96, 80, 4, 1e-3, 2, "mixed", 0),
    ("gauss", 60, 120, 3, 1e-3, 2, "mixed", 0),
    ("gauss", 256, 256, 4, 1e-3, 2, "mixed", 0),
    ("gauss", 256, 256, 4, 1e-3, 2, "mixed", 1),
    ("smooth", 64, 64, 1, 1e-2, 1, "mixed", 0),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}{c[1]}x{c[2]}_nt{c[3]}_{c[6]}_path{c[7]}")
def test_full_newton_matvec_matches_oracle(slnk, case):
    kind, n1, n2, nt, beta, reg, prec, path = case
    print(f"case {case}", flush=True)
    L, vgen, vt = problem(kind, n1, n2, nt=nt, beta=beta, reg=reg)
    L = _fn(L)
    v = _point(L, vgen, n1, n2)
    L.mT, L.mR, v, vt = same_inputs(prec, L.mT, L.mR, v, vt)
    tol = TOL[prec]
    ctx = _ctx(slnk, L, prec, sl_path=path)
    ctx.set_images(_t(L.mR, prec), _t(L.mT, prec))
    lin = O.linearize(L, v)
    g = torch.empty((2, n1, n2), dtype=ctx.dtype, device="cuda")
    ctx.gradient(_t(v, prec), g)
    h_ref = O.hessian_matvec(lin, vt)
    # the lambda terms are a sizeable part of the product at this point
    lin_gn = O.linearize(O.Level(L.grid, L.mT, L.mR, replace(L.prm, hessian="gn")), v)
    assert rel(O.hessian_matvec(lin_gn, vt), h_ref) > 20 * tol["matvec"]
    h = torch.empty_like(g)
    ctx.hessian_matvec(_t(vt, prec), h)
    _check_reg_op(L, prec, _np(h), h_ref, vt, tol["matvec"], "matvec")
    ctx.split_matvec(_t(vt, prec), h)
    assert rel(_np(h), O.split_matvec(lin, vt)) < tol["matvec"]
    # a second gradient at another point replaces every kept adjoint level
    v2 = same_inputs(prec, 0.3 * vgen)
    ctx.gradient(_t(v2, prec), g)
    ctx.hessian_matvec(_t(vt, prec), h)
    _check_reg_op(L, prec, _np(h), O.hessian_matvec(O.linearize(L, v2), vt), vt, tol["matvec"], "matvec")
    ctx.close()


def test_full_newton_matvec_at_zero_closed_form(slnk):
    """v = 0 (FP64): H vt = beta A vt + (f0 + div(lambda vt) / 2) grad m_T - (lambda / 2) grad f0,
    f0 = vt . grad m_T, lambda = m_R - m_T (the oracle's closed-form pin, on the GPU)."""
    n = 96
    L, vgen, vt = problem("gauss", n, n, nt=4, beta=1e-3, reg=2)
    L = _fn(L)
    g = L.grid
    ctx = _ctx(slnk, L, "fp64")
    ctx.set_images(_t(L.mR, "fp64"), _t(L.mT, "fp64"))
    gg = torch.empty((2, n, n), dtype=torch.float64, device="cuda")
    ctx.gradient(_t(np.zeros((2, n, n)), "fp64"), gg)
    gm = O.fft_grad(g, L.mT)
    lam = L.mR - L.mT
    f0 = vt[0] * gm[0] + vt[1] * gm[1]
    ref = L.prm.beta * O.apply_reg(g, vt, 2) + (f0 + 0.5 * O.fft_div(g, lam * vt)) * gm - 0.5 * lam * O.fft_grad(g, f0)
    h = torch.empty_like(gg)
    ctx.hessian_matvec(_t(vt, "fp64"), h)
    assert rel(_np(h), ref) < 1e-11
    ctx.close()


def test_full_newton_batch_items_match_single_contexts(slnk):
    """B = 3 different problems: item by item the results of three B = 1 contexts, bit for bit
    (the kept adjoint levels and full-Newton work buffers are per item)."""
    n1, n2, B, prec = 96, 80, 3, "mixed"
    probs = []
    for seed, amp in ((5, 0.3), (6, 0.15), (7, 0.45)):
        L, vgen, vt = problem("gauss", n1, n2, nt=4, beta=1e-3, reg=2, seed=seed, amp=amp)
        L = _fn(L)
        L.mT, L.mR = same_inputs(prec, L.mT, L.mR)
        probs.append((L, same_inputs(prec, _point(L, vgen, n1, n2)), same_inputs(prec, vt)))
    stack = lambda arrs: _t(np.stack(arrs), prec)
    cb = _ctx(slnk, probs[0][0], prec, pc="2l", batch=B)
    cb.set_images(stack([p[0].mR for p in probs]), stack([p[0].mT for p in probs]))
    gb = torch.empty((B, 2, n1, n2), dtype=cb.dtype, device="cuda")
    cb.gradient(stack([p[1] for p in probs]), gb)
    hb, sb = torch.empty_like(gb), torch.empty_like(gb)
    cb.hessian_matvec(stack([p[2] for p in probs]), hb)
    cb.split_matvec(stack([p[2] for p in probs]), sb)
    for z, (L, v, vt) in enumerate(probs):
        c1 = _ctx(slnk, L, prec, pc="2l")
        c1.set_images(_t(L.mR, prec), _t(L.mT, prec))
        g1 = torch.empty((2, n1, n2), dtype=c1.dtype, device="cuda")
        c1.gradient(_t(v, prec), g1)
        h1, s1 = torch.empty_like(g1), torch.empty_like(g1)
        c1.hessian_matvec(_t(vt, prec), h1)
        c1.split_matvec(_t(vt, prec), s1)
        assert torch.equal(hb[z], h1) and torch.equal(sb[z], s1), z
        c1.close()
        lin = O.linearize(L, v)
        _check_reg_op(L, prec, _np(hb[z]), O.hessian_matvec(lin, vt), vt, TOL[prec]["matvec"], "matvec")
    cb.close()


@pytest.mark.parametrize("pc", ["reg", "2l"])
def test_full_newton_solve_fp64_matches_oracle(slnk, pc):
    """Smooth 64^2 problem, H1, beta 1e-2, FP64, gtol 1e-5: the GPU takes the oracle's full-Newton
    path (same iteration counts and gradient history, quadratic final contraction)."""
    n, nt = 64, 4
    L, vgen, _ = problem("smooth", n, n, nt=nt, beta=1e-2, reg=1)
    L = _fn(L)
    v_ref, rep_ref = O.newton_solve(L, pc=pc, gtol_rel=1e-5, max_newton=8)
    ctx = _ctx(slnk, L, "fp64", pc=pc)
    ctx.set_images(_t(L.mR, "fp64"), _t(L.mT, "fp64"))
    v = torch.zeros((2, n, n), dtype=torch.float64, device="cuda")
    rep = ctx.newton_solve(v, max_newton=8, gtol_rel=1e-5)
    print(rep["grel"], rep_ref["grel"], flush=True)
    assert rep["status"] == "SLNK_OK"
    assert rep["newton_iters"] == rep_ref["newton_iters"]
    assert rep["pcg_iters"] == rep_ref["pcg_iters"]
    assert np.allclose(rep["grel"][:-1], rep_ref["grel"][:-1], rtol=1e-6, atol=0)
    assert rep["grel"][-1] <= 1e-5 and rep["grel"][-1] < 1e-2 * rep["grel"][-2]
    # the last step starts from ||g||rel ~ 2e-3 with an inexact PCG solve: rounding moves the
    # final iterate by ~1e-7 relative (its gradient, ~3e-6 of g_0, by ~1%)
    assert rel(_np(v), v_ref) < 1e-6
    ctx.close()


def test_full_newton_solve_two_level_mixed(slnk):
    """Gaussian 96^2, H2, beta 1e-3, P_2L, mixed precision.  Far from the minimiser the full-Newton
    Hessian is indefinite, so PCG leaves early on negative curvature and the path depends on
    rounding; the solve must still stop where the oracle's gradient at its result meets the stop
    rule."""
    n, nt, prec = 96, 4, "mixed"
    L, vgen, _ = problem("gauss", n, n, nt=nt, beta=1e-3, reg=2)
    L.mT, L.mR = same_inputs(prec, L.mT, L.mR)
    Lfn = _fn(L)
    g0 = O.gradient(O.linearize(L, np.zeros((2, n, n))))
    ctx = _ctx(slnk, Lfn, prec, pc="2l")
    ctx.set_images(_t(L.mR, prec), _t(L.mT, prec))
    v = torch.zeros((2, n, n), dtype=ctx.dtype, device="cuda")
    rep = ctx.newton_solve(v, max_newton=12)
    print(rep["grel"], rep["pcg"], flush=True)
    assert rep["status"] == "SLNK_OK"
    g_at = O.gradient(O.linearize(L, _np(v)))
    assert np.abs(g_at).max() / np.abs(g0).max() <= 1.02e-2
    ctx.close()
