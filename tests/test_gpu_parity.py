"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: FP64 context 1e-11 relative L2 per transport solve, gradient and matvec; mixed
context (FP32 fields, FP64 reductions) 1e-5 per transport solve and 1e-4 on gradients and
matvecs.  Sizes span several 16x16 tiles with ragged tails and non-power-of-two factors.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O
from gpu_common import TOL, check_reg_op, check_rel, problem, record, rel, same_inputs

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


def _ctx(slnk, L, prec, pc="reg", **kw):
    p = L.prm
    reg = {1: "h1", 2: "h2", 3: "h3"}[p.reg]
    return slnk.Context(L.grid.n1, L.grid.n2, p.nt, reg=reg, beta=p.beta, prec=prec, pc=pc, **kw)


CASES = [
    # kind, n1, n2, nt, beta, reg, prec
    ("smooth", 64, 64, 4, 1e-2, 1, "fp64"),
    ("gauss", 96, 80, 4, 1e-3, 2, "fp64"),
    ("gauss", 96, 80, 4, 1e-3, 2, "mixed"),
    ("gauss", 60, 120, 3, 1e-3, 2, "mixed"),
    ("gauss", 256, 256, 4, 1e-3, 2, "mixed"),
    ("gauss", 256, 256, 4, 1e-3, 2, "fp64"),
    ("smooth", 64, 64, 1, 1e-2, 1, "mixed"),
    # H3 (A = -Delta^3, symbol |k|^6)
    ("gauss", 96, 80, 4, 1e-3, 3, "fp64"),
    ("gauss", 128, 128, 4, 1e-3, 3, "mixed"),
]


def _check_reg_op(L, prec, got, ref, x, tol, what="operator"):
    """got ~ ref where ref contains beta A x (relative L2 and split-norm error, see check_reg_op)."""
    check_reg_op(L, got, ref, x, tol, f"{what} {prec}")


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}{c[1]}x{c[2]}_nt{c[3]}_{c[6]}")
def test_transport_gradient_matvec(slnk, case):
    kind, n1, n2, nt, beta, reg, prec = case
    print(f"case {case}", flush=True)
    L, vgen, vt = problem(kind, n1, n2, nt=nt, beta=beta, reg=reg)
    L.mT, L.mR, vgen, vt = same_inputs(prec, L.mT, L.mR, vgen, vt)
    tol = TOL[prec]
    ctx = _ctx(slnk, L, prec)
    # state transport of m_T by the generating velocity (eq. e:state-slm)
    m1 = torch.empty((n1, n2), dtype=ctx.dtype, device="cuda")
    ctx.transport_state(_t(vgen, prec), _t(L.mT, prec), m1)
    check_rel(f"transport {n1}x{n2} nt{nt} {prec}", _np(m1), O.transport_state(L.grid, vgen, L.mT, nt), tol["transport"])
    ctx.set_images(_t(L.mR, prec), _t(L.mT, prec))
    for scale in (0.0, 0.6):
        v = same_inputs(prec, scale * vgen)
        lin = O.linearize(L, v)
        g_ref = O.gradient(lin)
        g = torch.empty((2, n1, n2), dtype=ctx.dtype, device="cuda")
        J = ctx.gradient(_t(v, prec), g)
        assert abs(J - lin.J) / abs(lin.J) < tol["objective"]
        # beta A v is evaluated in FP64 from the given velocity in both contexts: only the FP64
        # rounding floor of the spectral symbol applies
        _check_reg_op(L, prec, _np(g), g_ref, v, tol["gradient"], "gradient")
        # internal fields of the linearisation: state at t = 1, adjoint at t = 0
        f = torch.empty((n1, n2), dtype=ctx.dtype, device="cuda")
        ctx.get_field(0, f)
        check_rel(f"state m1 {n1}x{n2} {prec}", _np(f), lin.m[-1], tol["transport"])
        ctx.get_field(4, f)
        if scale > 0:
            assert rel(_np(f), lin.lam[0]) < 10 * tol["transport"]
        # GN matvec (eq. e:hessian-matvec)
        h_ref = O.hessian_matvec(lin, vt)
        h = torch.empty_like(g)
        ctx.hessian_matvec(_t(vt, prec), h)
        _check_reg_op(L, prec, _np(h), h_ref, vt, tol["matvec"], "matvec")
        # split operator (no beta A: plain relative L2) and P_REG
        ctx.split_matvec(_t(vt, prec), h)
        check_rel(f"split matvec {n1}x{n2} {prec}", _np(h), O.split_matvec(lin, vt), tol["matvec"])
        ctx.precond_apply(_t(vt, prec), h)
        check_rel(f"P_REG {n1}x{n2} {prec}", _np(h), O.prec_reg(L.grid, vt, L.prm.beta, L.prm.reg), tol["matvec"])
    ctx.close()


def test_departure_points_and_adjoint_factor(slnk):
    L, vgen, _ = problem("gauss", 128, 128, nt=4)
    g = L.grid
    ctx = _ctx(slnk, L, "fp64")
    ctx.set_images(_t(L.mR, "fp64"), _t(L.mT, "fp64"))
    v = vgen
    ctx.objective(_t(v, "fp64"))
    lin = O.linearize(L, v)
    d = torch.empty((2, 128, 128), dtype=torch.float64, device="cuda")
    ctx.get_field(1, d)
    cells = (lin.Xf - g.X) / np.array(g.h)[:, None, None]
    assert np.abs(_np(d) - cells).max() < 1e-11
    ctx.get_field(2, d)
    cells = (lin.Xa - g.X) / np.array(g.h)[:, None, None]
    assert np.abs(_np(d) - cells).max() < 1e-11
    gam = torch.empty((128, 128), dtype=torch.float64, device="cuda")
    ctx.get_field(3, gam)
    assert np.abs(_np(gam) - lin.gamma).max() < 1e-12
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_two_level_preconditioner(slnk, prec):
    n = 128
    L, vgen, vt = problem("gauss", n, n, nt=4, beta=1e-3, reg=2)
    L.mT, L.mR, vgen, vt = same_inputs(prec, L.mT, L.mR, vgen, vt)
    ctx = _ctx(slnk, L, prec, pc="2l")
    ctx.set_images(_t(L.mR, prec), _t(L.mT, prec))
    tl = O.setup_two_level(L)
    emin, emax = ctx.cheb_bounds()
    assert abs(emin - tl.emin) < 1e-12 * tl.emin
    assert abs(emax - tl.emax) / tl.emax < (1e-9 if prec == "fp64" else 1e-5)
    v = same_inputs(prec, 0.5 * vgen)
    g = torch.empty((2, n, n), dtype=ctx.dtype, device="cuda")
    ctx.gradient(_t(v, prec), g)
    cg = tl.coarse.grid
    tl.lin_c = O.linearize(tl.coarse, np.stack([O.restrict(L.grid, cg, v[c]) for c in range(2)]))
    z_ref = O.apply_two_level(L, tl, vt)
    z = torch.empty_like(g)
    ctx.precond_apply(_t(vt, prec), z)
    # the bounds agree to 1e-5 in FP32, which the Chebyshev polynomial passes on
    check_rel(f"P_2L {n}^2 {prec}", _np(z), z_ref, (1e-11 if prec == "fp64" else 1e-4))
    ctx.close()


def test_global_gather_fallback_large_displacement(slnk):
    """Displacements beyond the LDS footprint take the coefficient pass + global gather."""
    n, nt = 64, 1
    L, _, vt = problem("smooth", n, n, nt=nt, beta=1e-2, reg=1)
    v = 7.0 * np.stack([np.ones((n, n)), 0.5 * np.ones((n, n))]) + L.grid.X[0] * 0
    v[0] += 0.3 * np.sin(L.grid.X[1])
    ctx = _ctx(slnk, L, "fp64")
    ctx.set_images(_t(L.mR, "fp64"), _t(L.mT, "fp64"))
    lin = O.linearize(L, v)
    g = torch.empty((2, n, n), dtype=torch.float64, device="cuda")
    ctx.gradient(_t(v, "fp64"), g)
    assert rel(_np(g), O.gradient(lin)) < 1e-11
    h = torch.empty_like(g)
    ctx.hessian_matvec(_t(vt, "fp64"), h)
    assert rel(_np(h), O.hessian_matvec(lin, vt)) < 1e-11
    ctx.close()


def test_errors_are_reported(slnk):
    n = 32
    L, vgen, vt = problem("smooth", n, n, nt=2, beta=1e-2, reg=1)
    with pytest.raises(slnk.SlnkError) as e:
        slnk.Context(30, 34, 2, prec="fp64", pc="reg")       # 17 is not a 2-3-5 number
    assert e.value.status == 1
    with pytest.raises(slnk.SlnkError):
        slnk.Context(32, 32, 0, prec="fp64", pc="reg")
    ctx = _ctx(slnk, L, "fp64")
    h = torch.empty((2, n, n), dtype=torch.float64, device="cuda")
    with pytest.raises(slnk.SlnkError) as e:
        ctx.hessian_matvec(_t(vt, "fp64"), h)       # no linearisation point yet
    assert e.value.status == 1
    bad = L.mR.copy()
    bad[3, 5] = np.nan
    with pytest.raises(slnk.SlnkError) as e:
        ctx.set_images(_t(bad, "fp64"), _t(L.mT, "fp64"))
    assert e.value.status == 4
    with pytest.raises(ValueError):
        ctx.gradient(_t(vgen, "mixed"), h)          # wrong dtype for an FP64 context
    ctx.close()


def test_newton_solve_fp64_matches_oracle(slnk):
    """Smooth 64^2 problem, H1, beta 1e-2, P_REG, FP64: the GPU takes the oracle's Newton path."""
    n, nt = 64, 4
    L, vgen, _ = problem("smooth", n, n, nt=nt, beta=1e-2, reg=1)
    v_ref, rep_ref = O.newton_solve(L, pc="reg", max_newton=10)
    ctx = _ctx(slnk, L, "fp64")
    ctx.set_images(_t(L.mR, "fp64"), _t(L.mT, "fp64"))
    v = torch.zeros((2, n, n), dtype=torch.float64, device="cuda")
    rep = ctx.newton_solve(v, max_newton=10)
    assert rep["status"] == "SLNK_OK"
    assert rep["newton_iters"] == rep_ref["newton_iters"]
    assert rep["pcg_iters"] == rep_ref["pcg_iters"]
    # the last entries of the history are gradient norms near the minimiser, where a 1e-15
    # perturbation of the data already moves the oracle's own values by ~3e-9 (inexact PCG)
    assert np.allclose(rep["grel"], rep_ref["grel"], rtol=1e-6, atol=0)
    assert np.allclose(rep["J"], rep_ref["J"], rtol=1e-11, atol=0)
    check_rel(f"Newton v smooth64 fp64", _np(v), v_ref, 1e-9)
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_newton_limit_status_matches_oracle(slnk, prec):
    """A solve that the Newton limit ends before the stop test reports SLNK_EMAXIT, as the oracle
    reports 'maxit'; with room for convergence both report success."""
    n, nt = 64, 4
    L, vgen, _ = problem("smooth", n, n, nt=nt, beta=1e-2, reg=1)
    L.mT, L.mR = same_inputs(prec, L.mT, L.mR)
    ctx = _ctx(slnk, L, prec)
    ctx.set_images(_t(L.mR, prec), _t(L.mT, prec))
    for max_newton, want, want_ref in ((1, "SLNK_EMAXIT", "maxit"), (10, "SLNK_OK", "ok")):
        _, rep_ref = O.newton_solve(L, pc="reg", max_newton=max_newton, gtol_rel=1e-3)
        v = torch.zeros((2, n, n), dtype=ctx.dtype, device="cuda")
        rep = ctx.newton_solve(v, max_newton=max_newton, gtol_rel=1e-3)
        assert rep_ref["status"] == want_ref
        assert rep["status"] == want, (max_newton, rep["status"])
        assert rep["newton_iters"] == rep_ref["newton_iters"]
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_underestimated_emax_is_reestimated(slnk, prec):
    """An e_max far below the coarse spectrum (CHEB(10) indefinite): the GPU detects r.z <= 0,
    re-estimates e_max by Lanczos at the current coarse linearisation and converges, taking the
    oracle's path (FP64: the same Newton and PCG counts and re-estimates; mixed: the same
    re-estimates and a final velocity within 1e-3)."""
    n = 64
    g = O.Grid(n, n)
    import synth
    rng = np.random.default_rng(21)
    mT = synth.gaussian_sum_isotropic(n, n, rng)
    vgen = synth.random_velocity(n, n, rng, modes=16, kmax=4, amplitude=0.3)
    mT = same_inputs(prec, mT)
    mR = same_inputs(prec, O.transport_state(g, vgen, mT, 4))
    L = O.Level(g, mT, mR, O.Params(nt=4, beta=1e-3, reg=2))
    ctx = _ctx(slnk, L, prec, pc="2l")
    ctx.set_images(_t(mR, prec), _t(mT, prec))
    emin, emax = ctx.cheb_bounds()
    low = 1.0 + 0.05 * (emax - 1.0)
    v_ref, rep_ref = O.newton_solve(L, pc="2l", max_newton=10, emax=low)
    assert rep_ref["cheb_reestimates"] >= 1
    ctx.set_cheb_emax(low)
    assert ctx.cheb_bounds() == (emin, low)
    v = torch.zeros((2, n, n), dtype=ctx.dtype, device="cuda")
    rep = ctx.newton_solve(v, max_newton=10)
    print(rep["grel"], rep["pcg"], rep["cheb_reestimates"], rep_ref["grel"], rep_ref["cheb_reestimates"], flush=True)
    assert rep["status"] == "SLNK_OK" and rep["grel"][-1] <= 1e-2
    assert rep["cheb_reestimates"] == rep_ref["cheb_reestimates"]
    if prec == "fp64":
        assert rep["newton_iters"] == rep_ref["newton_iters"] and rep["pcg_iters"] == rep_ref["pcg_iters"]
    check_rel(f"Newton v, e_max re-estimated, {prec}", _np(v), v_ref, 1e-9 if prec == "fp64" else 1e-3)
    # a second solve starts again from the set-up bound, not from the first solve's re-estimate
    v2 = torch.zeros_like(v)
    rep2 = ctx.newton_solve(v2, max_newton=10)
    assert rep2["emax"] == low and rep2["cheb_reestimates"] == rep["cheb_reestimates"]
    assert rep2["pcg"] == rep["pcg"] and torch.equal(v2, v)
    with pytest.raises(slnk.SlnkError) as e:
        ctx.set_cheb_emax(0.5 * emin)
    assert e.value.status == 1
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_headline_solve_matches_oracle(slnk, prec):
    """The 256^2 benchmark problem (32 Gaussians, 16-mode velocity of amplitude 0.3, seed 2, nt 4,
    H2, beta 1e-3, P_2L with a 128^2 coarse grid and CHEB(10)): the GPU's final velocity meets the
    stop rule as the oracle evaluates it (||g||_inf <= 1.02e-2 ||g_0||_inf) and lies within 1e-9
    (FP64) or 1e-3 (mixed) of the oracle's Newton solution."""
    import synth
    cfg = synth.config("gauss256")
    n, nt = cfg["n1"], cfg["nt"]
    g = O.Grid(n, n)
    mT, vgen = same_inputs(prec, cfg["mT"], cfg["v_gen"])
    mR = same_inputs(prec, O.transport_state(g, vgen, mT, nt))
    L = O.Level(g, mT, mR, O.Params(nt=nt, beta=cfg["beta"], reg=cfg["reg"]))
    v_ref, rep_ref = O.newton_solve(L, pc="2l", max_newton=20)
    assert rep_ref["status"] == "ok"
    ctx = _ctx(slnk, L, prec, pc="2l")
    ctx.set_images(_t(L.mR, prec), _t(L.mT, prec))
    v = torch.zeros((2, n, n), dtype=ctx.dtype, device="cuda")
    rep = ctx.newton_solve(v, max_newton=20)
    print("GPU", rep["grel"], rep["pcg"], "oracle", rep_ref["grel"], flush=True)
    assert rep["status"] == "SLNK_OK"
    vv = _np(v)
    g_at = O.gradient(O.linearize(L, vv))
    record(f"Newton 256^2 P_2L {prec}: oracle ||g||_rel at the GPU's v", np.abs(g_at).max() / rep_ref["g0_inf"],
           1.02e-2)
    assert np.abs(g_at).max() / rep_ref["g0_inf"] <= 1.02e-2
    check_rel(f"Newton v gauss256 P_2L {prec}", vv, v_ref, (1e-9 if prec == "fp64" else 1e-3))
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_newton_solve_two_level(slnk, prec):
    """Gaussian 96^2 problem, H2, beta 1e-3, P_2L: same final velocity as the oracle (1e-9 in
    FP64, 1e-3 mixed), and the oracle's gradient at the GPU's result meets the stop rule."""
    n, nt = 96, 4
    L, vgen, _ = problem("gauss", n, n, nt=nt, beta=1e-3, reg=2)
    L.mT, L.mR = same_inputs(prec, L.mT, L.mR)
    v_ref, rep_ref = O.newton_solve(L, pc="2l", max_newton=10)
    ctx = _ctx(slnk, L, prec, pc="2l")
    ctx.set_images(_t(L.mR, prec), _t(L.mT, prec))
    v = torch.zeros((2, n, n), dtype=ctx.dtype, device="cuda")
    rep = ctx.newton_solve(v, max_newton=10)
    print(rep["grel"], rep_ref["grel"], rep["pcg"], flush=True)
    assert rep["status"] == "SLNK_OK"
    vv = _np(v)
    check_rel(f"Newton v gauss96 P_2L {prec}", vv, v_ref, (1e-9 if prec == "fp64" else 1e-3))
    g_at = O.gradient(O.linearize(L, vv))
    assert np.abs(g_at).max() / rep_ref["g0_inf"] <= 1.02e-2
    ctx.close()


def test_graph_replays_match_eager_launches(slnk):
    """The captured matvec / preconditioner graphs give the eager results on every replay, with
    eager work (new linearisation points) between the replays."""
    n = 128
    L, vgen, vt = problem("gauss", n, n, nt=4, beta=1e-3, reg=2)
    L.mT, L.mR, vgen, vt = same_inputs("mixed", L.mT, L.mR, vgen, vt)
    ctxs = [_ctx(slnk, L, "mixed", pc="2l", use_graphs=flag) for flag in (True, False)]
    for c in ctxs:
        c.set_images(_t(L.mR, "mixed"), _t(L.mT, "mixed"))
    g = torch.empty((2, n, n), dtype=torch.float32, device="cuda")
    outs = [torch.empty_like(g) for _ in ctxs]
    for rep, scale in enumerate((0.5, 0.9, 0.2, 0.5)):
        for c, out in zip(ctxs, outs):
            c.gradient(_t(scale * vgen, "mixed"), g)       # new linearisation (eager work)
            torch.cuda.synchronize()
            c.precond_apply(_t(vt, "mixed"), out)
            torch.cuda.synchronize()
        assert torch.equal(outs[0], outs[1]), rep
    vs = [torch.zeros((2, n, n), dtype=torch.float32, device="cuda") for _ in ctxs]
    reps = [c.newton_solve(v, max_newton=6) for c, v in zip(ctxs, vs)]
    assert reps[0]["grel"] == reps[1]["grel"] and reps[0]["pcg"] == reps[1]["pcg"]
    assert torch.equal(vs[0], vs[1])
    for c in ctxs:
        c.close()


def _batch_problems(n1, n2, seeds, amps, nt=4, beta=1e-3, reg=2):
    return [problem("gauss", n1, n2, nt=nt, beta=beta, reg=reg, seed=s, amp=a) for s, a in zip(seeds, amps)]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_items_match_single_contexts(slnk, prec):
    """A context of B = 3 different problems gives, item by item, the results of three B = 1
    contexts bit for bit (items share no data), and each item matches the oracle."""
    n1, n2, B = 96, 80, 3
    probs = _batch_problems(n1, n2, seeds=(5, 6, 7), amps=(0.3, 0.15, 0.45))
    for L, vgen, vt in probs:
        L.mT, L.mR = same_inputs(prec, L.mT, L.mR)
    vts = [same_inputs(prec, p[2]) for p in probs]
    vs = [same_inputs(prec, 0.6 * p[1]) for p in probs]
    stack = lambda arrs: _t(np.stack(arrs), prec)
    L0 = probs[0][0]
    cb = _ctx(slnk, L0, prec, pc="2l", batch=B)
    cb.set_images(stack([p[0].mR for p in probs]), stack([p[0].mT for p in probs]))
    gb = torch.empty((B, 2, n1, n2), dtype=cb.dtype, device="cuda")
    Jb = cb.gradient(stack(vs), gb)
    hb, zb, sb = torch.empty_like(gb), torch.empty_like(gb), torch.empty_like(gb)
    cb.hessian_matvec(stack(vts), hb)
    cb.split_matvec(stack(vts), sb)
    cb.precond_apply(stack(vts), zb)
    bounds = cb.cheb_bounds()
    tol = TOL[prec]
    for z, (L, vgen, vt) in enumerate(probs):
        c1 = _ctx(slnk, L, prec, pc="2l")
        c1.set_images(_t(L.mR, prec), _t(L.mT, prec))
        g1 = torch.empty((2, n1, n2), dtype=c1.dtype, device="cuda")
        J1 = c1.gradient(_t(vs[z], prec), g1)
        h1, z1, s1 = torch.empty_like(g1), torch.empty_like(g1), torch.empty_like(g1)
        c1.hessian_matvec(_t(vts[z], prec), h1)
        c1.split_matvec(_t(vts[z], prec), s1)
        c1.precond_apply(_t(vts[z], prec), z1)
        assert Jb[z] == J1 and bounds[z] == c1.cheb_bounds(), z
        for a, b in ((gb[z], g1), (hb[z], h1), (sb[z], s1), (zb[z], z1)):
            assert torch.equal(a, b), z
        c1.close()
        lin = O.linearize(L, vs[z])
        assert abs(Jb[z] - lin.J) / abs(lin.J) < tol["objective"]
        _check_reg_op(L, prec, _np(gb[z]), O.gradient(lin), vs[z], tol["gradient"], "gradient")
        _check_reg_op(L, prec, _np(hb[z]), O.hessian_matvec(lin, vts[z]), vts[z], tol["matvec"], "matvec")
    cb.close()


def test_batch_mixed_halos_use_one_path(slnk):
    """Items whose displacements exceed the LDS footprint and items that fit share launches (the
    batch takes the coefficient pass + global gather): every item still matches the oracle."""
    n, nt = 64, 1
    L, _, vt = problem("smooth", n, n, nt=nt, beta=1e-2, reg=1)
    big = 7.0 * np.stack([np.ones((n, n)), 0.5 * np.ones((n, n))])
    big[0] += 0.3 * np.sin(L.grid.X[1])
    small = 0.05 * big
    ctx = _ctx(slnk, L, "fp64", batch=2)
    mm = lambda a: _t(np.stack([a, a]), "fp64")
    ctx.set_images(mm(L.mR), mm(L.mT))
    g = torch.empty((2, 2, n, n), dtype=torch.float64, device="cuda")
    ctx.gradient(_t(np.stack([small, big]), "fp64"), g)
    h = torch.empty_like(g)
    ctx.hessian_matvec(mm(vt), h)
    for z, v in enumerate((small, big)):
        lin = O.linearize(L, v)
        assert rel(_np(g[z]), O.gradient(lin)) < 1e-11, z
        assert rel(_np(h[z]), O.hessian_matvec(lin, vt)) < 1e-11, z
    ctx.close()


@pytest.mark.parametrize("prec,pc", [("fp64", "reg"), ("mixed", "2l")])
def test_batch_newton_items_stop_on_their_own(slnk, prec, pc):
    """Batched Newton--Krylov: items that need different numbers of Newton and PCG steps run in
    lock step; each item's report and velocity equal those of its own B = 1 solve."""
    n, B = 64, 3
    probs = _batch_problems(n, n, seeds=(11, 12, 13), amps=(0.35, 0.1, 0.25), beta=1e-3 if pc == "2l" else 1e-2,
                            reg=2 if pc == "2l" else 1)
    for L, _, _ in probs:
        L.mT, L.mR = same_inputs(prec, L.mT, L.mR)
    L0 = probs[0][0]
    cb = _ctx(slnk, L0, prec, pc=pc, batch=B)
    cb.set_images(_t(np.stack([p[0].mR for p in probs]), prec), _t(np.stack([p[0].mT for p in probs]), prec))
    vb = torch.zeros((B, 2, n, n), dtype=cb.dtype, device="cuda")
    reps = cb.newton_solve(vb, max_newton=10)
    iters = set()
    for z, (L, _, _) in enumerate(probs):
        c1 = _ctx(slnk, L, prec, pc=pc)
        c1.set_images(_t(L.mR, prec), _t(L.mT, prec))
        v1 = torch.zeros((2, n, n), dtype=c1.dtype, device="cuda")
        r1 = c1.newton_solve(v1, max_newton=10)
        for key in ("status", "newton_iters", "pcg_iters", "matvecs", "grel", "J", "pcg", "line_search_evals"):
            assert reps[z][key] == r1[key], (z, key)
        assert torch.equal(vb[z], v1), z
        iters.add((r1["newton_iters"], r1["pcg_iters"]))
        c1.close()
    assert len(iters) > 1  # the items really took different paths
    cb.close()


@pytest.mark.parametrize("path", [1, 2, 3])
def test_forced_sl_paths_match_oracle(slnk, path):
    """sl_path = 1 (coefficient pass + global gather for every step), 2 and 3 (the fused step with
    16 x 16 or 16 x 32 threads per tile whatever the launch size) give the oracle's results."""
    n, nt = 64, 4
    print(f"sl_path {path}", flush=True)
    L, vgen, vt = problem("smooth", n, n, nt=nt, beta=1e-2, reg=1)
    ctx = _ctx(slnk, L, "fp64", sl_path=path)
    ctx.set_images(_t(L.mR, "fp64"), _t(L.mT, "fp64"))
    v = 0.6 * vgen
    lin = O.linearize(L, v)
    g = torch.empty((2, n, n), dtype=torch.float64, device="cuda")
    J = ctx.gradient(_t(v, "fp64"), g)
    assert abs(J - lin.J) / abs(lin.J) < 1e-12
    assert rel(_np(g), O.gradient(lin)) < 1e-11
    h = torch.empty_like(g)
    ctx.hessian_matvec(_t(vt, "fp64"), h)
    assert rel(_np(h), O.hessian_matvec(lin, vt)) < 1e-11
    ctx.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_tiled_coefficient_pass_on_ragged_grid(slnk, prec):
    """sl_path = 1 on 96 x 160: the two-kernel step's 2-D coefficient pass (64 x 64 output tiles
    with their 90-point filter halo staged in LDS) on a grid that leaves partial tiles in both
    directions and is barely wider than the staged side, so the periodic wraps of the halo are
    exercised; transport, gradient and matvec against the oracle."""
    n1, n2 = 96, 160
    print(f"tiled coefficient pass {n1}x{n2} {prec}", flush=True)
    L, vgen, vt = problem("gauss", n1, n2, nt=4, beta=1e-3, reg=2, seed=71, amp=0.3)
    L.mT, L.mR, vgen, vt = same_inputs(prec, L.mT, L.mR, vgen, vt)
    ctx = _ctx(slnk, L, prec, pc="reg", sl_path=1)
    dt = torch.float64 if prec == "fp64" else torch.float32
    m1 = torch.empty((n1, n2), dtype=dt, device="cuda")
    ctx.transport_state(_t(vgen, prec), _t(L.mT, prec), m1)
    check_rel(f"transport {n1}x{n2} {prec}", _np(m1), O.transport_state(L.grid, vgen, L.mT, 4), TOL[prec]["transport"])
    ctx.set_images(_t(L.mR, prec), _t(L.mT, prec))
    v = same_inputs(prec, 0.7 * vgen)
    lin = O.linearize(L, v)
    g = torch.empty((2, n1, n2), dtype=dt, device="cuda")
    ctx.gradient(_t(v, prec), g)
    _check_reg_op(L, prec, _np(g), O.gradient(lin), v, TOL[prec]["gradient"], "gradient")
    h = torch.empty_like(g)
    ctx.hessian_matvec(_t(vt, prec), h)
    _check_reg_op(L, prec, _np(h), O.hessian_matvec(lin, vt), vt, TOL[prec]["matvec"], "matvec")
    ctx.close()


def test_ragged_batch_matches_single_contexts(slnk):
    """Pairs of three different grid sizes in one ragged batch: every pair's gradient, matvec and
    Newton solve equal those of its own batch-1 context; after autotuning, results still match the
    oracle."""
    prec, nt = "mixed", 4
    sizes = [(64, 64), (96, 80), (64, 64), (128, 128), (96, 80)]
    probs = [problem("gauss", a, b, nt=nt, beta=1e-3, reg=2, seed=30 + p, amp=0.2 + 0.05 * p)
             for p, (a, b) in enumerate(sizes)]
    for L, _, _ in probs:
        L.mT, L.mR = same_inputs(prec, L.mT, L.mR)
    bc = slnk.BatchContext(sizes, nt, reg="h2", beta=1e-3, prec=prec, pc="2l")
    assert [(k[0], k[1], k[2]) for k in bc.buckets()] == [(128, 128, 1), (96, 80, 2), (64, 64, 2)]
    bc.set_images([_t(L.mR, prec) for L, _, _ in probs], [_t(L.mT, prec) for L, _, _ in probs])
    vs = [_t(same_inputs(prec, 0.5 * v), prec) for _, v, _ in probs]
    vts = [_t(same_inputs(prec, vt), prec) for _, _, vt in probs]
    gs = [torch.empty((2,) + s, dtype=torch.float32, device="cuda") for s in sizes]
    hs = [torch.empty_like(g) for g in gs]
    Js = bc.gradient(vs, gs)
    bc.hessian_matvec(vts, hs)
    singles = []
    for p, (L, _, _) in enumerate(probs):
        c1 = _ctx(slnk, L, prec, pc="2l")
        c1.set_images(_t(L.mR, prec), _t(L.mT, prec))
        g1, h1 = torch.empty_like(gs[p]), torch.empty_like(gs[p])
        assert c1.gradient(vs[p], g1) == Js[p], p
        c1.hessian_matvec(vts[p], h1)
        assert torch.equal(g1, gs[p]) and torch.equal(h1, hs[p]), p
        singles.append(c1)
    v0 = [torch.zeros_like(g) for g in gs]
    reps = bc.newton_solve(v0, max_newton=8)
    for p, c1 in enumerate(singles):
        v1 = torch.zeros_like(gs[p])
        r1 = c1.newton_solve(v1, max_newton=8)
        for key in ("status", "newton_iters", "pcg_iters", "matvecs", "grel", "J", "pcg"):
            assert reps[p][key] == r1[key], (p, key)
        assert torch.equal(v1, v0[p]), p
        c1.close()
    # autotune at a linearisation point, then the tuned operators still match the oracle
    bc.gradient(vs, gs)
    best = bc.autotune(vts, reps=2)
    assert len(best) == 3 and all(b > 0 for b in best)
    bc.hessian_matvec(vts, hs)
    for p, (L, _, _) in enumerate(probs):
        v = _np(vs[p])
        lin = O.linearize(L, v)
        _check_reg_op(L, prec, _np(hs[p]), O.hessian_matvec(lin, _np(vts[p])), _np(vts[p]), TOL[prec]["matvec"], "matvec")
    bc.close()


@pytest.mark.parametrize("shape", [(384, 768, 0), (1024, 1024, 1)], ids=lambda s: f"{s[0]}x{s[1]}_path{s[2]}")
def test_large_grids_match_oracle(slnk, shape):
    """Grid sizes of the batched workload (factor-3 lengths, 1024^2): state transport, gradient
    and matvec of the mixed-precision context against the oracle; at these sizes the 0.3-amplitude
    velocity displaces by up to ~12 cells per step.  1024^2 runs the two-kernel SL step
    (coefficient pass + global gather), the path the batched solver takes at that size."""
    n1, n2, path = shape
    prec = "mixed"
    print(f"large grid {shape}", flush=True)
    L, vgen, vt = problem("gauss", n1, n2, nt=4, beta=1e-3, reg=2, seed=40)
    L.mT, L.mR, vgen, vt = same_inputs(prec, L.mT, L.mR, vgen, vt)
    ctx = _ctx(slnk, L, prec, pc="reg", sl_path=path)
    m1 = torch.empty((n1, n2), dtype=torch.float32, device="cuda")
    ctx.transport_state(_t(vgen, prec), _t(L.mT, prec), m1)
    check_rel(f"transport {n1}x{n2} {prec}", _np(m1), O.transport_state(L.grid, vgen, L.mT, 4), TOL[prec]["transport"])
    ctx.set_images(_t(L.mR, prec), _t(L.mT, prec))
    v = same_inputs(prec, 0.7 * vgen)
    lin = O.linearize(L, v)
    g = torch.empty((2, n1, n2), dtype=torch.float32, device="cuda")
    ctx.gradient(_t(v, prec), g)
    _check_reg_op(L, prec, _np(g), O.gradient(lin), v, TOL[prec]["gradient"], "gradient")
    h = torch.empty_like(g)
    ctx.hessian_matvec(_t(vt, prec), h)
    _check_reg_op(L, prec, _np(h), O.hessian_matvec(lin, vt), vt, TOL[prec]["matvec"], "matvec")
    ctx.close()


def test_wide_batch_matches_single_contexts(slnk):
    """A 16-item batch at 128^2 gives its column FFT passes wide panels (several adjacent columns
    per workgroup); every item still equals its own batch-1 context bit for bit, and the oracle.
    Both contexts run the fused SL step with 16 x 32 threads per tile (sl_path 3): by launch size
    the 1024-tile batch would take 16 x 16-thread blocks, whose filter tasks group their outputs
    differently (the same values up to rounding)."""
    n, B, prec = 128, 16, "mixed"
    probs = _batch_problems(n, n, seeds=tuple(range(50, 50 + B)), amps=[0.1 + 0.02 * i for i in range(B)])
    for L, _, _ in probs:
        L.mT, L.mR = same_inputs(prec, L.mT, L.mR)
    vs = [same_inputs(prec, 0.5 * p[1]) for p in probs]
    vts = [same_inputs(prec, p[2]) for p in probs]
    stack = lambda arrs: _t(np.stack(arrs), prec)
    cb = _ctx(slnk, probs[0][0], prec, pc="reg", batch=B, sl_path=3)
    cb.set_images(stack([p[0].mR for p in probs]), stack([p[0].mT for p in probs]))
    gb = torch.empty((B, 2, n, n), dtype=torch.float32, device="cuda")
    cb.gradient(stack(vs), gb)
    hb = torch.empty_like(gb)
    cb.hessian_matvec(stack(vts), hb)
    for z in (0, 7, 15):
        L = probs[z][0]
        c1 = _ctx(slnk, L, prec, pc="reg", sl_path=3)
        c1.set_images(_t(L.mR, prec), _t(L.mT, prec))
        g1, h1 = torch.empty_like(gb[0]), torch.empty_like(gb[0])
        c1.gradient(_t(vs[z], prec), g1)
        c1.hessian_matvec(_t(vts[z], prec), h1)
        assert torch.equal(g1, gb[z]) and torch.equal(h1, hb[z]), z
        c1.close()
    lin = O.linearize(probs[7][0], vs[7])
    _check_reg_op(probs[7][0], prec, _np(hb[7]), O.hessian_matvec(lin, vts[7]), vts[7], TOL[prec]["matvec"], "matvec")
    cb.close()


WAVE_SHAPES = [
    # n1, n2, prec: every common transform length (64 .. 1024, 96 .. 768) as a row or column
    # length of the fine or the coarse grid; (96, 192) has a coarse length (48) outside that set
    (96, 192, "fp64"),
    (96, 192, "mixed"),
    (192, 384, "fp64"),
    (192, 384, "mixed"),
    (512, 256, "mixed"),
    (768, 128, "mixed"),
    (128, 1024, "mixed"),
]


@pytest.mark.parametrize("shape", WAVE_SHAPES, ids=lambda s: f"{s[0]}x{s[1]}_{s[2]}")
def test_spectral_passes_all_lengths(slnk, shape):
    """Gradient, GN matvec, split operator, P_REG and the two-level preconditioner on grids whose
    lengths take the wave-level spectral passes (and, for a pair of grids, restriction and
    prolongation between them) against the oracle."""
    n1, n2, prec = shape
    print(f"shape {shape}", flush=True)
    L, vgen, vt = problem("gauss", n1, n2, nt=4, beta=1e-3, reg=2, seed=60)
    L.mT, L.mR, vgen, vt = same_inputs(prec, L.mT, L.mR, vgen, vt)
    tol = TOL[prec]
    v = same_inputs(prec, 0.5 * vgen)
    lin = O.linearize(L, v)
    ctx = _ctx(slnk, L, prec, pc="reg")
    ctx.set_images(_t(L.mR, prec), _t(L.mT, prec))
    g = torch.empty((2, n1, n2), dtype=ctx.dtype, device="cuda")
    ctx.gradient(_t(v, prec), g)
    _check_reg_op(L, prec, _np(g), O.gradient(lin), v, tol["gradient"], "gradient")
    h = torch.empty_like(g)
    ctx.hessian_matvec(_t(vt, prec), h)
    _check_reg_op(L, prec, _np(h), O.hessian_matvec(lin, vt), vt, tol["matvec"], "matvec")
    ctx.split_matvec(_t(vt, prec), h)
    check_rel(f"split matvec {n1}x{n2} {prec}", _np(h), O.split_matvec(lin, vt), tol["matvec"])
    ctx.precond_apply(_t(vt, prec), h)
    check_rel(f"P_REG {n1}x{n2} {prec}", _np(h), O.prec_reg(L.grid, vt, L.prm.beta, L.prm.reg), tol["matvec"])
    ctx.close()
    ctx = _ctx(slnk, L, prec, pc="2l")
    ctx.set_images(_t(L.mR, prec), _t(L.mT, prec))
    tl = O.setup_two_level(L)
    emin, emax = ctx.cheb_bounds()
    assert abs(emax - tl.emax) / tl.emax < (1e-9 if prec == "fp64" else 1e-5)
    ctx.gradient(_t(v, prec), g)
    cg = tl.coarse.grid
    tl.lin_c = O.linearize(tl.coarse, np.stack([O.restrict(L.grid, cg, v[c]) for c in range(2)]))
    z = torch.empty_like(g)
    ctx.precond_apply(_t(vt, prec), z)
    check_rel(f"P_2L {n1}x{n2} {prec}", _np(z), O.apply_two_level(L, tl, vt), (1e-11 if prec == "fp64" else 1e-4))
    ctx.close()


def test_brain512_recipe_matches_oracle(slnk):
    """The 512^2 nt = 8 H1 workload (64 anisotropic smoothed Gaussians, 24-mode velocity of
    amplitude 0.5, seed 3), mixed precision, both SL kernel paths: state transport, gradient and
    GN matvec at 0.7 v_gen against the oracle."""
    import synth
    cfg = synth.config("brain512")
    n1, n2, nt = cfg["n1"], cfg["n2"], cfg["nt"]
    prec = "mixed"
    g = O.Grid(n1, n2)
    mT, vgen, vt = same_inputs(prec, cfg["mT"], cfg["v_gen"], cfg["vt"])
    mR = same_inputs(prec, O.transport_state(g, vgen, mT, nt))
    L = O.Level(g, mT, mR, O.Params(nt=nt, beta=cfg["beta"], reg=cfg["reg"]))
    v = same_inputs(prec, 0.7 * vgen)
    lin = O.linearize(L, v)
    g_ref, h_ref = O.gradient(lin), O.hessian_matvec(lin, vt)
    m_ref = O.transport_state(g, vgen, mT, nt)
    for path in (0, 1):
        print(f"brain512 sl_path {path}", flush=True)
        ctx = _ctx(slnk, L, prec, pc="reg", sl_path=path)
        m1 = torch.empty((n1, n2), dtype=torch.float32, device="cuda")
        ctx.transport_state(_t(vgen, prec), _t(mT, prec), m1)
        check_rel(f"transport {n1}x{n2} {prec}", _np(m1), m_ref, TOL[prec]["transport"])
        ctx.set_images(_t(mR, prec), _t(mT, prec))
        gg = torch.empty((2, n1, n2), dtype=torch.float32, device="cuda")
        ctx.gradient(_t(v, prec), gg)
        _check_reg_op(L, prec, _np(gg), g_ref, v, TOL[prec]["gradient"], "gradient")
        h = torch.empty_like(gg)
        ctx.hessian_matvec(_t(vt, prec), h)
        _check_reg_op(L, prec, _np(h), h_ref, vt, TOL[prec]["matvec"], "matvec")
        ctx.close()


def test_largest_grid_closed_forms(slnk):
    """2000 x 2048, the largest grid a context takes (its lengths take the generic transforms),
    mixed precision: zero-velocity transport is the identity; a constant velocity of one cell per
    step along x1 and two along x2 shifts cyclically by nt and 2 nt cells; at v = 0 the gradient is
    (m_R - m_T) grad m_T and the GN matvec beta A vt + (vt . grad m_T) grad m_T (at v = 0 the state
    and adjoint are constant in time, so Heun and the trapezoid rule are exact)."""
    import synth
    n1, n2, nt, prec = 2000, 2048, 4, "mixed"
    print(f"grid {n1}x{n2}", flush=True)
    g = O.Grid(n1, n2)
    rng = np.random.default_rng(70)
    mT = synth.gaussian_sum_isotropic(n1, n2, rng)
    mR = np.roll(mT, (3, -5), axis=(0, 1)) * 0.9 + 0.05
    vt = synth.random_velocity(n1, n2, np.random.default_rng(71), modes=16, kmax=4, amplitude=0.1)
    mT, mR, vt = same_inputs(prec, mT, mR, vt)
    L = O.Level(g, mT, mR, O.Params(nt=nt, beta=1e-3, reg=2))
    ctx = slnk.Context(n1, n2, nt, reg="h2", beta=1e-3, prec=prec, pc="reg")
    m1 = torch.empty((n1, n2), dtype=torch.float32, device="cuda")
    zero = torch.zeros((2, n1, n2), dtype=torch.float32, device="cuda")
    ctx.transport_state(zero, _t(mT, prec), m1)
    assert rel(_np(m1), mT) < TOL[prec]["transport"]
    shift = np.stack([np.full((n1, n2), nt * g.h[0]), np.full((n1, n2), 2 * nt * g.h[1])])
    ctx.transport_state(_t(shift, prec), _t(mT, prec), m1)
    assert rel(_np(m1), np.roll(mT, (nt, 2 * nt), axis=(0, 1))) < TOL[prec]["transport"]
    ctx.set_images(_t(mR, prec), _t(mT, prec))
    gm = O.fft_grad(g, mT)
    gg = torch.empty((2, n1, n2), dtype=torch.float32, device="cuda")
    ctx.gradient(zero, gg)
    assert rel(_np(gg), (mR - mT)[None] * gm) < TOL[prec]["gradient"]
    h = torch.empty_like(gg)
    ctx.hessian_matvec(_t(vt, prec), h)
    h_ref = 1e-3 * O.apply_reg(g, vt, 2) + (vt[0] * gm[0] + vt[1] * gm[1])[None] * gm
    _check_reg_op(L, prec, _np(h), h_ref, vt, TOL[prec]["matvec"], "matvec")
    ctx.close()
