"""Shared helpers of the GPU parity tests (inputs from synth, expected values from the oracle)."""

import numpy as np

import oracle as O
import synth

TOL = {"fp64": {"transport": 1e-11, "gradient": 1e-11, "matvec": 1e-11, "objective": 1e-12},
       "mixed": {"transport": 1e-5, "gradient": 1e-4, "matvec": 1e-4, "objective": 1e-6}}


EPS = {"fp64": 2.0 ** -53, "mixed": 2.0 ** -24}


def same_inputs(prec, *arrays):
    """The arrays as the GPU receives them (FP32-rounded for the mixed context), in FP64."""
    out = [np.asarray(a, dtype=np.float32).astype(np.float64) if prec == "mixed" else np.asarray(a, dtype=np.float64)
           for a in arrays]
    return out if len(out) > 1 else out[0]


# measured errors of the GPU path against the oracle, written out at the end of the session when
# the environment names a file (PARITY_REPORT)
ERRORS = []


def record(what, err, tol):
    """Keep and print one measured relative error next to the tolerance it is held to."""
    ERRORS.append({"what": what, "rel_err": float(err), "tol": float(tol)})
    print(f"parity {what}: rel err {err:.3e} (tol {tol:.0e})", flush=True)


def reg_floor(L, x):
    """Rounding floor of an FP64 beta A x: the spectral symbol beta |k|^(2 reg) amplifies the
    rounding of the FFT of x (about eps log2 N relative to ||x||, on every mode) by up to
    beta max a(k).  Both contexts form beta A in FP64 (the mixed one from its FP32 input), and so
    does the oracle."""
    g = L.grid
    amax = float(((g.n1 / 2) ** 2 + (g.n2 / 2) ** 2) ** L.prm.reg)
    return 64.0 * EPS["fp64"] * L.prm.beta * amax * float(np.linalg.norm(x))


def split_floor(L, x):
    """Rounding floor of S (beta A x) in the split norm, S = (beta A')^{-1/2}: the FFT rounding of x
    (white over the modes, eps relative) is multiplied by beta a(k) and then by (beta a(k))^{-1/2},
    i.e. by up to sqrt(beta max a)."""
    g = L.grid
    amax = float(((g.n1 / 2) ** 2 + (g.n2 / 2) ** 2) ** L.prm.reg)
    return 8.0 * EPS["fp64"] * (L.prm.beta * amax) ** 0.5 * float(np.linalg.norm(x))


def split_norm(L, x):
    """||S x||, S = (beta A')^{-1/2}: the norm of the split-preconditioned Krylov iteration."""
    return float(np.linalg.norm(O.split_scale(L.grid, x, L.prm.beta, L.prm.reg)))


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def check_rel(what, got, ref, tol):
    """Relative L2 error of a GPU result against the oracle's, recorded and held to tol."""
    e = rel(got, ref)
    record(what, e, tol)
    assert e < tol, (what, e, tol)


def check_reg_op(L, got, ref, x, tol, what="operator"):
    """got ~ ref where ref contains beta A x: relative L2 error at most tol (plus the FP64 rounding
    floor of beta A x, far below the mixed tolerance; at large grids it sets the FP64 bound), and
    the same in the split norm that the split-preconditioned PCG works in."""
    d = got - ref
    nref = float(np.linalg.norm(ref))
    e = float(np.linalg.norm(d)) / nref
    floor = reg_floor(L, x) / nref
    record(f"{what} {L.grid.n1}x{L.grid.n2} reg{L.prm.reg}", e, tol + floor)
    assert e <= tol + floor
    assert split_norm(L, d) <= tol * split_norm(L, ref) + split_floor(L, x)


def problem(kind, n1, n2=None, nt=4, beta=1e-3, reg=2, seed=2, amp=0.3):
    """Oracle level + generating velocity for a 'smooth' or 'gauss' problem of size n1 x n2."""
    n2 = n1 if n2 is None else n2
    g = O.Grid(n1, n2)
    if kind == "smooth":
        mT = synth.smooth_a_template(n1, n2)
        v = synth.smooth_a_velocity(n1, n2)
    else:
        rng = np.random.default_rng(seed)
        mT = synth.gaussian_sum_isotropic(n1, n2, rng)
        v = synth.random_velocity(n1, n2, rng, modes=16, kmax=4, amplitude=amp)
    mR = O.transport_state(g, v, mT, nt)
    vt = synth.random_velocity(n1, n2, np.random.default_rng(seed + 1000), modes=16, kmax=4, amplitude=0.1)
    return O.Level(g, mT, mR, O.Params(nt=nt, beta=beta, reg=reg)), v, vt
