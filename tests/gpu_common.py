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


def reg_floor(L, prec, x):
    """Rounding floor of beta A x: the spectral symbol beta |k|^(2 reg) amplifies the rounding of
    x and of the FFT (about eps log2 N relative to ||x||) by up to beta max a(k)."""
    g = L.grid
    amax = float(((g.n1 / 2) ** 2 + (g.n2 / 2) ** 2) ** L.prm.reg)
    return 64.0 * EPS[prec] * L.prm.beta * amax * float(np.linalg.norm(x))


def split_floor(L, prec, x):
    """Rounding floor of S (beta A x) in the split norm, S = (beta A')^{-1/2}: the FFT rounding of x
    (white over the modes, eps relative) is multiplied by beta a(k) and then by (beta a(k))^{-1/2},
    i.e. by up to sqrt(beta max a); about 0.5 eps sqrt(beta max a) ||x|| is observed in FP32."""
    g = L.grid
    amax = float(((g.n1 / 2) ** 2 + (g.n2 / 2) ** 2) ** L.prm.reg)
    return 8.0 * EPS[prec] * (L.prm.beta * amax) ** 0.5 * float(np.linalg.norm(x))


def split_norm(L, x):
    """||S x||, S = (beta A')^{-1/2}: the norm of the split-preconditioned Krylov iteration."""
    return float(np.linalg.norm(O.split_scale(L.grid, x, L.prm.beta, L.prm.reg)))


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


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
