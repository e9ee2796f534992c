"""Seeded synthetic inputs shaped like the paper's 2-D registration problems.

This module holds only input recipes (images, velocity fields, search
directions); none of the registration method's arithmetic lives here.  Both
the FP64 oracle (in tests) and the GPU library (in tests and the benchmark)
consume what it produces.  The reference image m_R of each problem is the
template transported by the generating velocity; the caller computes it with
whichever implementation it is exercising.

Value ranges follow the paper's test problems: intensities in [0, 1], velocity
magnitudes of order 0.5 (section 4, synthetic problems figure), grids from 64^2
to 512^2.  The paper's own images are not available; these recipes stand in
for them.
"""

from __future__ import annotations

import math

import numpy as np

__all__ = ["grid_coords", "smooth_a_template", "smooth_a_velocity", "gaussian_sum_isotropic",
           "gaussian_sum_anisotropic", "random_velocity", "config", "CONFIGS", "BATCH_SIZES", "batch_sizes",
           "batch_pair", "gaussian_sum_3d", "random_velocity_3d", "config_3d", "CONFIGS_3D"]


def grid_coords(n1, n2):
    x1 = 2.0 * math.pi * np.arange(n1) / n1
    x2 = 2.0 * math.pi * np.arange(n2) / n2
    return np.meshgrid(x1, x2, indexing="ij")


def _wrap(d):
    """Minimum-image difference on the 2*pi-periodic line."""
    return (d + math.pi) % (2.0 * math.pi) - math.pi


def smooth_a_template(n1, n2):
    """m_T = (sin^2 x1 + sin^2 x2) / 2."""
    X1, X2 = grid_coords(n1, n2)
    return 0.5 * (np.sin(X1) ** 2 + np.sin(X2) ** 2)


def smooth_a_velocity(n1, n2, amplitude=0.5):
    """v* = amplitude * (sin x2 cos x1, -sin x1 cos x2): divergence free, -Laplacian v* = 2 v*."""
    X1, X2 = grid_coords(n1, n2)
    return amplitude * np.stack([np.sin(X2) * np.cos(X1), -np.sin(X1) * np.cos(X2)])


def _normalise(u):
    lo, hi = float(u.min()), float(u.max())
    return (u - lo) / (hi - lo)


def gaussian_sum_isotropic(n1, n2, rng, count=32, sigma=(0.1, 0.4), amplitude=(0.2, 1.0)):
    """Sum of isotropic periodic Gaussians (widths in radians), min-max normalised to [0, 1]."""
    x1 = 2.0 * math.pi * np.arange(n1) / n1
    x2 = 2.0 * math.pi * np.arange(n2) / n2
    centres = rng.uniform(0.0, 2.0 * math.pi, size=(count, 2))
    sig = rng.uniform(sigma[0], sigma[1], size=count)
    amp = rng.uniform(amplitude[0], amplitude[1], size=count)
    # an isotropic Gaussian is the outer product of two 1-D Gaussians: the sum is one product of
    # the (count x n1) and (count x n2) factor matrices
    d1 = _wrap(x1[None, :] - centres[:, :1])
    d2 = _wrap(x2[None, :] - centres[:, 1:])
    inv = 1.0 / (2.0 * sig * sig)[:, None]
    u = (amp[:, None] * np.exp(-d1 * d1 * inv)).T @ np.exp(-d2 * d2 * inv)
    return _normalise(u)


def gaussian_sum_anisotropic(n1, n2, rng, count=64, sigma_px=(2.0, 20.0), amplitude=(0.0, 1.0),
                             smooth_px=2.0):
    """Brain-like stand-in: rotated anisotropic Gaussians, Gaussian-smoothed, clipped to [0, 1]."""
    X1, X2 = grid_coords(n1, n2)
    h1, h2 = 2.0 * math.pi / n1, 2.0 * math.pi / n2
    centres = rng.uniform(0.0, 2.0 * math.pi, size=(count, 2))
    sig = rng.uniform(sigma_px[0], sigma_px[1], size=(count, 2))
    rot = rng.uniform(0.0, math.pi, size=count)
    amp = rng.uniform(amplitude[0], amplitude[1], size=count)
    u = np.zeros((n1, n2))
    for c, s, r, a in zip(centres, sig, rot, amp):
        d1 = _wrap(X1 - c[0]) / h1; d2 = _wrap(X2 - c[1]) / h2   # in pixels
        p = math.cos(r) * d1 + math.sin(r) * d2
        q = -math.sin(r) * d1 + math.cos(r) * d2
        u += a * np.exp(-0.5 * ((p / s[0]) ** 2 + (q / s[1]) ** 2))
    k1 = np.fft.fftfreq(n1, 1.0 / n1); k2 = np.fft.fftfreq(n2, 1.0 / n2)
    K1, K2 = np.meshgrid(k1, k2, indexing="ij")
    s1, s2 = smooth_px * h1, smooth_px * h2
    u = np.fft.ifft2(np.fft.fft2(u) * np.exp(-0.5 * ((K1 * s1) ** 2 + (K2 * s2) ** 2))).real
    return np.clip(u, 0.0, 1.0)


def random_velocity(n1, n2, rng, modes=16, kmax=4, amplitude=0.3):
    """Smooth periodic velocity from 'modes' random Fourier modes with 1 <= |k| <= kmax.

    Wavevectors are drawn without replacement from the integer lattice
    points in that annulus; each carries a complex 2-vector with standard
    normal real and imaginary parts; the field is rescaled so that
    max_{x,i} |v_i(x)| equals 'amplitude'.
    """
    cand = [(a, b) for a in range(-kmax, kmax + 1) for b in range(-kmax, kmax + 1)
            if 1 <= a * a + b * b <= kmax * kmax]
    pick = rng.choice(len(cand), size=modes, replace=False)
    x1 = 2.0 * math.pi * np.arange(n1) / n1
    x2 = 2.0 * math.pi * np.arange(n2) / n2
    coefs = []
    for _ in pick:
        coefs.append(rng.standard_normal(2) + 1j * rng.standard_normal(2))
    coefs = np.array(coefs)                       # [modes, 2]
    k = np.array([cand[i] for i in pick])         # [modes, 2]
    e1 = np.exp(1j * k[:, :1] * x1[None, :])      # the plane wave factorises: [modes, n1]
    e2 = np.exp(1j * k[:, 1:] * x2[None, :])      # [modes, n2]
    v = np.stack([((coefs[:, c:c + 1] * e1).T @ e2).real for c in range(2)])
    return v * (amplitude / float(np.max(np.abs(v))))


def random_solenoidal_velocity(n1, n2, rng, modes=16, kmax=4, amplitude=0.3):
    """Smooth periodic divergence-free velocity v = (d2 psi, -d1 psi) of a stream function psi
    with 'modes' random Fourier modes, 1 <= |k| <= kmax (drawn as in random_velocity, one
    complex coefficient per mode), rescaled so that max_{x,i} |v_i(x)| equals 'amplitude'."""
    cand = [(a, b) for a in range(-kmax, kmax + 1) for b in range(-kmax, kmax + 1)
            if 1 <= a * a + b * b <= kmax * kmax]
    pick = rng.choice(len(cand), size=modes, replace=False)
    x1 = 2.0 * math.pi * np.arange(n1) / n1
    x2 = 2.0 * math.pi * np.arange(n2) / n2
    coefs = np.array([rng.standard_normal() + 1j * rng.standard_normal() for _ in pick])
    k = np.array([cand[i] for i in pick])
    e1 = np.exp(1j * k[:, :1] * x1[None, :])
    e2 = np.exp(1j * k[:, 1:] * x2[None, :])
    # d2 of c e^{i k.x} is i k2 c e^{i k.x}; d1 likewise
    w1 = (1j * k[:, 1] * coefs)[:, None]
    w2 = (-1j * k[:, 0] * coefs)[:, None]
    v = np.stack([((w1 * e1).T @ e2).real, ((w2 * e1).T @ e2).real])
    return v * (amplitude / float(np.max(np.abs(v))))


CONFIGS = {
    # name: grid, nt, regulariser order, beta, preconditioner, image recipe, velocity recipe, seed
    "smooth64": dict(n1=64, n2=64, nt=4, reg=1, beta=1e-2, pc="reg", prec="fp64"),
    "gauss256": dict(n1=256, n2=256, nt=4, reg=2, beta=1e-3, pc="2l", prec="mixed", seed=2),
    "brain512": dict(n1=512, n2=512, nt=8, reg=1, beta=1e-3, pc="2l", prec="mixed", seed=3),
    "brain512ic": dict(n1=512, n2=512, nt=8, reg=1, beta=1e-3, pc="2l", prec="mixed", seed=3, proj="leray"),
}


def config(name, n=None, seed=None):
    """Inputs of one named problem: dict with sizes, parameters, m_T, v_gen and a direction vt.

    'smooth64': the smooth analytic pair (m_T, v*) on 64^2 (or n^2).
    'gauss256': 32 isotropic Gaussians, 16-mode velocity |k| <= 4, amplitude 0.3.
    'brain512': 64 anisotropic smoothed Gaussians, 24-mode velocity |k| <= 6,
                amplitude 0.5.
    'brain512ic': the same image with a divergence-free 24-mode velocity (stream
                function modes |k| <= 6), amplitude 0.5, for the incompressible case.
    The direction vt (for Hessian matvecs) is a 16-mode |k| <= 4 field of
    amplitude 0.1 from the seed + 1000 stream.
    """
    c = dict(CONFIGS[name])
    if n is not None:
        c["n1"] = c["n2"] = int(n)
    n1, n2 = c["n1"], c["n2"]
    s = c.get("seed", 1) if seed is None else seed
    rng = np.random.default_rng(s)
    if name == "smooth64":
        c["mT"] = smooth_a_template(n1, n2)
        c["v_gen"] = smooth_a_velocity(n1, n2)
    elif name == "gauss256":
        c["mT"] = gaussian_sum_isotropic(n1, n2, rng)
        c["v_gen"] = random_velocity(n1, n2, rng, modes=16, kmax=4, amplitude=0.3)
    elif name == "brain512":
        c["mT"] = gaussian_sum_anisotropic(n1, n2, rng)
        c["v_gen"] = random_velocity(n1, n2, rng, modes=24, kmax=6, amplitude=0.5)
    elif name == "brain512ic":
        c["mT"] = gaussian_sum_anisotropic(n1, n2, rng)
        c["v_gen"] = random_solenoidal_velocity(n1, n2, rng, modes=24, kmax=6, amplitude=0.5)
    else:
        raise KeyError(name)
    rng_t = np.random.default_rng(s + 1000)
    c["vt"] = random_velocity(n1, n2, rng_t, modes=16, kmax=4, amplitude=0.1)
    return c


# Grid sizes of the batched workload: 64 independent pairs, sizes drawn (seed 4) from these.
BATCH_SIZES = (128, 256, 384, 512, 768, 1024)


def batch_sizes(count=64, seed=4):
    """Grid size n (n x n) of each pair of the batched workload, drawn uniformly from BATCH_SIZES."""
    rng = np.random.default_rng(seed)
    return [int(BATCH_SIZES[i]) for i in rng.integers(0, len(BATCH_SIZES), size=count)]


def batch_pair(p, n):
    """Pair p of the batched workload on an n x n grid: the 'gauss256' recipe (32 isotropic
    Gaussians, 16-mode velocity |k| <= 4, amplitude 0.3) from the stream seeded 4000 + p."""
    return config("gauss256", n=n, seed=4000 + p)


# ---------------------------------------------------------------------------
# Three-dimensional recipes (the same families on [0, 2 pi)^3)
# ---------------------------------------------------------------------------

def gaussian_sum_3d(n1, n2, n3, rng, count=32, sigma=(0.2, 0.5), amplitude=(0.2, 1.0)):
    """Sum of isotropic periodic 3-D Gaussians (widths in radians), min-max normalised to [0, 1]."""
    xs = [2.0 * math.pi * np.arange(n) / n for n in (n1, n2, n3)]
    centres = rng.uniform(0.0, 2.0 * math.pi, size=(count, 3))
    sig = rng.uniform(sigma[0], sigma[1], size=count)
    amp = rng.uniform(amplitude[0], amplitude[1], size=count)
    inv = 1.0 / (2.0 * sig * sig)
    u = np.zeros((n1, n2, n3))
    for c in range(count):
        f = [np.exp(-_wrap(x - centres[c, i]) ** 2 * inv[c]) for i, x in enumerate(xs)]
        u += amp[c] * f[0][:, None, None] * f[1][None, :, None] * f[2][None, None, :]
    return _normalise(u)


def random_velocity_3d(n1, n2, n3, rng, modes=16, kmax=3, amplitude=0.3):
    """Smooth periodic 3-D velocity from 'modes' random Fourier modes with 1 <= |k| <= kmax
    (lattice points drawn without replacement, complex 3-vector coefficients with standard
    normal parts), rescaled so that max_{x,i} |v_i(x)| equals 'amplitude'."""
    cand = [(a, b, c) for a in range(-kmax, kmax + 1) for b in range(-kmax, kmax + 1)
            for c in range(-kmax, kmax + 1) if 1 <= a * a + b * b + c * c <= kmax * kmax]
    pick = rng.choice(len(cand), size=modes, replace=False)
    xs = [2.0 * math.pi * np.arange(n) / n for n in (n1, n2, n3)]
    v = np.zeros((3, n1, n2, n3))
    for i in pick:
        k = cand[i]
        coef = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        wave = (np.exp(1j * k[0] * xs[0])[:, None, None] * np.exp(1j * k[1] * xs[1])[None, :, None]
                * np.exp(1j * k[2] * xs[2])[None, None, :])
        for c in range(3):
            v[c] += (coef[c] * wave).real
    return v * (amplitude / float(np.max(np.abs(v))))


# name -> (n, nt, beta, reg, template count, velocity amplitude, seed): volumes of the 2-D
# recipes' kind (periodic Gaussian blobs moved by a smooth velocity)
CONFIGS_3D = {
    "gauss3d_small": (32, 4, 1e-3, 2, 12, 0.4, 21),
    "gauss3d128": (128, 4, 1e-3, 2, 32, 0.4, 22),
}


def config_3d(name, n=None, seed=None):
    """(mT, v_gen, nt, beta, reg) of a named 3-D recipe; m_R is mT transported by v_gen."""
    n0, nt, beta, reg, count, amp, s0 = CONFIGS_3D[name]
    n = n0 if n is None else n
    rng = np.random.default_rng(s0 if seed is None else seed)
    mT = gaussian_sum_3d(n, n, n, rng, count=count)
    v = random_velocity_3d(n, n, n, rng, amplitude=amp)
    return mT, v, nt, beta, reg
