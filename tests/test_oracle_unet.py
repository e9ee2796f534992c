"""Pins of the network reference (oracle/unet_oracle.py): BF16 rounding against torch's cast,
the periodic convolution against scipy's wrap-mode correlation, adjoint identities of pooling and
upsampling, hand-written backpropagation against central finite differences, and Adam's first
step against its closed form."""

import numpy as np
import pytest
from scipy import ndimage

from oracle import unet_oracle as U


def test_bf16_round_ties_to_even_and_matches_torch():
    one = 1.0
    assert U.bf16_round(one + 2.0 ** -8) == 1.0              # halfway, even neighbour below
    assert U.bf16_round(one + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6  # halfway, even neighbour above
    assert U.bf16_round(one + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    torch = pytest.importorskip("torch")
    x = np.random.default_rng(0).standard_normal(10000) * 10.0 ** np.random.default_rng(1).integers(-5, 5, 10000)
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(U.bf16_round(x.astype(np.float32)), ref)


def test_conv3x3_is_wrap_mode_correlation():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 7, 9, 3))
    w = rng.standard_normal((9, 4, 3))
    b = rng.standard_normal(4)
    y = U.conv3x3(x, w, b)
    for bi in range(2):
        for o in range(4):
            ref = b[o] + sum(ndimage.correlate(x[bi, :, :, c], w[:, o, c].reshape(3, 3), mode="wrap")
                             for c in range(3))
            assert np.allclose(y[bi, :, :, o], ref, rtol=0, atol=1e-12)


def test_pool_and_upsampling_adjoints():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 8, 6, 3))
    yl = rng.standard_normal((2, 4, 3, 3))
    assert np.isclose(np.sum(U.pool(x) * yl), np.sum(x * U.pool_backward(yl)), rtol=1e-13)
    assert np.isclose(np.sum(U.up(yl) * x), np.sum(yl * U.up_backward(x)), rtol=1e-13)
    assert np.allclose(U.pool(U.up(yl)), yl)


def test_conv3x3_backward_against_finite_differences():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((1, 5, 6, 2))
    w = rng.standard_normal((9, 3, 2))
    b = rng.standard_normal(3)
    g = rng.standard_normal((1, 5, 6, 3))
    dx, dw, db = U.conv3x3_backward(x, w, g)
    f = lambda x_, w_, b_: np.sum(g * U.conv3x3(x_, w_, b_))
    h = 1e-6
    for d_x, d_w, d_b in [(rng.standard_normal(x.shape), 0, 0), (0, rng.standard_normal(w.shape), 0),
                          (0, 0, rng.standard_normal(b.shape))]:
        fd = (f(x + h * d_x, w + h * d_w, b + h * d_b) - f(x - h * d_x, w - h * d_w, b - h * d_b)) / (2 * h)
        an = np.sum(dx * d_x) + np.sum(dw * d_w) + np.sum(db * d_b)
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))


@pytest.mark.parametrize("levels", [2, 3])
def test_network_gradient_against_finite_differences(levels):
    """Whole network + MSE in FP64: the backpropagated gradient along random directions equals
    the central difference of the loss (a dropped term, a wrong skip or index would not)."""
    arch = U.Arch(8, 8, levels=levels, base=2, in_c=3, out_c=2)
    rng = np.random.default_rng(5 + levels)
    params = U.random_params(arch, rng, scale=1.5)
    mR = rng.uniform(0, 1, (2, 8, 8))
    mT = rng.uniform(0, 1, (2, 8, 8))
    tgt = 0.3 * rng.standard_normal((2, 2, 8, 8))

    def loss(p):
        v, _ = U.forward(arch, p, mR, mT)
        return U.mse(v, tgt)[0]

    v, cache = U.forward(arch, params, mR, mT)
    _, dv = U.mse(v, tgt)
    g = U.backward(arch, cache, dv)
    h = 1e-6
    for _ in range(6):
        d = rng.standard_normal(arch.n)
        fd = (loss(params + h * d) - loss(params - h * d)) / (2 * h)
        assert abs(fd - g @ d) <= 1e-6 * max(abs(fd), 1e-3)
    # per-layer check on a single coordinate of each layer's weights and bias
    for ly in arch.layers:
        for off in (ly["woff"], ly["boff"]):
            e = np.zeros(arch.n)
            e[off] = 1.0
            fd = (loss(params + h * e) - loss(params - h * e)) / (2 * h)
            assert abs(fd - g[off]) <= 1e-6 * max(abs(fd), 1e-4)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(7)
    w, g = rng.standard_normal(50), rng.standard_normal(50)
    w1, m1, v1 = U.adam_step(w, g, np.zeros(50), np.zeros(50), 1, lr=1e-3)
    assert np.allclose(w1, w - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)


def test_layout_matches_the_documented_parameter_count():
    arch = U.Arch(256, 256, levels=4, base=32)
    assert len(arch.layers) == 2 * 4 + 2 * 3 + 1
    n = 0
    for ly in arch.layers:
        assert ly["woff"] == n and ly["boff"] == n + U._pad64(9 * ly["cout"] * ly["cin"])
        n = ly["boff"] + U._pad64(ly["cout"])
    assert n == arch.trunk_n == arch.hw_off and arch.hb_off == n + 512 and arch.n == n + 512 + 64


def test_head_gradient_against_finite_differences():
    arch = U.Arch(8, 8, levels=2, base=2, in_c=3, out_c=2)
    rng = np.random.default_rng(11)
    params = U.random_params(arch, rng, scale=1.5)
    params[arch.hw_off: arch.hw_off + 2 * arch.C[-1]] = rng.standard_normal(2 * arch.C[-1])
    mR, mT = rng.uniform(0, 1, (3, 8, 8)), rng.uniform(0, 1, (3, 8, 8))
    y = rng.standard_normal(3)

    def loss(p):
        _, c = U.forward(arch, p, mR, mT)
        return U.head_grad(arch, c, y)[0]

    _, cache = U.forward(arch, params, mR, mT)
    l0, g = U.head_grad(arch, cache, y)
    assert np.all(g[: arch.trunk_n] == 0)
    h = 1e-6
    for off in list(range(arch.hw_off, arch.hw_off + 2 * arch.C[-1])) + [arch.hb_off]:
        e = np.zeros(arch.n)
        e[off] = 1.0
        fd = (loss(params + h * e) - loss(params - h * e)) / (2 * h)
        assert abs(fd - g[off]) <= 1e-7 * max(1.0, abs(fd))
