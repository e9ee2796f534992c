"""GPU parity of the learned warm start's network (BF16 MFMA kernels, through the C ABI) against
the FP64 reference with BF16 rounding mirrored (oracle/unet_oracle.py), and of the warm-started
solve with its fallback."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import synth
from oracle import unet_oracle as U
from gpu_common import problem, record

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slnk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1604_02153_amd as pkg
    pkg.load_library()
    return pkg


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _case(seed, B=2, n=64):
    rng = np.random.default_rng(seed)
    mR = np.stack([synth.gaussian_sum_isotropic(n, n, rng) for _ in range(B)]).astype(np.float32)
    mT = np.stack([synth.gaussian_sum_isotropic(n, n, rng) for _ in range(B)]).astype(np.float32)
    tgt = np.stack([synth.random_velocity(n, n, rng, amplitude=0.3) for _ in range(B)]).astype(np.float32)
    return mR, mT, tgt


def _net(slnk, arch, params, B=2):
    net = slnk.UNet(arch.H, arch.W, arch.L, arch.base, max_batch=B)
    assert net.n_params == arch.n
    net.set_params(params.astype(np.float32))
    return net


@pytest.mark.parametrize("shape", [(64, 64, 3), (64, 128, 4), (32, 32, 3)])
def test_forward_matches_reference(slnk, shape):
    H, W, L = shape
    arch = U.Arch(H, W, levels=L, base=32)
    rng = np.random.default_rng(1)
    params = U.random_params(arch, rng)
    params[arch.hw_off: arch.hw_off + 2 * arch.C[-1]] = 0.1 * rng.standard_normal(2 * arch.C[-1])
    params[arch.hb_off] = 0.3
    params = params.astype(np.float32).astype(np.float64)
    net = _net(slnk, arch, params)
    mR, mT, _ = _case(2, n=H)
    if W != H:
        mR, mT = np.concatenate([mR, mR], axis=2), np.concatenate([mT, mT[:, ::-1]], axis=2)
    v = torch.empty((2, 2, H, W), dtype=torch.float32, device="cuda")
    head = torch.empty((2,), dtype=torch.float32, device="cuda")
    slnk.UNet.conv_variant_counts(reset=True)
    net.forward(_t(mR), _t(mT), v, head)
    counts = slnk.UNet.conv_variant_counts()
    if H == 32:  # coarsest level 8 x 8 = 64 pixels: output tiles of 16 pixels
        assert counts[(16, 4)] > 0, counts
    v_ref, cache = U.forward(arch, params, mR, mT, bf16=True)
    err = rel(v.cpu().numpy(), v_ref)
    print(f"forward rel err {err:.2e}", flush=True)
    assert err < 1e-2
    # the head reads the coarsest BF16 activations through per-channel maxima: one rounding flip
    # of an activation (one BF16 unit, 2^-8 relative), which the GPU's FP32 accumulation order can
    # cause where the reference's FP64 sums round the other way, moves a maximum by that much
    assert rel(head.cpu().numpy(), cache["head"]) < 2.0 ** -8
    net.close()


@pytest.mark.parametrize("n", [64, 32])
def test_gradients_match_reference(slnk, n):
    arch = U.Arch(n, n, levels=3, base=32)
    params = U.random_params(arch, np.random.default_rng(3)).astype(np.float32).astype(np.float64)
    net = _net(slnk, arch, params)
    mR, mT, tgt = _case(4, n=n)
    loss = net.train_step(_t(mR), _t(mT), _t(tgt), 0.0)
    g = net.get_grads().astype(np.float64)[: arch.trunk_n]
    v_ref, cache = U.forward(arch, params, mR, mT, bf16=True)
    l_ref, dv = U.mse(v_ref, tgt)
    g_ref = U.backward(arch, cache, dv, bf16=True)[: arch.trunk_n]
    assert abs(loss - l_ref) / l_ref < 1e-3
    errs = []
    for k, ly in enumerate(arch.layers):
        nw = 9 * ly["cout"] * ly["cin"]
        ew = rel(g[ly["woff"]: ly["woff"] + nw], g_ref[ly["woff"]: ly["woff"] + nw])
        eb = rel(g[ly["boff"]: ly["boff"] + ly["cout"]], g_ref[ly["boff"]: ly["boff"] + ly["cout"]])
        errs.append((k, ew, eb))
    print("per-layer grad rel err", [(k, f"{a:.1e}", f"{b:.1e}") for k, a, b in errs], flush=True)
    assert all(ew < 3e-2 and eb < 3e-2 for _, ew, eb in errs)
    assert rel(g, g_ref) < 1e-2
    net.close()


def _shipped(slnk, max_batch):
    import os
    path = os.path.join(os.path.dirname(slnk.__file__), "weights", "unet_gauss256.bin")
    net = slnk.UNet(256, 256, 4, 32, max_batch=max_batch, start_kmax=8)
    net.load(path)
    return net, U.Arch(256, 256, levels=4, base=32), net.get_params().astype(np.float64)


def test_shipped_network_forward_matches_reference(slnk):
    """The shipped 256^2, 4-level, 32-channel network at batch 1 (the learned solve's forward):
    output velocity and head against the reference.  Its launches take the LDS-tiled kernel
    (65536-pixel level, 32 channels per block) and the direct kernel with 32-pixel output tiles and
    the channel reduction split 2 (128^2 level) and 4 ways (the two coarsest levels)."""
    from paper_1604_02153_amd.train_unet import make_pair
    net, arch, params = _shipped(slnk, 1)
    assert arch.n == net.n_params
    mT, vg = make_pair(200100)
    import oracle as O
    mR = O.transport_state(O.Grid(256, 256), vg.astype(np.float64), mT.astype(np.float64), 4)
    mR, mT = mR[None].astype(np.float32), mT[None].astype(np.float32)
    v = torch.empty((1, 2, 256, 256), dtype=torch.float32, device="cuda")
    head = torch.empty((1,), dtype=torch.float32, device="cuda")
    slnk.UNet.conv_variant_counts(reset=True)
    net.forward(_t(mR), _t(mT), v, head)
    counts = slnk.UNet.conv_variant_counts()
    print("variants", counts, flush=True)
    assert counts[("lds", 32)] > 0 and counts[(32, 2)] > 0 and counts[(32, 4)] > 0, counts
    v_ref, cache = U.forward(arch, params, mR, mT, bf16=True)
    err = rel(v.cpu().numpy(), v_ref)
    record("U-Net 256^2 forward (shipped weights)", err, 1e-2)
    assert err < 1e-2
    eh = rel(head.cpu().numpy(), cache["head"])
    record("U-Net 256^2 head (shipped weights)", eh, 2.0 ** -8)
    assert eh < 2.0 ** -8
    net.close()


def test_shipped_network_gradients_match_reference(slnk):
    """A training step of the shipped 256^2 network at batch 2 (lr 0): the loss and every layer's
    weight and bias gradients against the reference.  The weight gradients of the 256^2 level sum
    64 pixel chunks; the forward and input-gradient launches take the LDS-tiled kernel on the two
    finest levels (32 and 64 channels per block) and the direct kernel below."""
    from paper_1604_02153_amd.train_unet import make_pair
    import oracle as O
    net, arch, params = _shipped(slnk, 2)
    mRs, mTs, tgts = [], [], []
    for s in (200200, 200201):
        mT, vg = make_pair(s)
        mRs.append(O.transport_state(O.Grid(256, 256), vg.astype(np.float64), mT.astype(np.float64), 4))
        mTs.append(mT)
        tgts.append(vg)
    mR, mT, tgt = (np.stack(a).astype(np.float32) for a in (mRs, mTs, tgts))
    slnk.UNet.conv_variant_counts(reset=True)
    loss = net.train_step(_t(mR), _t(mT), _t(tgt), 0.0)
    counts = slnk.UNet.conv_variant_counts()
    print("variants", counts, flush=True)
    assert counts[("lds", 32)] > 0 and counts[("lds", 64)] > 0 and counts[(32, 2)] > 0, counts
    g = net.get_grads().astype(np.float64)[: arch.trunk_n]
    v_ref, cache = U.forward(arch, params, mR, mT, bf16=True)
    l_ref, dv = U.mse(v_ref, tgt)
    g_ref = U.backward(arch, cache, dv, bf16=True)[: arch.trunk_n]
    assert abs(loss - l_ref) / l_ref < 1e-3
    worst = 0.0
    for k, ly in enumerate(arch.layers):
        nw = 9 * ly["cout"] * ly["cin"]
        ew = rel(g[ly["woff"]: ly["woff"] + nw], g_ref[ly["woff"]: ly["woff"] + nw])
        eb = rel(g[ly["boff"]: ly["boff"] + ly["cout"]], g_ref[ly["boff"]: ly["boff"] + ly["cout"]])
        print(f"layer {k}: weight grad {ew:.2e}, bias grad {eb:.2e}", flush=True)
        worst = max(worst, ew, eb)
    record("U-Net 256^2 per-layer gradients, worst (shipped weights)", worst, 3e-2)
    assert worst < 3e-2
    eg = rel(g, g_ref)
    record("U-Net 256^2 all gradients (shipped weights)", eg, 1e-2)
    assert eg < 1e-2
    net.close()


def test_head_gradients_match_reference(slnk):
    """The scalar head trains alone: its gradient matches the reference and the convolution
    layers receive none (their parameters stay put under a head-only Adam step)."""
    arch = U.Arch(64, 64, levels=3, base=32)
    rng = np.random.default_rng(9)
    params = U.random_params(arch, rng).astype(np.float32).astype(np.float64)
    params[arch.hw_off: arch.hw_off + 2 * arch.C[-1]] = 0.1 * rng.standard_normal(2 * arch.C[-1])
    params = params.astype(np.float32).astype(np.float64)
    net = _net(slnk, arch, params)
    mR, mT, _ = _case(10)
    y = np.array([0.5, -1.0], dtype=np.float32)
    _, hl = net.train_step(_t(mR), _t(mT), None, 1e-3, head_target=_t(y))
    g = net.get_grads().astype(np.float64)
    _, cache = U.forward(arch, params, mR, mT, bf16=True)
    l_ref, g_ref = U.head_grad(arch, cache, y)
    assert abs(hl - l_ref) / l_ref < 1e-3
    sl = slice(arch.hw_off, arch.n)
    # the features are BF16 activations: an FP32 (GPU) and an FP64 (reference) sum upstream can
    # round a value to neighbouring BF16 numbers (2^-8 apart), which the maxima pass on unaveraged
    assert rel(g[sl], g_ref[sl]) < 5e-3
    after = net.get_params().astype(np.float64)
    assert np.array_equal(after[: arch.trunk_n], params[: arch.trunk_n])
    net.close()


def test_adam_step_matches_reference(slnk):
    arch = U.Arch(64, 64, levels=3, base=32)
    params = U.random_params(arch, np.random.default_rng(5)).astype(np.float32).astype(np.float64)
    net = _net(slnk, arch, params)
    mR, mT, tgt = _case(6)
    net.train_step(_t(mR), _t(mT), _t(tgt), 1e-3)
    n = arch.trunk_n
    g = net.get_grads().astype(np.float64)[:n]
    w1, _, _ = U.adam_step(params[:n], g, np.zeros_like(g), np.zeros_like(g), 1, lr=1e-3)
    got = net.get_params().astype(np.float64)
    assert np.max(np.abs(got[:n] - w1)) < 1e-6
    assert np.array_equal(got[n:], params[n:])  # the head is not touched by the velocity loss
    net.close()


def test_training_fits_a_learnable_target(slnk):
    """Adam on a fixed batch whose target is a local function of the input (0.3 (m_R - m_T),
    0.3 m_T) drives the loss down by an order of magnitude."""
    net = slnk.UNet(64, 64, 3, 32, max_batch=4, seed=7)
    mR, mT, _ = _case(8, B=4)
    tgt = 0.3 * np.stack([mR - mT, mT], axis=1)
    mR, mT, tgt = _t(mR), _t(mT), _t(tgt)
    losses = [net.train_step(mR, mT, tgt, 2e-3) for _ in range(80)]
    print("losses", [f"{x:.3e}" for x in losses[::10]], flush=True)
    assert losses[-1] < 0.1 * losses[0]
    net.close()


def test_bad_start_falls_back_to_zero(slnk):
    """A start whose gradient is larger than at v = 0 is replaced by v = 0: the solve then takes
    exactly the cold-start path."""
    n = 64
    L, vgen, _ = problem("smooth", n, n, nt=4, beta=1e-2, reg=1)
    ctx = slnk.Context(n, n, 4, reg="h1", beta=1e-2, prec="fp64", pc="reg")
    ctx.set_images(torch.from_numpy(L.mR).cuda(), torch.from_numpy(L.mT).cuda())
    v0 = torch.zeros((2, n, n), dtype=torch.float64, device="cuda")
    cold = ctx.newton_solve(v0)
    vb = torch.from_numpy(-6.0 * vgen).cuda()
    warm = ctx.newton_solve(vb)
    assert warm["fallback"] and not cold["fallback"]
    for key in ("newton_iters", "pcg_iters", "grel", "J"):
        assert warm[key] == cold[key], key
    assert torch.equal(vb, v0)
    ctx.close()


def test_learned_solve_with_an_untrained_network(slnk):
    """The learned solve runs the network on the context's images and solves from its output; an
    untrained network's near-zero output is either kept or replaced, and the solve converges."""
    n = 64
    L, vgen, _ = problem("gauss", n, n, nt=4, beta=1e-3, reg=2, seed=21)
    mR, mT = L.mR.astype(np.float32), L.mT.astype(np.float32)
    ctx = slnk.Context(n, n, 4, reg="h2", beta=1e-3, prec="mixed", pc="2l", batch=2)
    ctx.set_images(_t(np.stack([mR, mR])), _t(np.stack([mT, mT])))
    net = slnk.UNet(n, n, 3, 32, max_batch=2)
    v = torch.empty((2, 2, n, n), dtype=torch.float32, device="cuda")
    reps = ctx.newton_solve_learned(net, v)
    v_net = torch.empty_like(v)
    net.forward(_t(np.stack([mR, mR])), _t(np.stack([mT, mT])), v_net)
    for r in reps:
        assert r["status"] == "SLNK_OK" and r["grel"][-1] <= 1e-2
    assert reps[0]["grel"] == reps[1]["grel"]
    net.close()
    ctx.close()


def test_learned_setup_takes_emax_from_the_head(slnk):
    """set_images_learned: e_max = 1 + 1.1 exp(head) / beta (no Lanczos), e_min unchanged; the
    learned solve then starts from the kept network output and converges."""
    n = 64
    L, vgen, _ = problem("gauss", n, n, nt=4, beta=1e-3, reg=2, seed=23)
    mR, mT = _t(L.mR[None]), _t(L.mT[None])
    net = slnk.UNet(n, n, 3, 32, max_batch=1)
    ctx = slnk.Context(n, n, 4, reg="h2", beta=1e-3, prec="mixed", pc="2l")
    ctx.set_images(mR[0], mT[0])
    emin, emax_lanczos = ctx.cheb_bounds()
    w = net.get_params()
    arch = U.Arch(n, n, levels=3, base=32)
    w[arch.hb_off] = np.log(1e-3 * (emax_lanczos - 1.0) / 1.1)   # head = that value (zero weights)
    net.set_params(w)
    ctx.set_images_learned(net, mR[0], mT[0])
    emin2, emax2 = ctx.cheb_bounds()
    assert emin2 == emin and abs(emax2 - emax_lanczos) / emax_lanczos < 1e-5
    v = torch.empty((2, n, n), dtype=torch.float32, device="cuda")
    r = ctx.newton_solve_learned(net, v)
    assert r["status"] == "SLNK_OK" and r["grel"][-1] <= 1e-2
    net.close()
    ctx.close()


def test_learned_emax_below_the_spectrum_is_reestimated(slnk):
    """A head that predicts e_max far below the Lanczos value (CHEB(10) indefinite): the learned
    solve detects it in PCG (r.z <= 0), re-estimates e_max by Lanczos and still converges."""
    n = 64
    L, vgen, _ = problem("gauss", n, n, nt=4, beta=1e-3, reg=2, seed=21)
    mR, mT = _t(L.mR[None]), _t(L.mT[None])
    net = slnk.UNet(n, n, 3, 32, max_batch=1)
    ctx = slnk.Context(n, n, 4, reg="h2", beta=1e-3, prec="mixed", pc="2l")
    ctx.set_images(mR[0], mT[0])
    emin, emax_lanczos = ctx.cheb_bounds()
    w = net.get_params()
    arch = U.Arch(n, n, levels=3, base=32)
    w[arch.hb_off] = np.log(1e-3 * 0.05 * (emax_lanczos - 1.0) / 1.1)   # e_max - 1 at 5% of Lanczos
    net.set_params(w)
    ctx.set_images_learned(net, mR[0], mT[0])
    assert ctx.cheb_bounds()[1] < 1.0 + 0.06 * (emax_lanczos - 1.0)
    v = torch.empty((2, n, n), dtype=torch.float32, device="cuda")
    r = ctx.newton_solve_learned(net, v)
    print(r["grel"], r["pcg"], r["cheb_reestimates"], flush=True)
    assert r["cheb_reestimates"] >= 1
    assert r["status"] == "SLNK_OK" and r["grel"][-1] <= 1e-2
    net.close()
    ctx.close()


def test_trained_network_saves_newton_work(slnk):
    """The shipped trained network (weights/unet_gauss256.bin) on 8 held-out gauss256 pairs (seeds
    200000..200007, outside its training seeds): every learned solve keeps the network's start and
    reaches ||g||rel <= 1e-2, and together they need fewer Newton iterations and fewer fine GN
    matvecs than the plain solves of the same pairs (the counts, not the wall times, which the
    benchmark reports)."""
    import os
    from paper_1604_02153_amd.train_unet import make_pair
    path = os.path.join(os.path.dirname(slnk.__file__), "weights", "unet_gauss256.bin")
    n = 256
    net = slnk.UNet(n, n, 4, 32, max_batch=1, start_kmax=8)
    net.load(path)
    ctx = slnk.Context(n, n, 4, reg="h2", beta=1e-3, prec="mixed", pc="2l")
    v = torch.zeros((2, n, n), dtype=torch.float32, device="cuda")
    plain_newton = learned_newton = plain_mv = learned_mv = 0
    for s in range(200000, 200008):
        mT, vg = make_pair(s)
        mT, vg = _t(mT), _t(vg)
        mR = torch.empty_like(mT)
        ctx.transport_state(vg, mT, mR)
        ctx.set_images(mR, mT)
        v.zero_()
        p = ctx.newton_solve(v)
        ctx.set_images_learned(net, mR, mT)
        q = ctx.newton_solve_learned(net, v)
        print(s, p["newton_iters"], p["matvecs"], q["newton_iters"], q["matvecs"], q["fallback"], flush=True)
        assert p["grel"][-1] <= 1e-2 and q["grel"][-1] <= 1e-2
        assert q["status"] == "SLNK_OK" and not q["fallback"]
        plain_newton += p["newton_iters"]
        learned_newton += q["newton_iters"]
        plain_mv += p["matvecs"]
        learned_mv += q["matvecs"]
    assert learned_newton < plain_newton and learned_mv < plain_mv
    net.close()
    ctx.close()
