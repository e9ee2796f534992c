"""The allocation-free state transport (slnk_transport_state_noalloc, through the C ABI) against the
context entry point slnk_transport_state on the same inputs: two calls in a row, the second on a
smaller grid, in FP32 (mixed) and FP64, both SL kernel paths; sizes beyond its scratch array are
refused."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from gpu_common import TOL, problem, rel, same_inputs

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


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
@pytest.mark.parametrize("path", [0, 1])
def test_noalloc_transport_matches_context_entry_point(slnk, prec, path):
    for (n1, n2, nt, seed) in ((128, 128, 4, 71), (96, 80, 3, 72)):   # second call: smaller grid
        print(f"noalloc {prec} path {path} {n1}x{n2} nt {nt}", flush=True)
        L, vgen, _ = problem("gauss", n1, n2, nt=nt, beta=1e-3, reg=2, seed=seed, amp=0.35)
        mT, vgen = same_inputs(prec, L.mT, vgen)
        v, m0 = _t(vgen, prec), _t(mT, prec)
        ctx = slnk.Context(n1, n2, nt, reg="h2", beta=1e-3, prec=prec, pc="reg", sl_path=path)
        ref = torch.empty_like(m0)
        ctx.transport_state(v, m0, ref)
        torch.cuda.synchronize()
        ctx.close()
        out = torch.full_like(m0, float("nan"))
        slnk.transport_state_noalloc(v, m0, out, nt, sl_path=path)
        torch.cuda.synchronize()
        got, want = out.double().cpu().numpy(), ref.double().cpu().numpy()
        assert np.isfinite(got).all()
        assert rel(got, want) < TOL[prec]["transport"], (n1, n2, rel(got, want))


def test_noalloc_batch_and_aliasing(slnk):
    """Three items in one call, m1 written over m0: each item equals its own context result."""
    n, nt, prec = 64, 4, "mixed"
    probs = [problem("gauss", n, n, nt=nt, beta=1e-3, reg=2, seed=80 + z, amp=0.2 + 0.1 * z) for z in range(3)]
    v = _t(np.stack([same_inputs(prec, p[1]) for p in probs]), prec)
    m = _t(np.stack([same_inputs(prec, p[0].mT) for p in probs]), prec)
    ctx = slnk.Context(n, n, nt, reg="h2", beta=1e-3, prec=prec, pc="reg", batch=3)
    ref = torch.empty_like(m)
    ctx.transport_state(v, m, ref)
    torch.cuda.synchronize()
    ctx.close()
    slnk.transport_state_noalloc(v, m, m, nt)      # in place
    torch.cuda.synchronize()
    for z in range(3):
        assert rel(m[z].double().cpu().numpy(), ref[z].double().cpu().numpy()) < TOL[prec]["transport"], z


def test_noalloc_rejects_sizes_beyond_its_scratch(slnk):
    n = 512
    v = torch.zeros((2, n, n), dtype=torch.float64, device="cuda")
    m = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    with pytest.raises(slnk.SlnkError) as e:
        slnk.transport_state_noalloc(v, m, m, 4)
    assert e.value.status == 1 and "scratch" in str(e.value)
