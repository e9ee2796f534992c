"""Benchmark of the semi-Lagrangian Gauss--Newton--Krylov hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload (the 256^2 problem the Hessian-matvec rate is quoted on): 32 isotropic Gaussians on a
256 x 256 periodic grid, m_R = m_T transported by a seeded 16-mode velocity (|k| <= 4, amplitude
0.3) over nt = 4 SL steps, H2 regularisation, beta = 1e-3, mixed precision (FP32 fields, FP64
reductions), two-level preconditioner (coarse 128^2, CHEB(10), 30-step Lanczos).

One step = the per-pair set-up (images, coarse problem, 30-step Lanczos for e_max) and one
Newton--Krylov solve from v = 0 until ||g||_inf / ||g_0||_inf <= 1e-2 (every stage of the path:
trace, state/adjoint/incremental transport, spectral operators, reductions, PCG, P_2L, Armijo line
search).  Inputs are resident on the GPU before the timed region.

value = Gauss--Newton Hessian matvecs per second at 256^2, back to back at the generating velocity
(the metric's first part); ms_per_step = wall time of one step (set-up + solve, the plain method's
time to ||g||_rel <= 1e-2; the learned-vs-plain section holds the metric's second part).  The same
line carries roofline entries (the incremental-adjoint SL step at 256^2 and at the 128^2 coarse
level, timed with HIP events on the library's stream, and the whole matvec), the all-FP64 GPU leg,
each result's error against the FP64 oracle, and the oracle timed on the host's cores.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# Algorithmic bytes per grid point of one incremental-adjoint SL step (FP32 fields), the per-step
# figure of the fused matvec's byte count (matvec_bytes): read the transported field (1), the
# adjoint displacements (2), the adjoint factor (1), grad m at the new level (2), read and write
# the time-integral accumulator (2 + 2), write the new field (1), and the prefilter's pass over
# the transported field (2; inside the fused kernel it runs from LDS).
INC_ADJ_FIELDS_PER_POINT = 13
COUNTERS_FILE = os.path.join(ROOT, "profiles", "sl_step_incadj_gauss256_counters.txt")
WEIGHTS = os.path.join(ROOT, "paper_1604_02153_amd", "weights", "unet_gauss256.bin")
BF16_MFMA_PEAK_TFLOPS = 2500.0  # MI355X dense BF16
# the step kernel's sources (the counters go stale when either changes)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1604_02153_amd", "csrc", f) for f in ("transport.hip", "common.hpp")]


def log(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--matvecs", type=int, default=200, help="isolated matvecs timed")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=8.0, help="length of the CPU oracle sample (s)")
    ap.add_argument("--no-batched", action="store_true", help="skip the 64-pair ragged batch workload")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned vs plain comparison")
    ap.add_argument("--no-brain", action="store_true", help="skip the 512^2 nt=8 single-pair workload")
    ap.add_argument("--no-full-newton", action="store_true", help="skip the full-Newton matvec workload")
    ap.add_argument("--learned-pairs", type=int, default=32, help="held-out pairs of the learned vs plain timing")
    ap.add_argument("--batched-matvecs", type=int, default=10, help="timed batched matvec calls (64 pairs each)")
    ap.add_argument("--brain-matvecs", type=int, default=100, help="timed matvecs of the 512^2 workload")
    ap.add_argument("--spectral", action="store_true",
                    help="spectral-pass probe: 20 two-field spectral scalings at 1024^2 x16, 256^2 x64 and 128^2 "
                         "x64 batches (for a kernel trace); no JSON line")
    ap.add_argument("--probe-coarse", action="store_true",
                    help="coarse-step probe: 200 incremental-adjoint SL steps of the 128^2 problem (the P_2L coarse "
                         "grid of the 256^2 workload) for a kernel trace; no JSON line")
    ap.add_argument("--no-3d", action="store_true", help="skip the 128^3 three-dimensional workload")
    ap.add_argument("--d3-matvecs", type=int, default=20, help="timed matvecs of the 128^3 workload")
    ap.add_argument("--probe-3d", action="store_true",
                    help="3-D probe: gradient and 20 Gauss-Newton matvecs of the 128^3 problem (mixed), for "
                         "rocprofv3")
    ap.add_argument("--probe", action="store_true",
                    help="counter probe: 20 incremental-adjoint SL steps of the 256^2 problem, then a plain "
                         "64 MiB elementwise kernel (the reference of the traffic counters); no JSON line")
    return ap.parse_args()


def probe():
    """Launch sequence profiled by the FETCH_SIZE / WRITE_SIZE counter runs."""
    import numpy as np
    import torch

    import synth
    from paper_1604_02153_amd import Context
    cfg = synth.config("gauss256")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=torch.float32)
    ctx = Context(256, 256, 4, reg="h2", beta=1e-3, prec="mixed", pc="2l")
    mT, vg = t(cfg["mT"]), t(cfg["v_gen"])
    mR = torch.empty_like(mT)
    ctx.transport_state(vg, mT, mR)
    ctx.set_images(mR, mT)
    g = torch.empty_like(vg)
    ctx.gradient(vg, g)
    print(f"incremental-adjoint step: {1e3 * ctx.time_kernel(3, 20):.2f} us per launch", flush=True)
    x = torch.ones(16 * 1024 * 1024, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.mul(x, 2.0, out=y)  # reads and writes 64 MiB
    torch.cuda.synchronize()
    ctx.close()


def coarse_probe():
    """Launch sequence of the coarse-step kernel trace: the gauss256 recipe on the 128^2 grid,
    linearised at its generating velocity, 200 incremental-adjoint SL steps."""
    import numpy as np
    import torch

    import synth
    from paper_1604_02153_amd import Context
    c = synth.config("gauss256", n=128)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=torch.float32)
    ctx = Context(128, 128, 4, reg="h2", beta=1e-3, prec="mixed", pc="reg")
    mT, vg = t(c["mT"]), t(c["v_gen"])
    mR = torch.empty_like(mT)
    ctx.transport_state(vg, mT, mR)
    ctx.set_images(mR, mT)
    g = torch.empty_like(vg)
    ctx.gradient(vg, g)
    print(f"128^2 incremental-adjoint step: {1e3 * ctx.time_kernel(3, 200):.2f} us per launch", flush=True)
    ctx.close()


def spectral_probe():
    """Launch sequence of the spectral-pass kernel trace: spec_scale (row pass, column pass with the
    symbol, inverse row pass) on two fields per item, batched."""
    import numpy as np
    import torch

    import synth
    from paper_1604_02153_amd import Context
    for n, B in [(1024, 16), (256, 64), (128, 64)]:
        cs = [synth.batch_pair(p, n) for p in range(B)]
        t = lambda a: torch.from_numpy(np.ascontiguousarray(np.stack(a))).to(device="cuda", dtype=torch.float32)
        mT, vg = t([c["mT"] for c in cs]), t([c["v_gen"] for c in cs])
        ctx = Context(n, n, 4, reg="h2", beta=1e-3, prec="mixed", pc="reg", batch=B, sl_path=1)
        mR = torch.empty_like(mT)
        ctx.transport_state(vg, mT, mR)
        ctx.set_images(mR, mT)
        g = torch.empty_like(vg)
        ctx.gradient(vg, g)
        print(f"{n}^2 x{B}: spectral scaling {1e3 * ctx.time_kernel(5, 20):.1f} us per call", flush=True)
        ctx.close()


def measured_traffic():
    """HBM bytes per launch of the incremental-adjoint step from the committed counter summary,
    or None if the kernel source changed since the counters were taken."""
    try:
        with open(COUNTERS_FILE) as f:
            kv = dict(line.split("=", 1) for line in f.read().splitlines() if "=" in line and not line.startswith("#"))
        sha = hashlib.sha256()
        for src in KERNEL_SOURCES:
            with open(src, "rb") as f:
                sha.update(f.read())
        h = sha.hexdigest()[:16]
        if kv.get("source_sha256_16", "").strip() != h:
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def matvec_bytes(n1, n2, nt, elem=4):
    """Algorithmic HBM bytes of one fused GN Hessian matvec: (23 nt + 32) fields of n1 n2 elements.
    Per incremental-state step 10 fields (gather 1, displacements 2, direction 2, grad m 2, write 1,
    prefilter 2), per incremental-adjoint step 13 (gather 1, displacements 2, gamma 1, write 1,
    prefilter 2, grad m 2, accumulator read + write 4), plus 32 fixed (first sources, two forward
    and two inverse real-FFT passes, the combine)."""
    return (23 * nt + 32) * n1 * n2 * elem


def fn_matvec_bytes(n1, n2, nt, elem=4):
    """Algorithmic HBM bytes of one full-Newton matvec: the GN matvec's (23 nt + 32) fields plus
    (38 nt + 18): lambda^j vt products 5 (nt + 1), their spectral divergences 9 (nt + 1), the
    interpolations of sigma^j 6 nt, the Heun sources 4 nt, the kept m~^j nt, their spectral
    gradients 9 nt, the source reads of the incremental adjoint nt, and lambda grad m~ into b~
    3 nt + 4."""
    return (61 * nt + 50) * n1 * n2 * elem


def full_newton(args, dev):
    """gauss256 with the full-Newton matvec: isolated matvec rate and Newton solves to
    ||g||rel <= 1e-2 and 1e-4 next to the Gauss-Newton solver on the same GPU."""
    import numpy as np
    import torch

    import synth
    from paper_1604_02153_amd import Context
    cfg = synth.config("gauss256")
    n1, n2, nt = cfg["n1"], cfg["n2"], cfg["nt"]
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=torch.float32)
    mT, vgen, vt = f32(cfg["mT"]), f32(cfg["v_gen"]), f32(cfg["vt"])
    out = {"workload": "gauss256 (256x256, nt=4, H2 beta=1e-3, P_2L mixed) with hessian = full Newton; "
                       "the coarse operator of P_2L stays Gauss-Newton"}
    for hess in ("gn", "fn"):
        ctx = Context(n1, n2, nt, reg="h2", beta=cfg["beta"], prec="mixed", pc="2l", hessian=hess)
        mR = torch.empty_like(mT)
        ctx.transport_state(vgen, mT, mR)
        ctx.set_images(mR, mT)
        v = torch.zeros_like(vgen)
        res = {}
        for gtol in (1e-2, 1e-4):
            v.zero_()
            ctx.newton_solve(v, gtol_rel=gtol, max_newton=20)  # warm-up (graph capture)
            v.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rep = ctx.newton_solve(v, gtol_rel=gtol, max_newton=20)
            torch.cuda.synchronize()
            res[f"solve_to_{gtol:g}"] = {"ms": round(1e3 * (time.perf_counter() - t0), 2), "status": rep["status"],
                                          "newton_iters": rep["newton_iters"], "pcg_iters": rep["pcg_iters"],
                                          "grel": [float(f"{x:.3g}") for x in rep["grel"]]}
        if hess == "fn":
            g = torch.empty_like(v)
            ctx.gradient(0.6 * vgen, g)
            h = torch.empty_like(v)
            for _ in range(10):
                ctx.hessian_matvec(vt, h)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(args.matvecs // 2):
                ctx.hessian_matvec(vt, h)
            torch.cuda.synchronize()
            rate = (args.matvecs // 2) / (time.perf_counter() - t1)
            gbs = fn_matvec_bytes(n1, n2, nt) * rate / 1e9
            res.update({"isolated_matvecs_per_s": round(rate, 1), "matvec_GBps_algorithmic": round(gbs, 1),
                        "matvec_roofline_frac": round(gbs / HBM_PEAK_GBS, 4)})
        out["gauss_newton" if hess == "gn" else "full_newton"] = res
        ctx.close()
    return out


def preconditioners(args, dev):
    """gauss256 Newton solves to ||g||rel <= 1e-2 under P_REG, P_2L with CHEB(10) and P_2L with the
    nested PCG(1e-1) coarse solve (the three schemes of section 4.2.2), all with SL transport at
    nt = 4, and the paper's earlier solver, P_REG with RK2A transport at CFL 0.2 (on this problem's
    m_R, made by SL transport)."""
    import numpy as np
    import torch

    import synth
    from paper_1604_02153_amd import Context
    cfg = synth.config("gauss256")
    n1, n2, nt = cfg["n1"], cfg["n2"], cfg["nt"]
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=torch.float32)
    mT, vgen = f32(cfg["mT"]), f32(cfg["v_gen"])
    out = {"workload": "gauss256 (256x256, nt=4, H2 beta=1e-3, mixed), Newton to ||g||rel<=1e-2"}
    # the paper's earlier solver: P_REG with the stabilised RK2 transport at CFL 0.2
    mR = None
    nt_rk = max(2, int(np.ceil(float(np.abs(cfg["v_gen"]).max()) * max(n1, n2) / (2 * np.pi * 0.2))))
    for name, kw in (("P_REG", dict(pc="reg")), ("P_2L_CHEB10", dict(pc="2l")),
                     ("P_2L_PCG0.1", dict(pc="2l", coarse_solver="pcg", coarse_eps=0.1)),
                     (f"P_REG_RK2A(0.2)_nt{nt_rk}", dict(pc="reg", transport="rk2a", nt=nt_rk))):
        kw = dict(kw)
        ctx = Context(n1, n2, kw.pop("nt", nt), reg="h2", beta=cfg["beta"], prec="mixed", **kw)
        if mR is None:  # one m_R for every solver: SL transport over nt = 4 steps
            mR = torch.empty_like(mT)
            ctx.transport_state(vgen, mT, mR)
        ctx.set_images(mR, mT)
        v = torch.zeros_like(vgen)
        ctx.newton_solve(v, max_newton=20)
        v.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep = ctx.newton_solve(v, max_newton=20)
        torch.cuda.synchronize()
        out[name] = {"ms": round(1e3 * (time.perf_counter() - t0), 2), "status": rep["status"],
                     "newton_iters": rep["newton_iters"], "pcg_iters": rep["pcg_iters"],
                     "coarse_matvecs": rep["coarse_matvecs"], "time_precond_ms": round(rep["time_precond_ms"], 2),
                     "grel_final": float(f"{rep['grel'][-1]:.3g}")}
        ctx.close()
    return out


def batched(args, dev):
    """64 independent pairs with grid sizes drawn from {128, ..., 1024}^2 (seed 4; pair p from the
    'gauss256' recipe with seed 4000 + p), one ragged batch: bucket per size, buckets concurrent."""
    import numpy as np
    import torch

    import synth
    from paper_1604_02153_amd import BatchContext, Context
    sizes = synth.batch_sizes(64, 4)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=torch.float32)
    pairs = [synth.batch_pair(p, n) for p, n in enumerate(sizes)]
    mT = [t(c["mT"]) for c in pairs]
    vgen = [t(c["v_gen"]) for c in pairs]
    vt = [t(c["vt"]) for c in pairs]
    del pairs
    # m_R = m_T transported by each pair's velocity (the library's state transport, per size)
    mR = [torch.empty_like(m) for m in mT]
    for n in sorted(set(sizes)):
        idx = [p for p in range(64) if sizes[p] == n]
        c = Context(n, n, 4, reg="h2", beta=1e-3, prec="mixed", pc="reg", batch=len(idx))
        out = torch.empty((len(idx), n, n), dtype=torch.float32, device=dev)
        c.transport_state(torch.stack([vgen[p] for p in idx]), torch.stack([mT[p] for p in idx]), out)
        for j, p in enumerate(idx):
            mR[p].copy_(out[j])
        c.close()
        del out
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log("batched inputs ready")
    bc = BatchContext([(n, n) for n in sizes], 4, reg="h2", beta=1e-3, prec="mixed", pc="2l")
    bc.set_images(mR, mT)
    g = [torch.empty_like(v) for v in vgen]
    out = [torch.empty_like(v) for v in vgen]
    bc.gradient(vgen, g)
    tuned = bc.autotune(vt, reps=3)
    for _ in range(2):
        bc.hessian_matvec(vt, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.batched_matvecs):
        bc.hessian_matvec(vt, out)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    mv_rate = 64 * args.batched_matvecs / dt
    gbs = sum(matvec_bytes(n, n, 4) for n in sizes) * args.batched_matvecs / dt / 1e9
    v = [torch.zeros_like(x) for x in vgen]
    warm = bc.newton_solve(v)  # warm-up solve (graph capture, LDS attributes)
    for x in v:
        x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = bc.newton_solve(v)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    counts = lambda rs: [(r["newton_iters"], r["pcg_iters"], r["cheb_reestimates"]) for r in rs]
    same = counts(warm) == counts(reps)
    if not same:
        log("batched: warm-up and timed solves differ: " +
            str([(p, a, b) for p, (a, b) in enumerate(zip(counts(warm), counts(reps))) if a != b]))
    stop = sorted(r["time_to_stop_ms"] for r in reps)
    buckets = bc.buckets()
    bc.close()
    return {
        "workload": "64 pairs, n^2 with n drawn (seed 4) from {128,256,384,512,768,1024}, gauss256 recipe per "
                    "pair (seed 4000+p), nt=4, H2 beta=1e-3, P_2L, mixed precision; one bucket per size, "
                    "buckets concurrent on their own streams",
        "sizes": {str(n): sizes.count(n) for n in sorted(set(sizes))},
        "matvecs_per_s": round(mv_rate, 1),
        "matvec_GBps_algorithmic": round(gbs, 1), "matvec_roofline_frac": round(gbs / HBM_PEAK_GBS, 4),
        "solve_wall_ms": round(1e3 * wall, 1),
        "solve_fine_matvecs_per_s": round(sum(r["matvecs"] for r in reps) / wall, 1),
        "per_pair_time_to_stop_ms": {"median": round(stop[len(stop) // 2], 1), "max": round(stop[-1], 1)},
        "all_pairs_grel_le_1e-2": all(r["grel"][-1] <= 1e-2 for r in reps),
        "newton_iters": [r["newton_iters"] for r in reps],
        "pcg_iters": [r["pcg_iters"] for r in reps],
        "cheb_reestimates": [r["cheb_reestimates"] for r in reps],
        "warmup_and_timed_counts_identical": same,
        "autotune": [{"n": b[0], "pairs": b[2], "sl_path": b[3], "graphs": b[4], "op_ms": round(ms, 3)}
                     for b, ms in zip(buckets, tuned)],
    }


def brain512(args, dev, oracle_ref=None):
    """Single 512^2 pair, nt = 8, H1 beta 1e-3, P_2L (the 'brain512' recipe): Newton solve time and
    isolated GN matvec rate under both SL kernel paths, with the fraction of the HBM roofline.  (H1
    without divergence control: on this pair the Gauss-Newton steps blow up at 256^2 and 512^2 and
    the solve ends in a failed line search -- the FP64 oracle takes the same path at 256^2 -- so
    its solve figures are reported with their status; the matvec figures are the measurement.)"""
    import numpy as np
    import torch

    import synth
    from paper_1604_02153_amd import Context
    cfg = synth.config("brain512")
    n1, n2, nt = cfg["n1"], cfg["n2"], cfg["nt"]
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=torch.float32)
    mT, vgen, vt = f32(cfg["mT"]), f32(cfg["v_gen"]), f32(cfg["vt"])
    out = {"workload": "brain512: 512x512, nt=8, H1 beta=1e-3, P_2L (256^2, CHEB(10)); 64 anisotropic smoothed "
                       "Gaussians, 24-mode velocity |k|<=6 amplitude 0.5 (seed 3)", "grid": [n1, n2], "nt": nt}
    rates = {}
    for path in (0, 1):
        ctx = Context(n1, n2, nt, reg="h1", beta=cfg["beta"], prec="mixed", pc="2l", sl_path=path)
        mR = torch.empty_like(mT)
        ctx.transport_state(vgen, mT, mR)
        ctx.set_images(mR, mT)
        v = torch.zeros_like(vgen)
        ctx.newton_solve(v)  # warm-up (graph capture, LDS attributes)
        v.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep = ctx.newton_solve(v)
        torch.cuda.synchronize()
        solve_ms = 1e3 * (time.perf_counter() - t0)
        g = torch.empty_like(v)
        ctx.gradient(vgen, g)
        h = torch.empty_like(v)
        for _ in range(10):
            ctx.hessian_matvec(vt, h)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.brain_matvecs):
            ctx.hessian_matvec(vt, h)
        torch.cuda.synchronize()
        rate = args.brain_matvecs / (time.perf_counter() - t1)
        gbs = matvec_bytes(n1, n2, nt) * rate / 1e9
        rates[path] = rate
        out["fused_sl_step" if path == 0 else "two_kernel_sl_step"] = {
            "solve_ms": round(solve_ms, 2), "solve_status": rep["status"], "newton_iters": rep["newton_iters"],
            "pcg_iters": rep["pcg_iters"], "grel_final": rep["grel"][-1], "matvecs_per_s": round(rate, 1),
            "matvec_GBps_algorithmic": round(gbs, 1), "matvec_roofline_frac": round(gbs / HBM_PEAK_GBS, 4)}
        ctx.close()
    # the paper's pairing of H1 with incompressibility: K = Leray, divergence-free generating velocity
    ic = synth.config("brain512ic")
    mT, vgen, vt = f32(ic["mT"]), f32(ic["v_gen"]), f32(ic["vt"])
    ctx = Context(n1, n2, nt, reg="h1", beta=ic["beta"], prec="mixed", pc="2l", proj="leray")
    mR = torch.empty_like(mT)
    ctx.transport_state(vgen, mT, mR)
    ctx.set_images(mR, mT)
    v = torch.zeros_like(vgen)
    ctx.newton_solve(v, max_newton=20)
    v.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = ctx.newton_solve(v, max_newton=20)
    torch.cuda.synchronize()
    solve_ms = 1e3 * (time.perf_counter() - t0)
    g = torch.empty_like(v)
    ctx.gradient(vgen, g)
    h = torch.empty_like(v)
    for _ in range(10):
        ctx.hessian_matvec(vt, h)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.brain_matvecs):
        ctx.hessian_matvec(vt, h)
    torch.cuda.synchronize()
    rate = args.brain_matvecs / (time.perf_counter() - t1)
    out["incompressible"] = {
        "workload": "brain512ic: the brain512 image, divergence-free 24-mode velocity |k|<=6 amplitude 0.5 (seed 3), "
                    "K = Leray projection, H1 beta=1e-3, P_2L, Newton to ||g||rel<=1e-2 (at most 20 steps)",
        "solve_ms": round(solve_ms, 2), "solve_status": rep["status"], "newton_iters": rep["newton_iters"],
        "pcg_iters": rep["pcg_iters"], "grel": [float(f"{x:.3g}") for x in rep["grel"]],
        "matvecs_per_s": round(rate, 1)}
    ctx.close()
    if oracle_ref is not None:
        out["errors_vs_oracle"] = {
            "inputs": "each recipe rounded to FP32, m_R by the oracle's transport, gradient and matvec at v_gen",
            "brain512": brain_errors(oracle_ref["brain512"], dev, proj="none"),
            "brain512ic": brain_errors(oracle_ref["brain512ic"], dev, proj="leray")}
    return out


def brain_errors(ref, dev, proj):
    """Mixed context against the FP64 oracle's results of the cpu_baseline leg on the 512^2 recipe's
    own inputs (rounded to FP32; m_R by the oracle's transport): relative L2 errors of the state
    transport, the gradient and the GN matvec at v_gen (nt = 8, H1, beta = 1e-3; K = Leray for the
    incompressible recipe)."""
    import numpy as np
    import torch

    from paper_1604_02153_amd import Context
    n1, n2 = ref["mT"].shape
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=torch.float32)
    host = lambda x: x.double().cpu().numpy()
    ctx = Context(n1, n2, ref["nt"], reg="h1", beta=ref["beta"], prec="mixed", pc="2l", proj=proj)
    m1g = torch.empty((n1, n2), dtype=torch.float32, device=dev)
    ctx.transport_state(t(ref["v_gen"]), t(ref["mT"]), m1g)
    ctx.set_images(t(ref["mR"]), t(ref["mT"]))
    gg = torch.empty((2, n1, n2), dtype=torch.float32, device=dev)
    ctx.gradient(t(ref["v_gen"]), gg)
    hg = torch.empty_like(gg)
    ctx.hessian_matvec(t(ref["vt"]), hg)
    ctx.close()
    return {"transport_state": float(f"{rel_l2(host(m1g), ref['m1']):.3g}"),
            "gradient": float(f"{rel_l2(host(gg), ref['grad']):.3g}"),
            "gn_matvec": float(f"{rel_l2(host(hg), ref['hvt']):.3g}")}


def d3_matvec_bytes(n, nt, elem=4):
    """Algorithmic HBM bytes of one 3-D Gauss-Newton matvec (each field read or written once per
    use): the incremental state's start (vt, grad m^0 in, q out: 7 fields), per incremental state
    step the B-spline coefficients (2) and the step (displacement 3, coefficients 1, grad m^j 3,
    vt 3, out 1), the last step's b~ start (3), per incremental adjoint step coefficients (2) and
    the step (displacement 3, coefficients 1, gamma 1, grad m 3, b~ 3 in and 3 out, out 1), beta A
    vt (6) and the final K b~ + beta A vt (9): 25 + 30 nt fields of n^3 values."""
    return (25 + 30 * nt) * n ** 3 * elem


def d3_setup(dev, prec, n=128, sl_path=0, pc="reg", hessian="gn", coarse_solver="cheb"):
    import numpy as np
    import torch

    import synth
    from paper_1604_02153_amd import Context3
    mT, vgen, nt, beta, reg = synth.config_3d("gauss3d128", n=n)
    dt = torch.float32 if prec == "mixed" else torch.float64
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=dt)
    vt = synth.random_velocity_3d(n, n, n, np.random.default_rng(1234), amplitude=0.1)
    ctx = Context3(n, n, n, nt, reg=reg, beta=beta, prec=prec, sl_path=sl_path, pc=pc, hessian=hessian,
                   coarse_solver=coarse_solver, coarse_eps=0.1)
    mT_t, vgen_t = t(mT), t(vgen)
    mR_t = torch.empty_like(mT_t)
    ctx.transport_state(vgen_t, mT_t, mR_t)
    if pc == "reg":
        ctx.set_images(mR_t, mT_t)
    return ctx, mR_t, mT_t, vgen_t, t(vt), nt, beta


def d3_probe():
    import torch
    dev = torch.device("cuda:0")
    for sl_path in (0, 1):
        ctx, mR, mT, vgen, vt, nt, beta = d3_setup(dev, "mixed", sl_path=sl_path)
        g = torch.empty_like(vgen)
        ctx.gradient(vgen, g)
        out = torch.empty_like(vgen)
        for _ in range(20):
            ctx.hessian_matvec(vt, out)
        torch.cuda.synchronize()
        log(f"3-D probe done: sl_path {sl_path}, 1 gradient, 20 matvecs at 128^3")
        ctx.close()


def d3_rk2a(dev, reps=3):
    """The 128^3 problem with RK2A transport at CFL 0.2 (nt from the generating velocity) and P_REG,
    the paper's earlier solver, mixed precision: m_R = m_T transported by RK2A, isolated GN matvecs
    at v_gen, and the Newton-PCG solve from v = 0."""
    import numpy as np
    import torch

    import synth
    from paper_1604_02153_amd import Context3
    n = 128
    mT, vgen, _, beta, reg = synth.config_3d("gauss3d128", n=n)
    nt = max(2, int(np.ceil(float(np.sqrt((vgen ** 2).sum(axis=0)).max()) * n / (2 * np.pi * 0.2))))
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=torch.float32)
    vt = t(synth.random_velocity_3d(n, n, n, np.random.default_rng(1234), amplitude=0.1))
    ctx = Context3(n, n, n, nt, reg=reg, beta=beta, prec="mixed", pc="reg", transport="rk2a")
    mT_t, vgen_t = t(mT), t(vgen)
    mR_t = torch.empty_like(mT_t)
    ctx.transport_state(vgen_t, mT_t, mR_t)
    ctx.set_images(mR_t, mT_t)
    g = torch.empty_like(vgen_t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.gradient(vgen_t, g)
    torch.cuda.synchronize()
    grad_ms = 1e3 * (time.perf_counter() - t0)
    hv = torch.empty_like(vgen_t)
    ctx.hessian_matvec(vt, hv)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.hessian_matvec(vt, hv)
    torch.cuda.synchronize()
    mv_ms = 1e3 * (time.perf_counter() - t0) / reps
    v = torch.zeros_like(vgen_t)
    rep = ctx.newton_solve(v)
    ctx.close()
    log(f"3-D RK2A: nt {nt}, matvec {mv_ms:.1f} ms, solve {rep['time_total_ms']:.0f} ms")
    return {"workload": f"gauss3d128 with RK2A transport, CFL 0.2 (nt={nt}), P_REG; m_R = m_T transported by RK2A",
            "nt": nt, "matvec_ms": round(mv_ms, 2), "gradient_ms": round(grad_ms, 2),
            "solve_ms": round(rep["time_total_ms"], 1), "newton_iters": rep["newton_iters"],
            "pcg_iters": rep["pcg_iters"], "grel_final": rep["grel"][-1], "status": rep["status"]}


def d3_workload(args, dev):
    """The method in three dimensions: the Gaussian-blob recipe on a 128^3 volume (nt = 4, H2,
    beta = 1e-3), mixed precision and FP64: isolated GN matvecs and a Newton-PCG solve with P_REG."""
    import torch
    out = {"workload": "gauss3d128: 128^3, nt=4, H2 beta=1e-3, K = I; P_REG and P_2L (64^3, CHEB(10)); "
                       "m_R = m_T transported by v_gen"}
    for prec in ("mixed", "fp64"):
        ctx, mR, mT, vgen, vt, nt, beta = d3_setup(dev, prec)
        g = torch.empty_like(vgen)
        ctx.gradient(vgen, g)
        hv = torch.empty_like(vgen)
        ctx.hessian_matvec(vt, hv)
        torch.cuda.synchronize()
        reps = args.d3_matvecs if prec == "mixed" else max(5, args.d3_matvecs // 2)
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.hessian_matvec(vt, hv)
        torch.cuda.synchronize()
        mv_ms = 1e3 * (time.perf_counter() - t0) / reps
        t0 = time.perf_counter()
        ctx.gradient(vgen, g)
        torch.cuda.synchronize()
        grad_ms = 1e3 * (time.perf_counter() - t0)
        v = torch.zeros_like(vgen)
        t0 = time.perf_counter()
        rep = ctx.newton_solve(v)
        solve_ms = 1e3 * (time.perf_counter() - t0)
        elem = 4 if prec == "mixed" else 8
        gbs = d3_matvec_bytes(128, nt, elem) / (mv_ms * 1e-3) / 1e9
        if prec == "mixed":  # the other SL path (stencils read from the global coefficients)
            ctx1, _, _, vgen1, vt1, _, _ = d3_setup(dev, prec, sl_path=1)
            g1 = torch.empty_like(vgen1)
            ctx1.gradient(vgen1, g1)
            ctx1.hessian_matvec(vt1, g1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                ctx1.hessian_matvec(vt1, g1)
            torch.cuda.synchronize()
            out["mixed_global_gather_matvec_ms"] = round(1e3 * (time.perf_counter() - t0) / reps, 3)
            ctx1.close()
            del g1, vgen1, vt1
            # the full-Newton matvec (incremental adjoint with its div(lambda vt) source, b~ with
            # lambda grad m~) at v_gen / 2, where lambda != 0, and a full-Newton P_2L solve from v = 0
            ctxf, mRf, mTf, vgenf, vtf, _, _ = d3_setup(dev, prec, pc="2l", hessian="fn")
            ctxf.set_images(mRf, mTf)
            gf = torch.empty_like(vgenf)
            ctxf.gradient(0.5 * vgenf, gf)
            ctxf.hessian_matvec(vtf, gf)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                ctxf.hessian_matvec(vtf, gf)
            torch.cuda.synchronize()
            fn_mv_ms = 1e3 * (time.perf_counter() - t0) / reps
            vf = torch.zeros_like(vgenf)
            repf = ctxf.newton_solve(vf)
            out["mixed_full_newton"] = {
                "matvec_ms": round(fn_mv_ms, 3), "matvec_at": "v_gen / 2",
                "two_level_solve": {"solve_ms": round(repf["time_total_ms"], 2), "newton_iters": repf["newton_iters"],
                                    "pcg_iters": repf["pcg_iters"], "coarse_matvecs": repf["coarse_matvecs"],
                                    "grel_final": repf["grel"][-1], "status": repf["status"]},
                "workspace_GB": round(ctxf.workspace_bytes() / 1e9, 3)}
            ctxf.close()
            del gf, vf, mRf, mTf, vgenf, vtf
            # P_2L with the nested PCG(0.1) coarse solve instead of CHEB(10)
            ctxp, mRp, mTp, vgenp, _, _, _ = d3_setup(dev, prec, pc="2l", coarse_solver="pcg")
            vp = torch.zeros_like(vgenp)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctxp.set_images(mRp, mTp)
            repp = ctxp.newton_solve(vp)
            out["mixed_two_level_pcg0.1"] = {
                "setup_plus_solve_ms": round(1e3 * (time.perf_counter() - t0), 2),
                "solve_ms": round(repp["time_total_ms"], 2), "newton_iters": repp["newton_iters"],
                "pcg_iters": repp["pcg_iters"], "coarse_matvecs": repp["coarse_matvecs"],
                "grel_final": repp["grel"][-1], "status": repp["status"],
                "time_precond_ms": round(repp["time_precond_ms"], 2)}
            ctxp.close()
            del vp, mRp, mTp, vgenp
            out["mixed_rk2a"] = d3_rk2a(dev, reps=3)
        # the same problem with P_2L (coarse grid 64^3, CHEB(10), 30 Lanczos steps at set-up)
        ctx2, mR2, mT2, vgen2, _, _, _ = d3_setup(dev, prec, pc="2l")
        v2 = torch.zeros_like(vgen2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx2.set_images(mR2, mT2)
        rep2 = ctx2.newton_solve(v2)
        setup_solve2 = 1e3 * (time.perf_counter() - t0)
        two_level = {"setup_plus_solve_ms": round(setup_solve2, 2), "solve_ms": round(rep2["time_total_ms"], 2),
                     "newton_iters": rep2["newton_iters"], "pcg_iters": rep2["pcg_iters"],
                     "coarse_matvecs": rep2["coarse_matvecs"], "grel_final": rep2["grel"][-1],
                     "status": rep2["status"], "emax": round(rep2["emax"], 3),
                     "time_precond_ms": round(rep2["time_precond_ms"], 2)}
        ctx2.close()
        del mR2, mT2, vgen2, v2
        out[prec] = {"matvec_ms": round(mv_ms, 3), "matvecs_per_s": round(1e3 / mv_ms, 2),
                     "matvec_GBps_algorithmic": round(gbs, 1), "matvec_frac_of_hbm": round(gbs / HBM_PEAK_GBS, 4),
                     "gradient_ms": round(grad_ms, 3), "solve_ms": round(solve_ms, 2),
                     "newton_iters": rep["newton_iters"], "pcg_iters": rep["pcg_iters"],
                     "grel_final": rep["grel"][-1], "status": rep["status"],
                     "workspace_GB": round(ctx.workspace_bytes() / 1e9, 3), "two_level": two_level}
        ctx.close()
        del g, hv, v, mR, mT, vgen, vt
        torch.cuda.empty_cache()
        log(f"3-D {prec}: matvec {mv_ms:.2f} ms, solve {solve_ms:.1f} ms")
    return out


def unet_flops(h, w, levels=4, base=32):
    """Multiply-add flops (2 per MAC) of one forward pass of the U-Net on an h x w pair."""
    C = [base << l for l in range(levels)]
    convs = []
    for l in range(levels):
        convs += [(32 if l == 0 else C[l - 1], C[l], l), (C[l], C[l], l)]
    for l in range(levels - 1):
        convs += [(C[l + 1] + C[l], C[l], l), (C[l], C[l], l)]
    convs.append((C[0], 32, 0))
    return sum(2 * 9 * ci * co * (h >> l) * (w >> l) for ci, co, l in convs)


def learned(args, dev):
    """Time to ||g||_rel <= 1e-2 of the plain and the learned solve (network forward + solve from
    its start, fallback to v = 0) on the 256^2 problem (seed 2) and held-out pairs (seeds 200000...,
    not seen in training), one pair per context, same GPU."""
    import numpy as np
    import torch

    from paper_1604_02153_amd import Context, UNet
    from paper_1604_02153_amd.train_unet import make_pair
    if not os.path.exists(WEIGHTS):
        return {"status": "no trained weights at " + os.path.relpath(WEIGHTS, ROOT)}
    ctx = Context(256, 256, 4, reg="h2", beta=1e-3, prec="mixed", pc="2l", cheb_iters=10, lanczos_steps=30)
    net = UNet(256, 256, 4, 32, max_batch=1)
    net.load(WEIGHTS)
    v = torch.zeros((2, 256, 256), dtype=torch.float32, device=dev)
    rows = []
    for i, seed in enumerate([2] + list(range(200000, 200000 + args.learned_pairs))):
        mT, vg = make_pair(seed)
        mT, vg = torch.from_numpy(mT).to(dev), torch.from_numpy(vg).to(dev)
        mR = torch.empty_like(mT)
        ctx.transport_state(vg, mT, mR)
        if i == 0:  # warm-up of both paths (graph capture, LDS attributes)
            ctx.set_images(mR, mT)
            v.zero_()
            ctx.newton_solve(v)
            ctx.set_images_learned(net, mR, mT)
            ctx.newton_solve_learned(net, v)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.set_images(mR, mT)                   # plain set-up: Lanczos for e_max
        v.zero_()
        ts = time.perf_counter()
        rp = ctx.newton_solve(v)
        t1 = time.perf_counter()
        ctx.set_images_learned(net, mR, mT)      # learned set-up: network start + e_max from its head
        tl = time.perf_counter()
        rl = ctx.newton_solve_learned(net, v)
        t2 = time.perf_counter()
        rows.append((1e3 * (t1 - ts), 1e3 * (t2 - tl), rp["newton_iters"], rl["newton_iters"], rp["pcg_iters"],
                     rl["pcg_iters"], rl["fallback"], rp["grel"][-1] <= 1e-2, rl["grel"][-1] <= 1e-2,
                     1e3 * (t1 - t0), 1e3 * (t2 - t1)))
    a = np.array(rows, dtype=np.float64)
    # network forward alone (BF16 MFMA), one 256^2 pair
    mR1, mT1 = mR.reshape(1, 256, 256).contiguous(), mT.reshape(1, 256, 256).contiguous()
    vo = torch.empty((1, 2, 256, 256), dtype=torch.float32, device=dev)
    for _ in range(3):
        net.forward(mR1, mT1, vo)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        net.forward(mR1, mT1, vo)
    torch.cuda.synchronize()
    fwd_ms = 1e3 * (time.perf_counter() - t0) / 20
    tf = unet_flops(256, 256) / (fwd_ms * 1e-3) / 1e12
    net.close()
    ctx.close()
    med = lambda c: round(float(np.median(a[:, c])), 2)
    return {
        "workload": f"gauss256 pair (seed 2) + {args.learned_pairs} held-out pairs (seeds 200000...), 256^2, "
                    "P_2L mixed; learned = U-Net (4 levels, 32 channels, BF16) start from its |k|<=8 modes and "
                    "e_max from its head; times from the solve call to ||g||rel<=1e-2, and set-up + solve",
        "seed2_ms": {"plain": round(a[0, 0], 2), "learned": round(a[0, 1], 2)},
        "median_ms": {"plain": med(0), "learned": med(1)},
        "median_setup_plus_solve_ms": {"plain": med(9), "learned": med(10)},
        "mean_ms": {"plain": round(float(a[:, 0].mean()), 2), "learned": round(float(a[:, 1].mean()), 2)},
        "speedup_median": round(float(np.median(a[:, 0]) / np.median(a[:, 1])), 3),
        "newton_mean": {"plain": round(float(a[:, 2].mean()), 2), "learned": round(float(a[:, 3].mean()), 2)},
        "pcg_mean": {"plain": round(float(a[:, 4].mean()), 2), "learned": round(float(a[:, 5].mean()), 2)},
        "fallback_rate": round(float(a[:, 6].mean()), 3),
        "reached_grel_1e-2": {"plain": int(a[:, 7].sum()), "learned": int(a[:, 8].sum()), "of": len(rows)},
        "unet_forward_ms": round(fwd_ms, 3),
        "unet_roofline": {"bound": "mfma", "achieved": round(tf, 1), "peak": BF16_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                          "frac": round(tf / BF16_MFMA_PEAK_TFLOPS, 4)},
    }


def _oracle_worker(args):
    """One host process of the all-cores oracle sample: GN matvecs of the 256^2 problem at v_gen
    (numpy pools at one thread) until 'seconds' have passed; returns the count and the time."""
    seconds, = args
    from threadpoolctl import threadpool_limits

    import oracle as O
    import synth
    with threadpool_limits(limits=1):
        cfg = synth.config("gauss256")
        g = O.Grid(cfg["n1"], cfg["n2"])
        L = O.Level(g, cfg["mT"], O.transport_state(g, cfg["v_gen"], cfg["mT"], cfg["nt"]),
                    O.Params(nt=cfg["nt"], beta=cfg["beta"], reg=cfg["reg"]))
        lin = O.linearize(L, cfg["v_gen"])
        O.hessian_matvec(lin, cfg["vt"])
        n, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < seconds:
            O.hessian_matvec(lin, cfg["vt"])
            n += 1
        return n, time.perf_counter() - t0


def host_cores():
    """Cores this process may run on (the box's share), at most 16."""
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        return max(1, min(16, os.cpu_count() or 1))


def cpu_baseline(cfg, min_seconds):
    """The FP64 oracle (numpy) on the host, before any GPU work:
    - the GN matvec rate of the 256^2 problem at the generating velocity, on one thread and as the
      throughput of one process per host core (independent matvecs, each process one thread);
    - its Newton--Krylov solve of the same problem (P_2L, CHEB(10)) on one thread;
    - the reference results the GPU's error statements compare against: inputs rounded to FP32
      (what the mixed context receives; the FP64 context gets the same values), m_R by the
      oracle's transport, the gradient and matvec at v_gen, the P_2L application and the solve."""
    import multiprocessing as mp

    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle as O
    r32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)
    cores = host_cores()
    ctx = mp.get_context("fork")  # no GPU has been touched yet in this process
    with ctx.Pool(cores) as pool:
        res = pool.map(_oracle_worker, [(min_seconds,)] * cores)
    all_rate = sum(n / dt for n, dt in res)
    all_n = sum(n for n, _ in res)
    with threadpool_limits(limits=1):
        g = O.Grid(cfg["n1"], cfg["n2"])
        mT, vgen, vt = r32(cfg["mT"]), r32(cfg["v_gen"]), r32(cfg["vt"])
        mR = r32(O.transport_state(g, vgen, mT, cfg["nt"]))
        L = O.Level(g, mT, mR, O.Params(nt=cfg["nt"], beta=cfg["beta"], reg=cfg["reg"]))
        lin = O.linearize(L, vgen)
        grad = O.gradient(lin)
        O.hessian_matvec(lin, vt)          # warm-up (FFT plans, caches)
        n_matvec = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < min_seconds and n_matvec < 2000:
            h = O.hessian_matvec(lin, vt)
            n_matvec += 1
        dt = time.perf_counter() - t0
        t1 = time.perf_counter()
        v_sol, rep = O.newton_solve(L, pc="2l", max_newton=20)
        solve_s = time.perf_counter() - t1
        tl = O.setup_two_level(L)
        cg = tl.coarse.grid
        tl.lin_c = O.linearize(tl.coarse, np.stack([O.restrict(g, cg, vgen[c]) for c in range(2)]))
        z = O.apply_two_level(L, tl, vt)
    timing = {"value": round(all_rate, 2), "unit": "matvecs/s", "cores": cores, "kind": "oracle",
              "sample": f"{all_n} FP64 GN Hessian matvecs of the 256^2 nt=4 H2 problem at v_gen, one numpy process "
                        f"per host core ({cores}, each {min_seconds:.0f} s, one thread each)",
              "single_thread": {"value": round(n_matvec / dt, 2), "unit": "matvecs/s", "cores": 1,
                                "sample": f"{n_matvec} matvecs in {dt:.1f} s"},
              "solve_single_thread_s": round(solve_s, 2),
              "solve": {"newton_iters": rep["newton_iters"], "pcg_iters": rep["pcg_iters"],
                        "grel_final": float(f"{rep['grel'][-1]:.4g}"), "status": rep["status"]}}
    ref = {"mT": mT, "mR": mR, "v_gen": vgen, "vt": vt, "J": lin.J, "m1": lin.m[-1], "grad": grad, "hvt": h,
           "p2l_vt": z, "v_sol": v_sol, "g0_inf": rep["g0_inf"], "emax": tl.emax, "emin": tl.emin}
    # the 512^2 recipes (nt = 8, H1; K = I and K = Leray): the oracle's transport, gradient and GN
    # matvec at v_gen on the inputs rounded to FP32
    import synth
    for name, proj in (("brain512", 0), ("brain512ic", 1)):
        bc = synth.config(name)
        with threadpool_limits(limits=1):
            gb = O.Grid(bc["n1"], bc["n2"])
            bT, bv, bvt = r32(bc["mT"]), r32(bc["v_gen"]), r32(bc["vt"])
            b1 = O.transport_state(gb, bv, bT, bc["nt"])
            Lb = O.Level(gb, bT, r32(b1), O.Params(nt=bc["nt"], beta=bc["beta"], reg=bc["reg"], proj=proj))
            linb = O.linearize(Lb, bv)
            gradb = O.gradient(linb)
            t0 = time.perf_counter()
            hvtb = O.hessian_matvec(linb, bvt)
            if proj == 0:  # one matvec of the 512^2 nt = 8 problem
                timing["matvec_512_single_thread_s"] = round(time.perf_counter() - t0, 2)
            ref[name] = {"mT": bT, "mR": Lb.mR, "v_gen": bv, "vt": bvt, "m1": b1, "grad": gradb,
                         "hvt": hvtb, "nt": bc["nt"], "beta": bc["beta"]}
    # the smooth 64^2 problem (FP64, H1, beta = 1e-2, P_REG): the oracle's solve on one thread
    sc = synth.config("smooth64")
    with threadpool_limits(limits=1):
        gs = O.Grid(sc["n1"], sc["n2"])
        Ls = O.Level(gs, sc["mT"], O.transport_state(gs, sc["v_gen"], sc["mT"], sc["nt"]),
                     O.Params(nt=sc["nt"], beta=sc["beta"], reg=sc["reg"]))
        t0 = time.perf_counter()
        _, reps = O.newton_solve(Ls, pc="reg", max_newton=20)
        timing["solve_smooth64_single_thread_s"] = round(time.perf_counter() - t0, 2)
        timing["solve_smooth64"] = {"newton_iters": reps["newton_iters"], "pcg_iters": reps["pcg_iters"],
                                    "status": reps["status"]}
    return timing, ref


def rel_l2(a, b):
    import numpy as np
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def errors_vs_oracle(ref, dev):
    """The precision form: the mixed context (FP32 fields and transforms, FP64 reductions, FP64
    iterate and beta A) and the all-FP64 context against the FP64 oracle on the same inputs (the
    oracle's, rounded to FP32): relative L2 error of each result, and for the solves the oracle's
    GPU's own ||g||_rel at its final velocity.""" 
    import numpy as np
    import torch

    from paper_1604_02153_amd import Context
    n1, n2 = ref["mT"].shape
    out = {"inputs": "gauss256 recipe rounded to FP32, m_R by the oracle's transport; gradient and matvec at "
                     "v_gen; P_2L at v_gen; Newton-PCG (P_2L) from v = 0 to ||g||rel<=1e-2"}
    for prec in ("mixed", "fp64"):
        dt = torch.float32 if prec == "mixed" else torch.float64
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=dt)
        host = lambda x: x.double().cpu().numpy()
        ctx = Context(n1, n2, 4, reg="h2", beta=1e-3, prec=prec, pc="2l")
        m1 = torch.empty((n1, n2), dtype=dt, device=dev)
        ctx.transport_state(t(ref["v_gen"]), t(ref["mT"]), m1)
        ctx.set_images(t(ref["mR"]), t(ref["mT"]))
        g = torch.empty((2, n1, n2), dtype=dt, device=dev)
        J = ctx.gradient(t(ref["v_gen"]), g)
        h = torch.empty_like(g)
        ctx.hessian_matvec(t(ref["vt"]), h)
        z = torch.empty_like(g)
        ctx.precond_apply(t(ref["vt"]), z)
        emin, emax = ctx.cheb_bounds()
        v = torch.zeros_like(g)
        rep = ctx.newton_solve(v, max_newton=20)
        out[prec] = {"transport_state": rel_l2(host(m1), ref["m1"]), "objective": abs(J - ref["J"]) / abs(ref["J"]),
                     "gradient": rel_l2(host(g), ref["grad"]), "gn_matvec": rel_l2(host(h), ref["hvt"]),
                     "p2l_apply": rel_l2(host(z), ref["p2l_vt"]), "cheb_emax": abs(emax - ref["emax"]) / ref["emax"],
                     "newton_v": rel_l2(host(v), ref["v_sol"]), "newton_status": rep["status"],
                     "newton_grel_gpu": float(f"{rep['grel'][-1]:.4g}")}
        out[prec] = {k: (float(f"{x:.3g}") if isinstance(x, float) else x) for k, x in out[prec].items()}
        ctx.close()
    return out


def time_matvecs(ctx, vt, out, count):
    """Back-to-back GN Hessian matvecs at the context's linearisation point: matvecs per second."""
    import torch
    for _ in range(20):
        ctx.hessian_matvec(vt, out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(count):
        ctx.hessian_matvec(vt, out)
    torch.cuda.synchronize()
    return count / (time.perf_counter() - t1)


def timed_solves(ctx, mR, mT, v, steps, warmup):
    """'steps' solves of one pair after 'warmup' untimed ones; one step is the per-pair set-up
    (images, coarse problem, Lanczos for e_max) and the Newton--Krylov solve from v = 0.  Returns
    the wall time of all steps, the solve-only times and the last report."""
    import torch
    for _ in range(warmup):
        ctx.set_images(mR, mT)
        v.zero_()
        ctx.newton_solve(v)
    torch.cuda.synchronize()
    solve_ms, reps = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.set_images(mR, mT)
        v.zero_()
        ts = time.perf_counter()
        reps.append(ctx.newton_solve(v))   # returns after its final synchronisation
        solve_ms.append(1e3 * (time.perf_counter() - ts))
    torch.cuda.synchronize()
    return time.perf_counter() - t0, solve_ms, reps[-1]


def roofline_entry(ctx, n1, n2, what):
    """The incremental-adjoint SL step of a context: HIP-event duration of 200 back-to-back launches
    on the library's stream, against the step's algorithmic bytes."""
    k_ms = ctx.time_kernel(3, 200)
    bytes_per_launch = INC_ADJ_FIELDS_PER_POINT * 4 * n1 * n2
    achieved = bytes_per_launch / (k_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "kernel": "k_sl_step<float, IncAdjoint> (fused LDS prefilter + "
            "gather), " + what, "avg_launch_us": round(k_ms * 1e3, 3), "algorithmic_bytes_per_launch": bytes_per_launch,
            "fields_per_point": INC_ADJ_FIELDS_PER_POINT}


def main():
    args = parse()
    if args.spectral:
        spectral_probe()
        return
    if args.probe:
        probe()
        return
    if args.probe_coarse:
        coarse_probe()
        return
    if args.probe_3d:
        d3_probe()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); runs on several GPUs are not "
              "part of this benchmark.", file=sys.stderr)
        sys.exit(2)
    import numpy as np

    import synth
    cfg = synth.config("gauss256")
    oracle_timing = oracle_ref = None
    if not args.no_cpu_baseline:  # before any GPU work: the host pool forks this process
        oracle_timing, oracle_ref = cpu_baseline(cfg, args.cpu_seconds)
        log("cpu baseline done")

    import torch

    from paper_1604_02153_amd import Context
    n1, n2, nt = cfg["n1"], cfg["n2"], cfg["nt"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=torch.float32)
    ctx = Context(n1, n2, nt, reg="h2", beta=cfg["beta"], prec="mixed", pc="2l", cheb_iters=10, lanczos_steps=30)
    mT, vgen, vt = f32(cfg["mT"]), f32(cfg["v_gen"]), f32(cfg["vt"])
    mR = torch.empty_like(mT)
    ctx.transport_state(vgen, mT, mR)
    v = torch.zeros((2, n1, n2), dtype=torch.float32, device=dev)
    wall, solve_ms, last = timed_solves(ctx, mR, mT, v, args.steps, args.warmup)
    ms_per_step = 1e3 * wall / args.steps
    log(f"single-pair set-up + solve: {ms_per_step:.1f} ms each")

    # isolated GN matvecs at the generating velocity (linearisation point), back to back: the
    # headline rate
    g = torch.empty_like(v)
    ctx.gradient(vgen, g)
    out = torch.empty_like(v)
    iso = time_matvecs(ctx, vt, out, args.matvecs)
    roof = roofline_entry(ctx, n1, n2, "256^2 fine level")
    roof["traffic"] = measured_traffic()
    ctx.close()

    # the P_2L coarse level's step: the same recipe on the 128^2 coarse grid
    c128 = synth.config("gauss256", n=128)
    cc = Context(128, 128, nt, reg="h2", beta=cfg["beta"], prec="mixed", pc="reg")
    m128, v128 = f32(c128["mT"]), f32(c128["v_gen"])
    r128 = torch.empty_like(m128)
    cc.transport_state(v128, m128, r128)
    cc.set_images(r128, m128)
    g128 = torch.empty_like(v128)
    cc.gradient(v128, g128)
    roof_coarse = roofline_entry(cc, 128, 128, "128^2 (the P_2L coarse grid of the 256^2 problem, where most "
                                 "of a solve's SL steps run)")
    cc.close()

    # all-FP64 GPU leg (same problem, same inputs)
    d64 = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=torch.float64)
    c64 = Context(n1, n2, nt, reg="h2", beta=cfg["beta"], prec="fp64", pc="2l", cheb_iters=10, lanczos_steps=30)
    mT64, vgen64, vt64 = d64(cfg["mT"]), d64(cfg["v_gen"]), d64(cfg["vt"])
    mR64 = torch.empty_like(mT64)
    c64.transport_state(vgen64, mT64, mR64)
    v64 = torch.zeros((2, n1, n2), dtype=torch.float64, device=dev)
    wall64, solve64, last64 = timed_solves(c64, mR64, mT64, v64, max(1, args.steps // 2), 1)
    g64 = torch.empty_like(v64)
    c64.gradient(vgen64, g64)
    iso64 = time_matvecs(c64, vt64, torch.empty_like(v64), max(20, args.matvecs // 2))
    c64.close()
    log("FP64 leg done")

    def solve_summary(rep, step_ms, solve_list):
        return {"setup_plus_solve_ms": round(step_ms, 3), "solve_ms_median": round(float(np.median(solve_list)), 3),
                "newton_iters": rep["newton_iters"], "pcg_iters": rep["pcg_iters"], "fine_matvecs": rep["matvecs"],
                "coarse_matvecs": rep["coarse_matvecs"], "grel_final": rep["grel"][-1], "status": rep["status"],
                "time_pcg_ms": round(rep["time_pcg_ms"], 3), "time_precond_ms": round(rep["time_precond_ms"], 3),
                "time_gradient_ms": round(rep["time_gradient_ms"], 3),
                "time_linesearch_ms": round(rep["time_linesearch_ms"], 3)}

    mv_bytes = matvec_bytes(n1, n2, nt)
    line = {
        "metric": "Hessian matvecs/s @256²; time to ‖g‖rel≤1e-2, learned vs plain, same GPU",
        "value": round(iso, 1), "unit": "matvecs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 fields, f64 reductions", "data": "synthetic",
        "config": {"workload": "gauss256: 256x256, nt=4, H2 beta=1e-3, P_2L (128^2, CHEB(10)), mixed precision",
                   "value": "isolated Gauss-Newton Hessian matvecs per second at the generating velocity "
                            "(back to back, beta A in FP64, transport and its transforms in FP32)",
                   "step": "one plain solve: per-pair set-up (images, coarse problem, 30-step Lanczos for e_max) "
                           "and Newton-PCG from v = 0 to ||g||rel<=1e-2",
                   "grid": [n1, n2], "nt": nt},
        "solve": solve_summary(last, ms_per_step, solve_ms),
        "isolated_matvec_GBps_algorithmic": round(mv_bytes * iso / 1e9, 1),
        "roofline": roof,
        "roofline_coarse_step": roof_coarse,
        "roofline_matvec": {"bound": "hbm", "achieved": round(mv_bytes * iso / 1e9, 1), "peak": HBM_PEAK_GBS,
                            "unit": "GB/s", "frac": round(mv_bytes * iso / 1e9 / HBM_PEAK_GBS, 4),
                            "algorithmic_bytes_per_matvec": mv_bytes,
                            "what": "whole GN matvec, (23 nt + 32) FP32 fields"},
        "fp64": {"isolated_matvecs_per_s": round(iso64, 1), "solve": solve_summary(last64, 1e3 * wall64 / max(1, args.steps // 2), solve64),
                 "isolated_matvec_GBps_algorithmic": round(matvec_bytes(n1, n2, nt, 8) * iso64 / 1e9, 1)},
    }
    if oracle_ref is not None:
        line["errors_vs_oracle"] = errors_vs_oracle(oracle_ref, dev)
        log("errors vs oracle done")
    if not args.no_learned:
        line["learned_vs_plain"] = learned(args, dev)
        log("learned vs plain done")
    if not args.no_brain:
        line["brain512"] = brain512(args, dev, oracle_ref)
        log("512^2 workload done")
    if not args.no_full_newton:
        line["full_newton"] = full_newton(args, dev)
        log("full-Newton workload done")
        line["preconditioners"] = preconditioners(args, dev)
        log("preconditioner comparison done")
    if not args.no_batched:
        line["batched"] = batched(args, dev)
        log("batched workload done")
    if not args.no_3d:
        line["d3"] = d3_workload(args, dev)
        log("3-D workload done")
    if oracle_timing is not None:
        line["cpu_baseline"] = oracle_timing
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
