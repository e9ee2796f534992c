"""Train and evaluate the learned warm start on the 256^2 Gaussian-blob problems.

    python -m paper_1604_02153_amd.train_unet --out unet_gauss256.bin [--train-pairs 20000]
        [--epochs 8] [--eval-pairs 1000] [--time-limit 600]

1. Data: pairs p = train_seed0 ... (the 'gauss256' recipe: 32 isotropic Gaussians, a 16-mode
   |k| <= 4 velocity of amplitude 0.3, seed p; m_R = m_T transported by that velocity), solved by
   the plain method (mixed precision, H2, beta = 1e-3, P_2L, Newton-PCG to ||g||_rel <= 1e-2) in
   batches of 64 on the GPU.  The targets are the solver's velocities, not the generating ones.
2. Training: the U-Net (4 levels, 32 base channels, BF16 on the matrix cores) on mean squared
   error against the solved velocities, and its scalar head on log(beta (e_max - 1)) of the
   two-level preconditioner's Lanczos bound of each pair; Adam with a cosine learning-rate decay,
   batches drawn by a seeded permutation.  --head-only trains the head on a loaded network.
3. Evaluation on held-out pairs (eval_seed0 ...): wall time to ||g||_rel <= 1e-2 of the plain
   path (set-up with Lanczos, solve from v = 0) and of the learned path (set-up with the network:
   e_max from the head, start from its velocity; solve with the fallback to v = 0), one pair per
   context, same GPU; solve-only times are reported too.

Every step runs in the library's kernels; this script only moves tensors and calls the C ABI.
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N = 256
NT = 4
BETA = 1e-3
CHUNK = 64


def log(msg):
    print(f"[train_unet] {msg}", flush=True)


def make_pair(seed, n=N):
    """(m_T, v_gen) of the gauss256 recipe for one seed (the same draws as synth.config)."""
    import synth
    rng = np.random.default_rng(seed)
    mT = synth.gaussian_sum_isotropic(n, n, rng)
    v = synth.random_velocity(n, n, rng, modes=16, kmax=4, amplitude=0.3)
    return mT.astype(np.float32), v.astype(np.float32)


def generate(seeds, torch, dev, log_every=2048):
    """Solve every pair with the plain method; returns GPU tensors (m_R, m_T, v_star) of the pairs
    that met the stopping rule, and the solve statistics."""
    from paper_1604_02153_amd import Context
    ctx = Context(N, N, NT, reg="h2", beta=BETA, prec="mixed", pc="2l", batch=CHUNK)
    M = len(seeds)
    mR_all = torch.empty((M, N, N), dtype=torch.float32, device=dev)
    mT_all = torch.empty_like(mR_all)
    v_all = torch.empty((M, 2, N, N), dtype=torch.float32, device=dev)
    y_all = torch.empty((M,), dtype=torch.float32, device=dev)
    keep = np.zeros(M, dtype=bool)
    iters = []
    pool = cf.ThreadPoolExecutor(max_workers=8)
    chunks = [seeds[i:i + CHUNK] for i in range(0, M, CHUNK)]
    fut = [pool.submit(lambda c=c: [make_pair(s) for s in c]) for c in chunks[:2]]
    t0 = time.perf_counter()
    for k, c in enumerate(chunks):
        pairs = fut[k].result()
        if k + 2 < len(chunks):
            fut.append(pool.submit(lambda c=chunks[k + 2]: [make_pair(s) for s in c]))
        B = len(c)
        mT = torch.from_numpy(np.stack([p[0] for p in pairs])).to(dev)
        vg = torch.from_numpy(np.stack([p[1] for p in pairs])).to(dev)
        if B < CHUNK:  # pad the last chunk with copies of its first pair (results dropped)
            mT = torch.cat([mT, mT[:1].expand(CHUNK - B, N, N)])
            vg = torch.cat([vg, vg[:1].expand(CHUNK - B, 2, N, N)])
        mT = mT.contiguous()
        vg = vg.contiguous()
        mR = torch.empty_like(mT)
        ctx.transport_state(vg, mT, mR)
        ctx.set_images(mR, mT)
        emax = np.array([b[1] for b in ctx.cheb_bounds()])
        v = torch.zeros_like(vg)
        reps = ctx.newton_solve(v)
        sl = slice(k * CHUNK, k * CHUNK + B)
        mR_all[sl] = mR[:B]
        mT_all[sl] = mT[:B]
        v_all[sl] = v[:B]
        y_all[sl] = torch.from_numpy(np.log(BETA * (emax[:B] - 1.0)).astype(np.float32)).to(dev)
        for j in range(B):
            ok = reps[j]["status"] == "SLNK_OK" and reps[j]["grel"][-1] <= 1e-2
            keep[k * CHUNK + j] = ok
            iters.append((reps[j]["newton_iters"], reps[j]["pcg_iters"]))
        if (k + 1) * CHUNK % log_every < CHUNK:
            log(f"solved {min((k + 1) * CHUNK, M)}/{M} pairs ({time.perf_counter() - t0:.1f} s)")
    pool.shutdown()
    ctx.close()
    idx = torch.from_numpy(np.nonzero(keep)[0]).to(dev)
    stats = {"pairs": M, "kept": int(keep.sum()), "solve_s": round(time.perf_counter() - t0, 1),
             "newton_mean": float(np.mean([a for a, _ in iters])), "pcg_mean": float(np.mean([b for _, b in iters]))}
    return mR_all[idx], mT_all[idx], v_all[idx], y_all[idx], stats


def train(net, data, epochs, batch, lr0, seed, time_limit, torch, dev, head_only=False):
    mR, mT, vs, ys = data
    M = mR.shape[0]
    steps_per_epoch = M // batch
    total = epochs * steps_per_epoch
    g = torch.Generator().manual_seed(seed)
    t0 = time.perf_counter()
    history, hist_h = [], []
    step = 0
    for ep in range(epochs):
        perm = torch.randperm(M, generator=g).to(dev)
        run = hrun = 0.0
        for s in range(steps_per_epoch):
            idx = perm[s * batch:(s + 1) * batch]
            warm = min(1.0, (step + 1) / 200.0)
            lr = lr0 * warm * (0.05 + 0.95 * 0.5 * (1.0 + math.cos(math.pi * step / max(1, total))))
            loss, hloss = net.train_step(mR[idx].contiguous(), mT[idx].contiguous(),
                                         None if head_only else vs[idx].contiguous(), lr,
                                         head_target=ys[idx].contiguous())
            run += loss
            hrun += hloss
            step += 1
            if step % 250 == 0:
                log(f"epoch {ep} step {step}/{total} loss {run / (s + 1):.4e} head {hrun / (s + 1):.4e} "
                    f"({time.perf_counter() - t0:.1f} s)")
            if time.perf_counter() - t0 > time_limit:
                break
        history.append(run / max(1, s + 1))
        hist_h.append(hrun / max(1, s + 1))
        log(f"epoch {ep} mean loss {history[-1]:.4e} head {hist_h[-1]:.4e}")
        if time.perf_counter() - t0 > time_limit:
            log("time limit reached")
            break
    return {"steps": step, "epochs_done": len(history), "loss_per_epoch": history, "head_loss_per_epoch": hist_h,
            "train_s": round(time.perf_counter() - t0, 1), "ms_per_step": round(1e3 * (time.perf_counter() - t0) / max(1, step), 2)}


def evaluate(net, seeds, torch, dev):
    """Plain vs learned solve of each held-out pair on a one-pair context (same GPU)."""
    from paper_1604_02153_amd import Context
    ctx = Context(N, N, NT, reg="h2", beta=BETA, prec="mixed", pc="2l")
    rows = []
    v = torch.zeros((2, N, N), dtype=torch.float32, device=dev)
    for i, s in enumerate(seeds):
        mT, vg = make_pair(s)
        mT, vg = torch.from_numpy(mT).to(dev), torch.from_numpy(vg).to(dev)
        mR = torch.empty_like(mT)
        ctx.transport_state(vg, mT, mR)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.set_images(mR, mT)
        v.zero_()
        ts = time.perf_counter()
        plain = ctx.newton_solve(v)
        t1 = time.perf_counter()
        ctx.set_images_learned(net, mR, mT)
        tl = time.perf_counter()
        learned = ctx.newton_solve_learned(net, v)
        t2 = time.perf_counter()
        ratio = (learned["emax"] - 1.0) / (plain["emax"] - 1.0)
        rows.append(dict(plain_ms=1e3 * (t1 - t0), learned_ms=1e3 * (t2 - t1),
                         plain_solve_ms=1e3 * (t1 - ts), learned_solve_ms=1e3 * (t2 - tl),
                         plain_newton=plain["newton_iters"], learned_newton=learned["newton_iters"],
                         plain_pcg=plain["pcg_iters"], learned_pcg=learned["pcg_iters"],
                         plain_ok=plain["grel"][-1] <= 1e-2, learned_ok=learned["grel"][-1] <= 1e-2,
                         fallback=learned["fallback"], emax_ratio=ratio,
                         plain_reest=plain["cheb_reestimates"] > 0,
                         learned_reest=learned["cheb_reestimates"] > 0))
        if (i + 1) % 200 == 0:
            log(f"evaluated {i + 1}/{len(seeds)}")
    ctx.close()
    col = lambda k: np.array([r[k] for r in rows], dtype=np.float64)
    return {
        "pairs": len(rows),
        "plain_ms_median": round(float(np.median(col("plain_ms"))), 2),
        "plain_solve_ms_median": round(float(np.median(col("plain_solve_ms"))), 2),
        "learned_solve_ms_median": round(float(np.median(col("learned_solve_ms"))), 2),
        "learned_ms_median": round(float(np.median(col("learned_ms"))), 2),
        "plain_ms_mean": round(float(np.mean(col("plain_ms"))), 2),
        "learned_ms_mean": round(float(np.mean(col("learned_ms"))), 2),
        "plain_newton_mean": round(float(np.mean(col("plain_newton"))), 2),
        "learned_newton_mean": round(float(np.mean(col("learned_newton"))), 2),
        "plain_pcg_mean": round(float(np.mean(col("plain_pcg"))), 2),
        "learned_pcg_mean": round(float(np.mean(col("learned_pcg"))), 2),
        "plain_reached": int(col("plain_ok").sum()), "learned_reached": int(col("learned_ok").sum()),
        "fallback_rate": round(float(np.mean(col("fallback"))), 4),
        # solves in which PCG met r.z <= 0 and re-estimated e_max by Lanczos
        "cheb_reestimate_rate_learned": round(float(np.mean(col("learned_reest"))), 4),
        "cheb_reestimate_rate_plain": round(float(np.mean(col("plain_reest"))), 4),
        "learned_faster_fraction": round(float(np.mean(col("learned_ms") < col("plain_ms"))), 4),
        "emax_ratio_learned_over_lanczos": {q: round(float(np.percentile(col("emax_ratio"), p)), 4)
                                            for q, p in (("p5", 5), ("median", 50), ("p95", 95))},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None, help="weights file to write (required unless --eval-only)")
    ap.add_argument("--train-pairs", type=int, default=20000)
    ap.add_argument("--train-seed0", type=int, default=100000)
    ap.add_argument("--eval-pairs", type=int, default=1000)
    ap.add_argument("--eval-seed0", type=int, default=200000)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0xC0FFEE)
    ap.add_argument("--time-limit", type=float, default=600.0, help="training wall-time budget (s)")
    ap.add_argument("--init", default=None, help="weights to start from")
    ap.add_argument("--start-kmax", type=int, default=8, help="Fourier cut-off of the learned start")
    ap.add_argument("--head-only", action="store_true", help="train only the e_max head of a loaded network")
    ap.add_argument("--report", default=None, help="JSON file for the statistics")
    ap.add_argument("--eval-only", action="store_true", help="evaluate the --init weights on the held-out pairs only")
    args = ap.parse_args()
    if args.eval_only and not args.init:
        ap.error("--eval-only needs --init")
    if not args.eval_only and not args.out:
        ap.error("--out is required")
    import torch
    from paper_1604_02153_amd import UNet
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.eval_only:
        net = UNet(N, N, 4, 32, max_batch=args.batch, seed=args.seed, start_kmax=args.start_kmax)
        net.load(args.init)
        estats = evaluate(net, list(range(args.eval_seed0, args.eval_seed0 + args.eval_pairs)), torch, dev)
        rep = {"weights": args.init, "evaluation": estats}
        if args.report:
            with open(args.report, "w") as f:
                json.dump(rep, f, indent=1)
        print(json.dumps(rep), flush=True)
        net.close()
        return
    seeds = list(range(args.train_seed0, args.train_seed0 + args.train_pairs))
    log(f"generating and solving {len(seeds)} training pairs")
    mR, mT, vs, ys, gstats = generate(seeds, torch, dev)
    log(f"data: {gstats}")
    net = UNet(N, N, 4, 32, max_batch=args.batch, seed=args.seed, start_kmax=args.start_kmax)
    if args.init:
        net.load(args.init)
    tstats = train(net, (mR, mT, vs, ys), args.epochs, args.batch, args.lr, args.seed, args.time_limit, torch, dev,
                   head_only=args.head_only)
    log(f"training: {tstats}")
    net.save(args.out)
    del mR, mT, vs, ys
    torch.cuda.empty_cache()
    eseeds = list(range(args.eval_seed0, args.eval_seed0 + args.eval_pairs))
    estats = evaluate(net, eseeds, torch, dev)
    log(f"evaluation: {estats}")
    rep = {"data": gstats, "training": tstats, "evaluation": estats}
    if args.report:
        with open(args.report, "w") as f:
            json.dump(rep, f, indent=1)
    print(json.dumps(rep), flush=True)
    net.close()


if __name__ == "__main__":
    main()
