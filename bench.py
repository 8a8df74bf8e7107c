"""Benchmark: batched block solves D_Lambda^{-1} b on one MI355X.

Default workload (c5): the block-local multi-boson action of eq. (localMB) on
a 64^4 lattice (antiperiodic time, SU(3) links exp(0.2 i H) drawn on the GPU
from seed 5101, kappa = 0.1365): 4096 blocks Omega of 8^4 with inner
Lambda_0 of 6^4, 12 boson fields (N = 24, c = 0.5), chi and xi Gaussian
(seeds 5102, 5103).  One step = one dd_multiboson_action call: 49 152
independent block solves D_Omega^{-1} xi_k to a per-pair FP64 true relative
residual <= 1e-10, then the boundary norms.  Headline form: FP32 even-odd
BiCGStab inner solves inside FP64 defect correction; plain FP64 solves and
FP32 solves right-preconditioned by a network trained on this lattice are
timed beside it.

--workload c2: 32^4 lattice, 256 blocks of 8^4, 12 sources per block (3072
solves per step), FP32 BiCGStab inside FP64 defect correction.
--workload c3: 48^3 x 96 lattice, 2160 uneven blocks (1296 of 8^4 and 864 of
8^3 x 12), 12 sources per block, persistent autotuned GMRES(16) with BF16
links.  --workload c4: the learned preconditioner's training and gain test.
--workload dlam: y = D_Lambda x alone (the one-pass walk) on the 64^4 blocks, 12 rhs.
--workload nnapply: the network preconditioner's forward pass alone.
--workload global: the global pieces of Section 4 on a 48^4 lattice (the rest
S^r_MB, W_z chi on dPi, the field generation chi = W_u^{-1} eta, the ln W_N
estimate), 4 fields, kappa 0.12.
--workload exterior: the exact sources xi from chi (exterior hops) on the 64^4 blocks.
--workload logdet: per-block log-determinants of 4096 blocks of 4^4.

The timed steps run the library's default path (inner iterations replayed
from captured hipGraphs, no kernel timers); one extra step with the kernel
timers on (HIP events around every launch on the library's stream) gives the
dominant kernel's algorithmic bandwidth for the roofline object.  Inputs are
resident in HBM before timing; links are packed once before timing.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-nn] [--workload c5|c2|c3|c4|dlam|nnapply|global|exterior|logdet]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "block D_Λ solves/sec at 1e-10 rel. residual; Dslash HBM GB/s vs peak"
HBM_PEAK_GBS = 8000.0

TOL = 1e-10
WORKLOADS = {
    "c2": dict(L=(32, 32, 32, 32), kappa=0.1355, eps=0.3, seed_u=2101, seed_src=2102, segs=[[8] * 4] * 4, nrhs=12,
               method="bicgstab", inner="f32",
               text="32^4 lattice, 256 blocks of 8^4 (Dirichlet), 12 rhs per block, kappa 0.1355, SU(3) links "
                    "exp(0.3 i H); %s eo-BiCGStab inner solves, FP64 defect correction, per-pair FP64 true "
                    "relative residual <= 1e-10"),
    "c3": dict(L=(96, 48, 48, 48), kappa=0.1355, eps=0.3, seed_u=3101, seed_src=3102,
               segs=[[12, 8, 12, 8, 12, 8, 12, 8, 8, 8]] + [[8] * 6] * 3, nrhs=12, method="gmres", inner="bf16",
               text="48^3 x 96 lattice, 2160 uneven blocks (1296 of 8^4, 864 of 8^3 x 12, Dirichlet), 12 rhs per "
                    "block, kappa 0.1355, SU(3) links exp(0.3 i H); persistent autotuned GMRES(16) inner solves "
                    "(%s), FP64 defect correction, per-pair FP64 true relative residual <= 1e-10"),
}


def _block_sites(L, segs):
    """Tiles in the library's block order (direction 3 fastest) as boxes
    [origin, extent], and the lattice sites of all blocks, each block in
    box-local canonical order (x3 fastest)."""
    starts = [np.concatenate([[0], np.cumsum(s)[:-1]]) for s in segs]
    boxes, sites = [], []
    for i0 in range(len(segs[0])):
        for i1 in range(len(segs[1])):
            for i2 in range(len(segs[2])):
                for i3 in range(len(segs[3])):
                    o = [int(starts[m][i]) for m, i in enumerate((i0, i1, i2, i3))]
                    e = [int(segs[m][i]) for m, i in enumerate((i0, i1, i2, i3))]
                    boxes.append(o + e)
                    y = np.indices(e).reshape(4, -1).T + np.array(o)
                    sites.append(((y[:, 0] * L[1] + y[:, 1]) * L[2] + y[:, 2]) * L[3] + y[:, 3])
    return np.asarray(boxes), np.concatenate(sites)


def _inputs(w):
    """Links on the host; sources in block order, on the GPU."""
    import torch

    import synth

    U = synth.gauge_field(w["L"], w["eps"], w["seed_u"])
    boxes, sites = _block_sites(w["L"], w["segs"])
    if w is WORKLOADS["c2"]:
        src = synth.spinor_field(w["L"], w["nrhs"], w["seed_src"])[:, sites]
        b = torch.from_numpy(np.ascontiguousarray(src)).cuda()
    else:
        # too large to draw on the host: iid Gaussian sources drawn directly in block order
        b = synth.spinor_field_device(w["nrhs"], len(sites), w["seed_src"])
    return U, b, boxes


def cpu_baseline(w, U, b, boxes):
    """The oracle's FP64 block solve (OpenMP over pairs) on a bounded sample."""
    from oracle import wilson

    nthr = wilson.num_threads()
    nb = len(boxes)
    npairs = max(1, min(8 * nthr, nb * w["nrhs"]))  # about 10-30 s of CPU work
    S = np.array([int(np.prod(bx[4:8])) for bx in boxes])
    off = np.concatenate([[0], np.cumsum(S)])
    pick = [((k * 37) % nb, k % w["nrhs"]) for k in range(npairs)]
    sel_boxes = np.asarray([boxes[blk] for blk, _ in pick])
    bh = np.concatenate([b[r, off[blk]:off[blk + 1]].cpu().numpy() for blk, r in pick])[None]
    t0 = time.perf_counter()
    _, iters, rel, fails = wilson.solve_many(w["L"], -1, w["kappa"], U, sel_boxes, bh, tol=TOL, nthreads=nthr)
    dt = time.perf_counter() - t0
    return {"value": npairs / dt, "unit": "solves/s", "cores": nthr, "cpu_model": cpu_model(), "kind": "oracle",
            "sample": "%d (block, rhs) pairs of the same workload (8 per thread), FP64 eo-BiCGStab with FP64 "
                      "defect correction to 1e-10 (%.1f s wall, %d failed)" % (npairs, dt, fails)}


def net_roofline(net, n_blocks, reps=5):
    """BF16 network applications on n_blocks blocks of random rows, timed with HIP events on the
    library's stream (dd_nn_apply synchronizes that stream before returning): (total ms, launches,
    total flops)."""
    import torch

    x = torch.randn(n_blocks, net.sites, 24, dtype=torch.float32, device="cuda")
    net.apply(x, prec="bf16")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        net.apply(x, prec="bf16")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt * 1e3, reps, reps * 2.0 * 81 * (24 * 32 + 32 * 32 + 32 * 24) * n_blocks * net.sites


def run_nnapply(args):
    """The network's BF16 application alone: 1024 blocks of 8^4 random rows (an untrained network),
    `--steps` timed applications after one warm-up."""
    import torch

    import synth
    from paper_2211_06902_amd import dd

    ctx = dd.Context(0)
    net = ctx.nn_create((8, 8, 8, 8), synth.convnet_weights(5))
    ms, n, flops = net_roofline(net, 1024, reps=args.steps)
    achieved = flops / (ms * 1e-3) / 1e12
    print(json.dumps({
        "metric": "network application throughput", "value": achieved, "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": 1, "ms_per_step": ms / n, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "24-32-32-24 3^4 conv net, BF16 matrix-core inference on 1024 blocks of 8^4 "
                               "(414 720 flop per site), wall time around dd_nn_apply"},
        "roofline": {"kernel": "k_conv_mfma_lds", "bound": "mfma", "achieved": achieved, "peak": 2500.0,
                     "unit": "TFLOP/s", "frac": achieved / 2500.0, "traffic": None},
    }), flush=True)
    net.close()
    ctx.close()


def run_c4(args):
    """The learned preconditioner: train the network on ~20k (source, D^{-1} source) pairs of the
    32^4 lattice's 8^4 blocks (sources on even sites, made by the block solver), then solve fresh
    sources on a held-out gauge field with FGMRES(16) + network against plain GMRES(16)."""
    import torch

    import synth
    from paper_2211_06902_amd import dd

    L, kappa, eps = (32, 32, 32, 32), 0.1355, 0.3
    V = 32**4
    n_tr, n_va = 70, 8  # rhs per block: 70 x 256 = 17 920 training and 2048 validation pairs
    ctx = dd.Context(0)
    blk = ctx.make_blocks(L, -1, [[8] * 4] * 4)
    t0 = time.perf_counter()
    g = ctx.load_gauge(blk, torch.from_numpy(synth.gauge_field(L, eps, 2101)).cuda(), "f32")
    odd = torch.from_numpy(np.indices((8, 8, 8, 8)).sum(axis=0).reshape(-1) % 2 == 1).cuda()
    src = synth.spinor_field_device(n_tr + n_va, V, 4100)
    src.view(n_tr + n_va, 256, 4096, 4, 3)[:, :, odd] = 0
    sol = torch.empty_like(src)
    p_gen = dd.solve_params(inner_prec="f32")
    for c in range(0, n_tr + n_va, 12):
        _, _, st = ctx.block_solve(blk, g, kappa, src[c:c + 12], sol[c:c + 12], params=p_gen)
        if st != dd.DD_OK:
            raise SystemExit("training-pair solve did not converge")
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    g.close()

    print("c4: %d training + %d validation pairs solved in %.1f s" % (n_tr * 256, n_va * 256, t_pairs),
          file=sys.stderr, flush=True)
    net = ctx.nn_create((8, 8, 8, 8), synth.convnet_weights(4100))
    t0 = time.perf_counter()
    tl, vl = [], []
    for ep in range(args.epochs):  # one epoch per call (shuffle stream seed 4100 + epoch)
        tp = dd.nn_train_params(epochs=1, batch=32, lr=1e-3, seed=4100 + ep)
        a, v = net.train(blk, src[:n_tr], sol[:n_tr], n_tr, src[n_tr:], sol[n_tr:], n_va, params=tp)
        tl.append(float(a[0]))
        vl.append(float(v[0]))
        print("c4: epoch %d train loss %.5f val loss %.5f (%.1f s)" % (ep, a[0], v[0], time.perf_counter() - t0),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del src, sol
    torch.cuda.empty_cache()

    # held-out gauge field, fresh sources
    g2 = ctx.load_gauge(blk, torch.from_numpy(synth.gauge_field(L, eps, 4201)).cuda(), "f32")
    b = synth.spinor_field_device(12, V, 4202)
    x = torch.empty_like(b)
    runs = {
        "gmres16": dd.solve_params(method=dd.GMRES, restart=16, inner_prec="f32"),
        "fgmres16_nn_every_cycle": dd.solve_params(method=dd.GMRES, restart=16, inner_prec="f32", precond=net,
                                                   precond_cycles=1),
        "fgmres16_nn_once": dd.solve_params(method=dd.GMRES, restart=16, inner_prec="f32", precond=net,
                                            precond_cycles=0),
        "bicgstab": dd.solve_params(inner_prec="f32"),
        "bicgstab_nn": dd.solve_params(inner_prec="f32", precond=net),
    }
    res = {}
    for name, prm in runs.items():
        ctx.block_solve(blk, g2, kappa, b, x, params=prm)  # warm-up
        ctx.timer_enable(True)
        ctx.timer_reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ok, steps = True, []
        for _ in range(args.steps):
            _, info, st = ctx.block_solve(blk, g2, kappa, b, x, params=prm)
            ok = ok and st == dd.DD_OK and bool(np.all(info["true_relres"] <= TOL))
            steps.append(float(info["iters"].mean()))
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        ctx.timer_enable(False)
        res[name] = {"solves_per_s": 3072 / dt if ok else 0.0, "ms_per_step": dt * 1e3, "all_converged": ok,
                     "mean_inner_steps_per_pair": steps[-1]}
        print("c4: %s %s" % (name, res[name]), file=sys.stderr, flush=True)
    nn_ms, nn_n, nn_flops = net_roofline(net, 3072)
    achieved = nn_flops / (nn_ms * 1e-3) / 1e12 if nn_ms > 0 else 0.0
    best = res["bicgstab_nn"]
    out = {
        "metric": METRIC,
        "value": best["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 1,
        "ms_per_step": best["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "learned preconditioner: 24-32-32-24 3^4 conv net (FP32 training, BF16 matrix-core "
                        "inference) trained on 17 920 (source, D^{-1} source) pairs of the 32^4 lattice's 8^4 blocks "
                        "(links exp(0.3 i H) seed 2101, kappa 0.1355, sources on even sites), validated on 2048; "
                        "tested on a held-out gauge field (seed 4201), 12 fresh sources per block, FP32 inner "
                        "BiCGStab right-preconditioned by the network (value) against plain BiCGStab, and FGMRES(16) "
                        "+ network against plain GMRES(16), FP64 defect correction to 1e-10",
            "pairs_generation_s": t_pairs,
            "training_s": t_train,
            "epochs": args.epochs,
            "train_loss": [round(v, 5) for v in tl],
            "val_loss": [round(v, 5) for v in vl],
            "solvers": res,
        },
        "roofline": {
            "kernel": "k_conv_mfma_lds (network application on 3072 blocks of 8^4: 3 BF16 matrix-core launches, "
                      "414 720 flop per site; wall time around dd_nn_apply)",
            "bound": "mfma",
            "achieved": achieved,
            "peak": 2500.0,
            "unit": "TFLOP/s",
            "frac": achieved / 2500.0,
            "traffic": None,
            "launches": nn_n,
            "avg_launch_us": nn_ms * 1e3 / max(nn_n, 1),
        },
    }
    print(json.dumps(out), flush=True)
    net.close()
    g2.close()
    blk.close()
    ctx.close()


C5 = dict(L=(64, 64, 64, 64), kappa=0.1365, eps=0.2, nf=12, N=24, c=0.5, seed_u=5101, seed_chi=5102, seed_xi=5103,
          seed_nn=5104)


CLOVER_CSW = 1.6  # c_sw of the clover form timed beside the headline


def _mb_inputs(ctx, dd):
    """The 64^4 lattice's blocks, packed links and multi-boson fields, all drawn on the GPU; the
    canonical links are kept on the host for the oracle's sample."""
    import torch

    import synth

    w = C5
    V = 64**4
    blk = ctx.make_blocks(w["L"], -1, [[8] * 8] * 4, inner_d=1)
    U = synth.gauge_field_device(w["L"], w["eps"], w["seed_u"])
    torch.cuda.synchronize()
    t = time.perf_counter()
    g = ctx.load_gauge(blk, U, "f32")  # packing: FP64 and FP32 link records of every block
    torch.cuda.synchronize()
    _mb_inputs.pack_s = time.perf_counter() - t
    U_host = U.cpu().numpy()
    del U
    torch.cuda.empty_cache()  # the library sizes its field groups by the free device memory
    chi = synth.spinor_field_device(w["nf"], blk.total_bnd_sites, w["seed_chi"])
    xi = synth.spinor_field_device(w["nf"], V, w["seed_xi"])
    u = dd.mb_roots(w["N"], w["c"])
    return blk, g, U_host, chi, xi, u


def _mb_train_net(ctx, dd, blk, g, epochs):
    """A network for this lattice: FP32 training on (even source, block solution) pairs of its blocks
    made by the block solver (4 sources per block, 16 384 pairs)."""
    import torch

    import synth

    w = C5
    n_tr = 4
    odd = torch.from_numpy(np.indices((8, 8, 8, 8)).sum(axis=0).reshape(-1) % 2 == 1).cuda()
    src = synth.spinor_field_device(n_tr, 64**4, w["seed_nn"])
    src.view(n_tr, 4096, 4096, 4, 3)[:, :, odd] = 0
    sol = torch.empty_like(src)
    _, _, st = ctx.block_solve(blk, g, w["kappa"], src, sol, params=dd.solve_params(inner_prec="f32"))
    if st != dd.DD_OK:
        raise SystemExit("training-pair solve did not converge")
    net = ctx.nn_create((8, 8, 8, 8), synth.convnet_weights(w["seed_nn"]))
    tl = []
    for ep in range(epochs):
        a, _ = net.train(blk, src, sol, n_tr,
                         params=dd.nn_train_params(epochs=1, batch=32, lr=1e-3, seed=w["seed_nn"] + ep))
        tl.append(float(a[0]))
    del src, sol
    torch.cuda.empty_cache()
    return net, tl


def mb_cpu_baseline(U_host, xi):
    """The oracle's FP64 block solve (OpenMP over pairs) on a bounded sample of the 64^4 workload's
    (block, field) pairs: the same xi sources, FP64 eo-BiCGStab with FP64 defect correction to 1e-10."""
    from oracle import wilson

    nthr = wilson.num_threads()
    w = C5
    npairs = 8 * nthr  # about 10-30 s of CPU work
    nb, S = 4096, 4096
    pick = [((k * 977) % nb, k % w["nf"]) for k in range(npairs)]
    boxes = []
    for blk, _ in pick:
        t = [(blk >> (3 * (3 - m))) & 7 for m in range(4)]  # tile coordinates, direction 3 fastest
        boxes.append([8 * v for v in t] + [8, 8, 8, 8])
    bh = np.concatenate([xi[f, blk * S:(blk + 1) * S].cpu().numpy() for blk, f in pick])[None]
    t0 = time.perf_counter()
    _, iters, rel, fails = wilson.solve_many(w["L"], -1, w["kappa"], U_host, np.asarray(boxes), bh, tol=TOL,
                                             nthreads=nthr)
    dt = time.perf_counter() - t0
    # context: the oracle's D_Lambda on one 8^4 block (one thread, FP64, one rhs) for about a second,
    # with the algorithmic bytes S 48 s_f + L_in 18 s_l per application
    o, e = np.asarray(boxes[0][:4]), np.asarray(boxes[0][4:])
    psi = bh[0, :S]
    napp, t1 = 0, time.perf_counter()
    while napp == 0 or time.perf_counter() - t1 < 1.0:
        wilson.dirac_box(w["L"], -1, w["kappa"], U_host, o, e, psi)
        napp += 1
    dt1 = time.perf_counter() - t1
    dslash = napp * (S * 48 * 8 + 4 * 8**3 * 7 * 18 * 8) / dt1 / 1e9
    return {"value": npairs / dt, "unit": "solves/s", "cores": nthr, "cpu_model": cpu_model(), "kind": "oracle",
            "sample": "%d (block, field) pairs of the 64^4 multi-boson workload (8 per thread; xi sources of "
                      "%d blocks), FP64 eo-BiCGStab with FP64 defect correction to 1e-10 (%.1f s wall, "
                      "%d failed)" % (npairs, len(set(b for b, _ in pick)), dt, fails),
            "dslash_GBs_one_thread": dslash,
            "dslash_sample": "%d applications of D_Lambda (FP64, one rhs) on one 8^4 block in %.2f s, one thread"
                             % (napp, dt1)}


def solve_byte_model(blk, info, inner, seconds):
    """The evaluation against the byte model of eo-BiCGStab: per pair and iteration two Dhat, each
    two eo hops (S 24 s_f spinor bytes, every link inside the block once at 18 s_l, the links shared
    by the pairs of one launch) and an axpy (S 12 s_f), plus 14 half-field passes of vector updates
    (S 12 s_f each), i.e. S 288 s_f + 72 L_in s_l / (pairs per launch) bytes per pair and iteration,
    summed over every pair's iterations; the FP64 defect-correction passes are left out.  The
    library fuses several of the 14 passes into the Dhat walks, so the effective bandwidth can
    exceed the stencil kernel's own."""
    sf = 8.0 if inner == "f64" else 4.0
    sl = {"f64": 8.0, "f32": 4.0, "bf16": 2.0}[inner]
    S = blk.total_sites / blk.n_blocks
    L_in = blk.inner_links / blk.n_blocks
    pair_its = float(np.sum(info["iters"]))
    per = S * 288.0 * sf + 72.0 * L_in * sl / max(int(info["rhs_per_solve"]), 1)
    total = pair_its * per
    eff = total / seconds / 1e9
    return {"pair_iterations": pair_its, "bytes_per_pair_iteration": per, "bytes_per_evaluation": total,
            "t_min_s": total / (HBM_PEAK_GBS * 1e9), "effective_GBs": eff, "frac_of_peak": eff / HBM_PEAK_GBS}


def run_c5(args):
    """The default workload: the block-local multi-boson action of the 64^4 lattice, 4096 blocks
    Omega of 8^4 (inner Lambda_0 of 6^4), 12 boson fields (N = 24, c = 0.5), one D_Omega^{-1} xi_k
    solve per field and block (49 152 solves per evaluation).  The headline is the fastest form
    that brings every pair to 1e-10 (FP32 inner BiCGStab, FP64 defect correction); plain FP64
    solves, FP32 solves right-preconditioned by a network trained on this lattice, and the same
    workload with the clover term are measured beside it."""
    import torch

    from paper_2211_06902_amd import dd

    w = C5
    say = lambda m: print("c5: " + m, file=sys.stderr, flush=True)  # noqa: E731
    t0 = time.perf_counter()
    ctx = dd.Context(0)
    blk, g, U_host, chi, xi, u = _mb_inputs(ctx, dd)
    t_gen = time.perf_counter() - t0
    say("inputs ready (%.1f s)" % t_gen)
    n_solves = blk.n_blocks * w["nf"]
    inner = args.inner or "f32"

    def evaluate(prm):
        S, tot, info, st = ctx.multiboson_action(blk, g, w["kappa"], u, chi, xi, params=prm)
        ok = st == dd.DD_OK and bool(np.all(info["true_relres"] <= TOL))
        return tot, info, ok

    def timed(prm, steps, warmup):
        """Wall time of `steps` evaluations after `warmup` untimed ones, with the library's default
        path (inner iterations replayed from a captured graph, no kernel timers)."""
        for _ in range(warmup):
            evaluate(prm)
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = [evaluate(prm) for _ in range(steps)]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        return dt, res

    head = dd.solve_params(inner_prec=inner, use_graph=0 if args.no_graph else 1)
    dt, res = timed(head, args.steps, args.warmup)
    ok = all(r[2] for r in res)
    S_head = res[-1][0]
    say("%s: %.3f s per evaluation, all converged %s" % (inner, dt / args.steps, ok))

    # one more evaluation with the kernel timers on (events around every launch, graph replay off):
    # the stencil kernel's time and algorithmic bytes for the roofline
    ctx.timer_enable(True)
    ctx.timer_reset()
    evaluate(head)
    kname, (k_ms, k_n, k_bytes) = stencil_timer(ctx, inner)
    ctx.timer_enable(False)
    achieved = k_bytes / (k_ms * 1e-3) / 1e9 if k_ms > 0 else 0.0

    forms = {}
    side = max(1, min(args.steps, 2))
    if inner != "f64" and not args.only_head:
        dt64, r64 = timed(dd.solve_params(inner_prec="f64"), side, 1)
        forms["fp64"] = {"solves_per_s": n_solves * side / dt64 if all(r[2] for r in r64) else 0.0,
                         "s_per_evaluation": dt64 / side, "all_converged": all(r[2] for r in r64),
                         "S_rel_diff_vs_headline": abs(r64[-1][0] - S_head) / abs(S_head)}
        say("fp64 %s" % forms["fp64"])
    if not args.no_nn and not args.only_head:
        t1 = time.perf_counter()
        net, tl = _mb_train_net(ctx, dd, blk, g, args.epochs)
        t_train = time.perf_counter() - t1
        dtn, rn = timed(dd.solve_params(inner_prec="f32", precond=net), side, 1)
        forms["fp32_nn"] = {"solves_per_s": n_solves * side / dtn if all(r[2] for r in rn) else 0.0,
                            "s_per_evaluation": dtn / side, "all_converged": all(r[2] for r in rn),
                            "S_rel_diff_vs_headline": abs(rn[-1][0] - S_head) / abs(S_head),
                            "training_s": t_train, "train_loss": [round(v, 5) for v in tl],
                            "mean_inner_iterations_per_pair": float(rn[-1][1]["iters"].mean())}
        say("fp32_nn %s" % forms["fp32_nn"])
        net.close()
    if inner != "f64" and not args.only_head:
        # the same workload with the Sheikholeslami-Wohlert term (c_sw = 1.6): another operator, so its
        # action is not the headline's; the term is removed again afterwards
        U_dev = torch.from_numpy(U_host).cuda()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g.set_clover(U_dev, w["kappa"], CLOVER_CSW)
        torch.cuda.synchronize()
        t_cl = time.perf_counter() - t1
        del U_dev
        torch.cuda.empty_cache()
        dtc, rcl = timed(dd.solve_params(inner_prec=inner), side, 1)
        forms["clover"] = {"c_sw": CLOVER_CSW,
                           "solves_per_s": n_solves * side / dtc if all(r[2] for r in rcl) else 0.0,
                           "s_per_evaluation": dtc / side, "all_converged": all(r[2] for r in rcl),
                           "clover_build_s": t_cl, "outer_cycles": int(rcl[-1][1]["outer_cycles"]),
                           "mean_inner_iterations_per_pair": float(rcl[-1][1]["iters"].mean())}
        say("clover %s" % forms["clover"])
        g.set_clover(None, w["kappa"], 0.0)

    value = n_solves * args.steps / dt if ok else 0.0
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": inner,
        "data": "synthetic",
        "config": {
            "workload": "multi-boson local action (eq. localMB) on a 64^4 lattice (antiperiodic time; SU(3) links "
                        "exp(0.2 i H) drawn on the GPU from seed 5101; kappa 0.1365): 4096 blocks Omega of 8^4 "
                        "(Dirichlet) with inner Lambda_0 of 6^4 (1040 boundary sites), 12 boson fields (N = 24, "
                        "c = 0.5), chi on dLambda_0 and xi on Omega Gaussian (seeds 5102, 5103); one evaluation = "
                        "49 152 block solves to per-pair FP64 true relative residual <= 1e-10 plus the boundary "
                        "norms; %s inner eo-BiCGStab inside FP64 defect correction" % inner.upper(),
            "solves_per_step": n_solves,
            "all_converged": ok,
            "S_total": S_head,
            "mean_inner_iterations_per_pair": float(res[-1][1]["iters"].mean()),
            "outer_cycles": int(res[-1][1]["outer_cycles"]),
            "graph_replay": not args.no_graph,
            "fields_per_solve": int(res[-1][1]["rhs_per_solve"]),
            "input_generation_s": t_gen,
            "gauge_pack_s": getattr(_mb_inputs, "pack_s", None),
            "other_forms": forms,
        },
        "roofline": {
            "kernel": kname,
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": profiled_traffic(PROFILE_C5) if inner == "f32" else None,
            "launches": k_n,
            "avg_launch_us": k_ms * 1e3 / max(k_n, 1),
            "alg_bytes_per_launch": k_bytes / max(k_n, 1),
            "timing": "HIP events around each launch on the library stream, in one extra evaluation",
        },
    }
    out["config"]["solve_byte_model"] = solve_byte_model(blk, res[-1][1], inner, dt / args.steps)
    if "fp64" in forms and forms["fp64"]["solves_per_s"] > 0:
        out["config"]["speedup_over_fp64"] = value / forms["fp64"]["solves_per_s"]
    if not args.no_cpu:
        out["cpu_baseline"] = mb_cpu_baseline(U_host, xi)
    print(json.dumps(out), flush=True)
    g.close()
    blk.close()
    ctx.close()


PROFILE_C2 = os.path.join(ROOT, "profiles", "k_dhat_walk_f32_c2_32x4_12rhs.md")
PROFILE_C5 = os.path.join(ROOT, "profiles", "k_dhat_walk_f32_c5_64x4_12fields.md")
PROFILE_GLOBAL = os.path.join(ROOT, "profiles", "k_hop_f32_inactive_48x4_4fields.md")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def stencil_timer(ctx, inner):
    """(description, (ms, launches, bytes)) of the stencil kernel of the BiCGStab inner solves: the
    one-kernel x0-walk of Dhat when it ran, else the hop (two launches per Dhat)."""
    from paper_2211_06902_amd import dd

    dhat = {"f32": dd.KCLASS_DHAT_F32, "bf16": dd.KCLASS_DHAT_BF16}.get(inner)
    link = "FP32 spinor / BF16 link" if inner == "bf16" else inner.upper()
    if dhat is not None:
        t = ctx.timer_read(dhat)
        if t[1] > 0:
            return ("k_dhat_walk (%s; Dhat = 1 - kappa^2 H_eo H_oe as one x0-walk, the intermediate in LDS, "
                    "with the fused BiCGStab updates and dots)" % link, t)
    hop = {"f64": dd.KCLASS_HOP_F64, "f32": dd.KCLASS_HOP_F32, "bf16": dd.KCLASS_HOP_BF16}[inner]
    return ("k_hop_walk (%s; the x0-walk hop, all its fused-dot variants)" % link, ctx.timer_read(hop))


def profiled_traffic(path):
    """HBM bytes per launch of the dominant kernel from a committed rocprofv3 summary, if it was
    taken on the current kernel source (else None)."""
    try:
        from paper_2211_06902_amd.rocprof_summary import kernel_source_hash

        txt = open(path).read()
        js = json.loads(txt.split("```json", 1)[1].split("```", 1)[0])
        if js.get("kernel_source_sha256_16") != kernel_source_hash():
            return None
        return js["hbm_traffic_bytes_per_launch"]
    except (OSError, IndexError, KeyError, ValueError):
        return None


def run_dlam(args):
    """--workload dlam: y = D_Lambda x alone (dd_apply_D_block, FP32 arithmetic: pack to half
    fields, the one-pass x0-walk of D_Lambda, unpack) on the 64^4 lattice's 4096 blocks of 8^4,
    12 rhs, `--steps` timed applications after `--warmup`.  The stencil's bandwidth counts
    n_rhs * S * 48 * 4 bytes of spinors plus every link inside the blocks once as 18 reals."""
    import torch

    import synth
    from paper_2211_06902_amd import dd

    L, nr, kappa = (64, 64, 64, 64), 12, 0.1365
    ctx = dd.Context(0)
    blk = ctx.make_blocks(L, -1, [[8] * 8] * 4)
    U = synth.gauge_field_device(L, 0.2, 5101)
    g = ctx.load_gauge(blk, U, "f32")
    del U
    torch.cuda.empty_cache()
    x = synth.spinor_field_device(nr, blk.total_sites, 5103)
    y = torch.empty_like(x)
    for _ in range(max(args.warmup, 1)):
        ctx.apply_D_block(blk, g, kappa, "f32", x, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.apply_D_block(blk, g, kappa, "f32", x, y)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    ctx.timer_enable(True)
    ctx.timer_reset()
    for _ in range(args.steps):
        ctx.apply_D_block(blk, g, kappa, "f32", x, y)
    k_ms, k_n, k_bytes = ctx.timer_read(dd.KCLASS_HOP_F32)
    ctx.timer_enable(False)
    achieved = k_bytes / (k_ms * 1e-3) / 1e9 if k_ms > 0 else 0.0
    print(json.dumps({
        "metric": "block D_Lambda applications (all blocks, all rhs) per second", "value": 1.0 / dt,
        "unit": "applications/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "y = D_Lambda x on the 64^4 lattice (antiperiodic time, SU(3) links exp(0.2 i H) from "
                               "seed 5101): 4096 blocks of 8^4 (Dirichlet), 12 rhs; FP64 in and out, FP32 arithmetic "
                               "(pack, one-pass x0-walk, unpack)", "rhs": nr},
        "roofline": {"kernel": "k_dlam_walk (FP32; D_Lambda in one x0-walk over both parities)", "bound": "hbm",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "launches": k_n, "avg_launch_us": k_ms * 1e3 / max(k_n, 1),
                     "alg_bytes_per_launch": k_bytes / max(k_n, 1),
                     "timing": "HIP events around each launch on the library stream, in extra applications"},
    }), flush=True)
    g.close()
    blk.close()
    ctx.close()


def run_global(args):
    """--workload global: the global pieces of Section 4 on a 48^4 lattice of 8^4 tiles with 4^4
    active boxes (kappa 0.12, links exp(0.2 i H)), 4 fields at the u_k of N = 8, c = 0.5: the global
    rest S^r_MB (one batched solve on the inactive region), W_z chi on dPi (the block solves and the
    inactive-region solve), the field generation chi = W_u^{-1} eta (FP64 BiCGStab over dPi to 1e-10,
    inner solves to 1e-12) and the ln W_N estimate (order 1, 4 noise vectors).  `value` = generated
    fields per second; the other timings are in config."""
    import torch

    import synth
    from paper_2211_06902_amd import dd

    L, kappa, nf = (48, 48, 48, 48), 0.12, 4
    ctx = dd.Context(0)
    blk = ctx.make_blocks(L, -1, [[8] * 6] * 4, inner_d=2)
    D = ctx.make_inactive(blk)
    U = synth.gauge_field_device(L, 0.2, 7001)
    g = ctx.load_gauge(blk, U, "f32")
    gd = ctx.load_gauge(D, U, "f32")
    del U
    torch.cuda.empty_cache()
    eta = synth.spinor_field_device(nf, 48**4, 7002) / np.sqrt(2)
    u = dd.mb_roots(2 * nf, 0.5)
    prm = dd.solve_params(tol=1e-12)
    steps = max(1, min(args.steps, 2))

    def wall(fn, what):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        print(f"# global: {what} {dt:.3f} s, status {r[-1]}", file=sys.stderr, flush=True)
        return dt, r

    ctx.mb_global_action(D, gd, kappa, u, eta, params=prm)  # workspaces
    ctx.mb_apply_W(blk, g, D, gd, kappa, u, eta, params=prm)
    t_sr, (Sr, _, info_sr, st_sr) = wall(lambda: ctx.mb_global_action(D, gd, kappa, u, eta, params=prm), "S^r")
    t_w, (_, info_w, st_w) = wall(lambda: ctx.mb_apply_W(blk, g, D, gd, kappa, u, eta, params=prm), "W_z chi")
    t_gen = 0.0
    for _ in range(steps):
        dt, (chi, its, rel, info_g, st_g) = wall(lambda: ctx.mb_generate(blk, g, D, gd, kappa, u, eta, tol=1e-10,
                                                                           maxit=60, params=prm), "generation")
        t_gen += dt
    t_gen /= steps
    t_rw, (terms, est, info_rw, st_rw) = wall(lambda: ctx.mb_log_reweight(blk, g, D, gd, kappa, 2 * nf, 0.5, 1, eta,
                                                                             params=prm), "ln W_N")
    ok = all(st == dd.DD_OK for st in (st_sr, st_w, st_g, st_rw)) and bool(np.all(rel <= 1e-9))
    # one more W_z chi with the kernel timers on: the kernel classes of its two batched solves
    ctx.timer_enable(True)
    ctx.timer_reset()
    wall(lambda: ctx.mb_apply_W(blk, g, D, gd, kappa, u, eta, params=prm), "W_z chi, kernel timers on")
    names = {dd.KCLASS_HOP_F64: "k_hop (FP64; the defect-correction residuals)",
             dd.KCLASS_HOP_F32: "k_hop (FP32; the hop of the inner solves on blocks or the inactive region)",
             dd.KCLASS_DHAT_F32: "k_dhat_walk (FP32; the one-kernel Dhat of the inner solves)"}
    per = {k: ctx.timer_read(k) for k in names}
    ctx.timer_enable(False)
    top = max(per, key=lambda k: per[k][0])
    k_ms, k_n, k_bytes = per[top]
    achieved = k_bytes / (k_ms * 1e-3) / 1e9 if k_ms > 0 else 0.0
    print(json.dumps({
        "metric": "multi-boson field generations (chi = W_u^{-1} eta on dPi) per second", "value": nf / t_gen if ok else 0.0,
        "unit": "fields/s", "n_gpus": 1, "steps": steps, "warmup": 1, "ms_per_step": t_gen * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "global pieces of the multi-boson action on a 48^4 lattice (antiperiodic time, SU(3) "
                               "links exp(0.2 i H) from seed 7001, kappa 0.12): 1296 tiles of 8^4 with 4^4 active "
                               "boxes, the inactive region one solve domain; 4 fields (N = 8, c = 0.5), eta Gaussian "
                               "(seed 7002); FP32 inner solves to 1e-12, generation to 1e-10",
                   "all_ok": ok, "global_rest_s": t_sr, "S_r": [float(v) for v in Sr],
                   "apply_W_s": t_w, "generation_s": t_gen, "generation_iterations": [int(v) for v in its],
                   "generation_true_relres_max": float(rel.max()), "log_reweight_s": t_rw,
                   "log_reweight_estimate": [est.real, est.imag],
                   "apply_W_kernel_ms": {"hop_f64": per[dd.KCLASS_HOP_F64][0], "hop_f32": per[dd.KCLASS_HOP_F32][0],
                                         "dhat_walk_f32": per[dd.KCLASS_DHAT_F32][0]}},
        "roofline": {"kernel": names[top], "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": profiled_traffic(PROFILE_GLOBAL) if top == dd.KCLASS_HOP_F32 else None,
                     "launches": k_n, "ms_per_launch": k_ms / max(k_n, 1), "scope": "one W_z chi"},
    }), flush=True)
    for h in (gd, g, D, blk):
        h.close()
    ctx.close()


def run_exterior(args):
    """--workload exterior: the exact source of eq. (localMB) from chi alone, xi^a += the hops of chi
    from the sites of dPi outside each block into it (dd_mb_exterior_source, both parts), for the
    64^4 lattice's 4096 blocks of 8^4 (inner 6^4) and 12 fields, `--steps` timed calls after one.
    Algorithmic bytes per call: every exterior hop reads the field's neighbour spinor (24 doubles
    per field) and its link once (18 doubles), every receiving site reads and writes its xi entry
    (2 x 24 doubles per field)."""
    import torch

    import synth
    from paper_2211_06902_amd import dd

    w = C5
    ctx = dd.Context(0)
    blk = ctx.make_blocks(w["L"], -1, [[8] * 8] * 4, inner_d=1)
    U = synth.gauge_field_device(w["L"], w["eps"], w["seed_u"])
    g = ctx.load_gauge(blk, U, "f32")
    del U
    torch.cuda.empty_cache()
    chi = synth.spinor_field_device(w["nf"], 64**4, w["seed_chi"])
    xi = torch.zeros((w["nf"], blk.total_sites, 4, 3), dtype=torch.complex128, device="cuda")
    b, site, _, _ = blk.exterior()
    n_hops = int(b.size)
    n_recv = int(np.unique(b.astype(np.int64) * blk.total_sites + site).size)
    alg = n_hops * (24 * 8 * w["nf"] + 18 * 8) + n_recv * 2 * 24 * 8 * w["nf"]
    ctx.mb_exterior_source(blk, g, w["kappa"], chi, xi)
    torch.cuda.synchronize()
    steps = max(1, args.steps)
    t = time.perf_counter()
    for _ in range(steps):
        ctx.mb_exterior_source(blk, g, w["kappa"], chi, xi)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / steps
    achieved = alg / dt / 1e9
    print(json.dumps({
        "metric": "exact multi-boson sources xi from chi (dPi exterior hops into every block) per second",
        "value": 1.0 / dt, "unit": "sources/s (all 4096 blocks x 12 fields)", "n_gpus": 1, "steps": steps,
        "warmup": 1, "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "64^4 lattice (links exp(0.2 i H), seed 5101), 4096 blocks of 8^4 with inner 6^4, "
                               "12 Gaussian fields chi (seed 5102) on the whole lattice (read on dPi)",
                   "exterior_hops": n_hops, "receiving_sites": n_recv},
        "roofline": {"kernel": "k_mb_exterior", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "alg_bytes_per_launch": alg, "timing": "wall time of the synchronising call"},
    }), flush=True)
    g.close()
    blk.close()
    ctx.close()


def run_logdet(args):
    """--workload logdet: per-block ln det D_Lambda (dd_block_logdet, FP64) of 4096 blocks of 4^4 on a
    32^4 lattice (the largest blocks the dense route takes have 12 h <= 6144; 4^4 gives 12 h = 1536),
    `--steps` timed calls after one.  The work is dominated by the batched complex LU: (8/3) n^3 real
    flops per block with n = 12 h, set against the FP64 peak."""
    import torch

    import synth
    from paper_2211_06902_amd import dd

    L, kappa = (32, 32, 32, 32), 0.1365
    ctx = dd.Context(0)
    blk = ctx.make_blocks(L, -1, [[4] * 8] * 4)
    U = synth.gauge_field_device(L, 0.2, 6101)
    g = ctx.load_gauge(blk, U, "f32")
    del U
    ld, tot = ctx.block_logdet(blk, g, kappa)
    torch.cuda.synchronize()
    steps = max(1, min(args.steps, 3))
    t = time.perf_counter()
    for _ in range(steps):
        ld2, tot2 = ctx.block_logdet(blk, g, kappa)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / steps
    n = 12 * (blk.total_sites // blk.n_blocks) // 2
    flops = blk.n_blocks * (8.0 / 3.0) * n**3
    achieved = flops / dt / 1e12
    print(json.dumps({
        "metric": "per-block log-determinants ln det D_Lambda per second", "value": blk.n_blocks / dt,
        "unit": "blocks/s", "n_gpus": 1, "steps": steps, "warmup": 1, "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "32^4 lattice (links exp(0.2 i H), seed 6101, kappa 0.1365), 4096 blocks of 4^4; "
                               "det D_Lambda = det(1 - kappa^2 H_eo H_oe) assembled densely (n = 1536) and "
                               "factorised by batched LU",
                   "total_logdet": [tot.real, tot.imag], "repeatable": bool(np.array_equal(ld, ld2))},
        "roofline": {"kernel": "dd_block_logdet (assembly and batched LU)", "bound": "mfma", "achieved": achieved,
                     "peak": 78.6, "unit": "TFLOP/s", "frac": achieved / 78.6, "traffic": None,
                     "alg_flops_per_launch": flops, "timing": "wall time of the synchronising call"},
    }), flush=True)
    g.close()
    blk.close()
    ctx.close()


def run_solve(args):
    """--workload c2 / c3: one dd_block_solve over all (block, rhs) pairs per step."""
    import torch

    from paper_2211_06902_amd import dd

    w = WORKLOADS[args.workload]
    inner = args.inner or w["inner"]
    gmres = w["method"] == "gmres"
    t0 = time.perf_counter()
    U, b, boxes = _inputs(w)
    t_gen = time.perf_counter() - t0
    ctx = dd.Context(0)
    blk = ctx.make_blocks(w["L"], -1, w["segs"])
    U_dev = torch.from_numpy(U).cuda()
    x = torch.empty_like(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = ctx.load_gauge(blk, U_dev, "bf16" if inner == "bf16" else "f32")
    t_pack = time.perf_counter() - t0
    del U_dev
    params = dd.solve_params(inner_prec=inner, tol=TOL, method=dd.GMRES if gmres else dd.BICGSTAB, restart=16,
                             use_graph=0 if args.no_graph else 1)
    sched = None
    if gmres:
        tried, best = ctx.autotune_gmres(blk, g, w["kappa"], b, params=params, scratch=x)
        sched = {"threads": best[0], "queues": best[1], "wg_per_cu": best[2],
                 "candidates_ms": [[r[0], r[1], r[2], round(r[3], 3)] for r in tried]}

    for _ in range(args.warmup):
        _, info, st = ctx.block_solve(blk, g, w["kappa"], b, x, params=params)
        if st != dd.DD_OK:
            raise SystemExit("warmup solve did not converge: %s" % info["flags"])

    # the timed steps run the library's default path (graph replay, no kernel timers)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ok = True
    cycles, iters = [], []
    for _ in range(args.steps):
        _, info, st = ctx.block_solve(blk, g, w["kappa"], b, x, params=params)
        ok = ok and st == dd.DD_OK and bool(np.all(info["true_relres"] <= TOL))
        cycles.append(info["outer_cycles"])
        iters.append(info["inner_iterations"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    # one more step with the kernel timers on for the roofline
    ctx.timer_enable(True)
    ctx.timer_reset()
    ctx.block_solve(blk, g, w["kappa"], b, x, params=params)
    if gmres:
        kname = "k_gmres (persistent GMRES(16), FP32 spinor / %s link, whole inner solve per launch)" % inner.upper()
        k_ms, k_n, k_bytes = ctx.timer_read(dd.KCLASS_GMRES)
    else:
        kname, (k_ms, k_n, k_bytes) = stencil_timer(ctx, inner)
    ctx.timer_enable(False)

    n_solves = blk.n_blocks * w["nrhs"]
    achieved = k_bytes / (k_ms * 1e-3) / 1e9 if k_ms > 0 else 0.0
    out = {
        "metric": METRIC,
        "value": (n_solves * args.steps / dt) if ok else 0.0,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": inner,
        "data": "synthetic",
        "config": {
            "workload": w["text"] % inner.upper(),
            "solves_per_step": n_solves,
            "all_converged": ok,
            "outer_cycles_per_step": cycles,
            "inner_iterations_per_step": iters,
            "link_pack_s": t_pack,
            "input_generation_s": t_gen,
        },
        "roofline": {
            "kernel": kname,
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": profiled_traffic(PROFILE_C2) if (args.workload == "c2" and inner == "f32") else None,
            "launches": k_n,
            "avg_launch_us": k_ms * 1e3 / max(k_n, 1),
            "alg_bytes_per_launch": k_bytes / max(k_n, 1),
            "timing": "HIP events around each launch on the library stream, in one extra step",
        },
    }
    if sched:
        out["config"]["gmres_schedule"] = sched
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, U, b, boxes)
    print(json.dumps(out), flush=True)
    g.close()
    blk.close()
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle's CPU baseline")
    ap.add_argument("--no-nn", action="store_true", help="c5: skip the network-preconditioned form")
    ap.add_argument("--only-head", action="store_true", help="c5: time the headline form only (no FP64, no network)")
    ap.add_argument("--no-graph", action="store_true", help="launch every inner iteration from the host")
    ap.add_argument("--inner", default=None, choices=["f32", "bf16", "f64"],
                    help="inner precision (default: FP32; BF16 links for c3)")
    ap.add_argument("--workload", default="c5",
                    choices=sorted(WORKLOADS) + ["c4", "c5", "dlam", "exterior", "global", "logdet", "nnapply"])
    ap.add_argument("--epochs", type=int, default=4, help="c4, c5: training epochs of the network")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (4 times), to calibrate HBM byte counters")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch

        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4, "copies": 4}))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the block solves need no communication and the library has "
              "no multi-GPU path (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    {"c4": run_c4, "c5": run_c5, "dlam": run_dlam, "nnapply": run_nnapply, "global": run_global,
     "exterior": run_exterior, "logdet": run_logdet}.get(args.workload, run_solve)(args)


if __name__ == "__main__":
    main()
