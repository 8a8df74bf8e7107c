"""Benchmark: batched block solves D_Lambda^{-1} b on one MI355X.

Default workload (c2): 32^4 lattice (antiperiodic time), SU(3) links
exp(i 0.3 H) from seed 2101, kappa = 0.1355, 256 blocks of 8^4 (Dirichlet),
12 Gaussian sources per block from seed 2102, i.e. 3072 independent block
solves per step.  Method: FP32 even-odd BiCGStab inner solves inside FP64
defect correction, every pair to an FP64 true relative residual <= 1e-10.

--workload c3: 48^3 x 96 lattice, kappa 0.1355, links exp(i 0.3 H) from seed
3101, 2160 uneven blocks (1296 of 8^4 and 864 of 8^3 x 12), 12 sources per
block (25 920 solves per step) drawn on the GPU from seed 3102; persistent
GMRES(16) inner solves with BF16 links and FP32 spinors (schedule chosen by
the autotuner before timing) inside FP64 defect correction.

A step is one dd_block_solve call over the whole batch: the sources are
already on the GPU; the step packs them into the library layout, solves all
pairs and unpacks the solutions.  Links are packed once before timing.

Printed (one JSON line): solves/s, the dominant kernel's achieved
algorithmic bandwidth against the 8 TB/s HBM peak measured with HIP events
inside the timed steps, and the CPU oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--workload c2|c3]
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
    return {"value": npairs / dt, "unit": "solves/s", "cores": nthr, "kind": "oracle",
            "sample": "%d (block, rhs) pairs of the same workload (8 per thread), FP64 eo-BiCGStab with FP64 "
                      "defect correction to 1e-10 (%.1f s wall, %d failed)" % (npairs, dt, fails)}


PROFILE = os.path.join(ROOT, "profiles", "k_hop_f32_c2_32x4_12rhs.md")


def profiled_traffic():
    """HBM bytes per launch of the hop from the committed rocprofv3 summary, if it
    was taken on the current kernel source (else None)."""
    try:
        from paper_2211_06902_amd.rocprof_summary import kernel_source_hash

        txt = open(PROFILE).read()
        js = json.loads(txt.split("```json", 1)[1].split("```", 1)[0])
        if js.get("kernel_source_sha256_16") != kernel_source_hash():
            return None
        return js["hbm_traffic_bytes_per_launch"]
    except (OSError, IndexError, KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--inner", default=None, choices=["f32", "bf16", "f64"],
                    help="inner precision (default: FP32 for c2, BF16 links for c3)")
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
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
        print("bench.py measures one GPU only: the block solves need no communication and this build has no "
              "multi-GPU path (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

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
    params = dd.solve_params(inner_prec=inner, tol=TOL, method=dd.GMRES if gmres else dd.BICGSTAB, restart=16)
    sched = None
    if gmres:
        tried, best = ctx.autotune_gmres(blk, g, w["kappa"], b, params=params, scratch=x)
        sched = {"threads": best[0], "queues": best[1], "wg_per_cu": best[2],
                 "candidates_ms": [[r[0], r[1], r[2], round(r[3], 3)] for r in tried]}

    for _ in range(args.warmup):
        _, info, st = ctx.block_solve(blk, g, w["kappa"], b, x, params=params)
        if st != dd.DD_OK:
            raise SystemExit("warmup solve did not converge: %s" % info["flags"])

    ctx.timer_enable(True)
    ctx.timer_reset()
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
    if gmres:
        kclass = dd.KCLASS_GMRES
        kname = "k_gmres (persistent GMRES(16), FP32 spinor / %s link, whole inner solve per launch)" % inner.upper()
    else:
        kclass = {"f64": dd.KCLASS_HOP_F64, "f32": dd.KCLASS_HOP_F32, "bf16": dd.KCLASS_HOP_BF16}[inner]
        kname = "k_hop (%s, 12 rhs)" % ("FP32 spinor / BF16 link" if inner == "bf16" else inner.upper())
    k_ms, k_n, k_bytes = ctx.timer_read(kclass)
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
            "traffic": profiled_traffic() if (args.workload == "c2" and inner == "f32") else None,
            "launches": k_n,
            "avg_launch_us": k_ms * 1e3 / max(k_n, 1),
            "alg_bytes_per_launch": k_bytes / max(k_n, 1),
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


if __name__ == "__main__":
    main()
