"""Benchmark: batched block solves D_Lambda^{-1} b on one MI355X.

Workload: 32^4 lattice (antiperiodic time), SU(3) links exp(i 0.3 H) from
seed 2101, kappa = 0.1355, 256 blocks of 8^4 (Dirichlet), 12 Gaussian sources
per block from seed 2102, i.e. 3072 independent block solves per step.
Method: FP32 even-odd BiCGStab inner solves inside FP64 defect correction,
every pair to an FP64 true relative residual <= 1e-10.

A step is one dd_block_solve call over the whole batch: the sources are
already on the GPU; the step packs them into the library layout, solves all
pairs and unpacks the solutions.  Links are packed once before timing.

Printed (one JSON line): solves/s, the hop (Dslash) kernel's achieved
algorithmic bandwidth against the 8 TB/s HBM peak measured with HIP events
inside the timed steps, and the CPU oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
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

L = (32, 32, 32, 32)
KAPPA = 0.1355
EPS = 0.3
SEED_U, SEED_SRC = 2101, 2102
SEGS = [[8] * 4] * 4
NRHS = 12
TOL = 1e-10


def _inputs():
    import synth

    U = synth.gauge_field(L, EPS, SEED_U)
    # tile order: direction 3 fastest; each block in box-local canonical order
    t = np.arange(4)
    sites = []
    for a in t:
        for b in t:
            for c in t:
                for d in t:
                    y = np.indices((8, 8, 8, 8)).reshape(4, -1).T + 8 * np.array([a, b, c, d])
                    sites.append(((y[:, 0] * L[1] + y[:, 1]) * L[2] + y[:, 2]) * L[3] + y[:, 3])
    sites = np.concatenate(sites)
    src = synth.spinor_field(L, NRHS, SEED_SRC)[:, sites]
    return U, src, sites


def cpu_baseline(U, src):
    """The oracle's FP64 block solve (OpenMP over pairs) on a bounded sample."""
    from oracle import wilson

    nthr = wilson.num_threads()
    npairs = max(1, min(8 * nthr, 3072))  # about 10-20 s of CPU work
    S = 8**4
    boxes = []
    b = np.zeros((1, npairs * S, 4, 3), dtype=np.complex128)
    for k in range(npairs):
        blk, r = (k * 37) % 256, k % NRHS
        a0, a1, a2, a3 = blk // 64, (blk // 16) % 4, (blk // 4) % 4, blk % 4
        boxes.append([8 * a0, 8 * a1, 8 * a2, 8 * a3, 8, 8, 8, 8])
        b[0, k * S:(k + 1) * S] = src[r, blk * S:(blk + 1) * S]
    t0 = time.perf_counter()
    _, iters, rel, fails = wilson.solve_many(L, -1, KAPPA, U, np.asarray(boxes), b, tol=TOL, nthreads=nthr)
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
    ap.add_argument("--inner", default="f32", choices=["f32", "bf16", "f64"])
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

    t0 = time.perf_counter()
    U, src, _ = _inputs()
    t_gen = time.perf_counter() - t0
    ctx = dd.Context(0)
    blk = ctx.make_blocks(L, -1, SEGS)
    U_dev = torch.from_numpy(U).cuda()
    b = torch.from_numpy(np.ascontiguousarray(src)).cuda()
    x = torch.empty_like(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g = ctx.load_gauge(blk, U_dev, "bf16" if args.inner == "bf16" else "f32")
    t_pack = time.perf_counter() - t0
    params = dd.solve_params(inner_prec=args.inner, tol=TOL)

    for _ in range(args.warmup):
        _, info, st = ctx.block_solve(blk, g, KAPPA, b, x, params=params)
        if st != dd.DD_OK:
            raise SystemExit("warmup solve did not converge: %s" % info["flags"])

    ctx.timer_enable(True)
    ctx.timer_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ok = True
    cycles, iters = [], []
    for _ in range(args.steps):
        _, info, st = ctx.block_solve(blk, g, KAPPA, b, x, params=params)
        ok = ok and st == dd.DD_OK and bool(np.all(info["true_relres"] <= TOL))
        cycles.append(info["outer_cycles"])
        iters.append(info["inner_iterations"])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kclass = {"f64": dd.KCLASS_HOP_F64, "f32": dd.KCLASS_HOP_F32, "bf16": dd.KCLASS_HOP_BF16}[args.inner]
    hop_ms, hop_n, hop_bytes = ctx.timer_read(kclass)
    ctx.timer_enable(False)

    n_solves = blk.n_blocks * NRHS
    achieved = hop_bytes / (hop_ms * 1e-3) / 1e9 if hop_ms > 0 else 0.0
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
        "dtype": args.inner,
        "data": "synthetic",
        "config": {
            "workload": "32^4 lattice, 256 blocks of 8^4 (Dirichlet), 12 rhs per block, kappa 0.1355, "
                        "SU(3) links exp(0.3 i H); %s eo-BiCGStab inner solves, FP64 defect correction, "
                        "per-pair FP64 true relative residual <= 1e-10" % args.inner.upper(),
            "solves_per_step": n_solves,
            "all_converged": ok,
            "outer_cycles_per_step": cycles,
            "inner_iterations_per_step": iters,
            "link_pack_s": t_pack,
            "input_generation_s": t_gen,
        },
        "roofline": {
            "kernel": "k_hop (%s, 12 rhs)" % ("FP32 spinor / BF16 link" if args.inner == "bf16" else args.inner.upper()),
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": profiled_traffic() if args.inner == "f32" else None,
            "launches": hop_n,
            "avg_launch_us": hop_ms * 1e3 / max(hop_n, 1),
            "alg_bytes_per_launch": hop_bytes / max(hop_n, 1),
        },
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(U, src)
    print(json.dumps(out), flush=True)
    g.close()
    blk.close()
    ctx.close()


if __name__ == "__main__":
    main()
