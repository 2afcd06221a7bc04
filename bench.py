#!/usr/bin/env python3
"""Throughput benchmark of the MI355X TA / CTA solvers: CTA mixed+batched vs
FP64 plain.

Workload: the LP-shaped rectangular minimum-norm system, A = S + [I 0] with
m = 10,000 rows, n = 1,000,000 columns, six N(0,1) nonzeros per column at
uniformly drawn rows plus the identity slack block (about 6.0e6 nonzeros);
right-hand sides b = A x* with x* ~ N(0,1); CTA of order t = 3 in the
minimum-norm (y) form; every solve stops on the FP64 true relative residual
||b - A x|| / ||b|| <= 1e-6.

Headline (value): mixed+batched -- one step solves a block of 32 right-hand
sides with the batched engine, FP32 matrix values and vectors in the Krylov
chain, FP64 Gram entries, steps, y and true-residual checks; the value is
right-hand sides solved per second.  Beside it, measured in the same run:
FP64 plain (one right-hand side per solve on a prepared operator) and FP64
batched (32 right-hand sides, all FP64).  Matrix preparation (transposes,
low-precision copies) happens once per matrix, before timing, and is
reported as plan_ms.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the batched SpMM passes on this workload, from two
# rocprofv3 counter runs (FETCH_SIZE and WRITE_SIZE, scaled by a 1 GiB copy
# kernel); see profiles/k_bspmm_fp32_k32_lp_shaped_traffic.md.  Valid for
# fp32, k = 32 only.
MEASURED_TRAFFIC = {("fp32", 32, "A"): 748.9e6, ("fp32", 32, "AT"): 192.3e6}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def csr_pass_bytes(rows: int, cols: int, nnz: int, val_bytes: int, idx_bytes: int,
                   vec_bytes: int, k: int = 1) -> int:
    """Algorithmic HBM bytes of one Y = M X pass over a CSR matrix M (rows x
    cols) with k right-hand sides: values and column indices once, row
    pointers once, the input block once, the output block written once."""
    return (nnz * (val_bytes + idx_bytes) + (rows + 1) * 4 + cols * k * vec_bytes
            + rows * k * vec_bytes)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--k", type=int, default=32, help="right-hand sides per batched step")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-solves", type=int, default=8,
                    help="oracle solves timed for the CPU baseline (about 1.5 s each)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU layout is described, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2304_12168_amd as P
    from workloads import lp_shaped

    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    P.load_library()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    m, n, tol, t, K = 10_000, 1_000_000, 1e-6, 3, args.k
    log(f"[bench] generating LP-shaped {m}x{n} (seed {args.seed})")
    prob = lp_shaped(m, n, per_col=6, seed=args.seed)
    A = P.to_device(prob.A)
    nnz = A.nnz
    sp = prob.A.to_scipy()
    g = np.random.default_rng([args.seed, 99])
    nblk = 4  # distinct right-hand-side blocks, cycled over the steps
    blocks = [torch.from_numpy(sp @ g.standard_normal((n, K))).to(dev) for _ in range(nblk)]
    singles = [blocks[i % nblk][:, i // nblk].contiguous() for i in range(args.warmup + args.steps)]
    torch.cuda.synchronize()

    # ---- prepared operators ----
    t0 = time.perf_counter()
    pl = P.plan(A)
    bp = P.BatchPlan([A], args.precision)
    bp64 = P.BatchPlan([A], "fp64") if args.precision != "fp64" else bp
    torch.cuda.synchronize()
    plan_ms = 1e3 * (time.perf_counter() - t0)
    log(f"[bench] plans built in {plan_ms:.1f} ms")

    def check(infos, what):
        bad = [i for i in infos if i.stop != "residual" or not i.rel_res <= tol]
        if bad:
            raise SystemExit(f"{what}: {len(bad)} solves missed the tolerance: {bad[0]}")

    # ---- headline: mixed + batched ----
    def batched_step(plan, prec, i):
        _, infos = P.cta_solve_batched(plan, [blocks[i % nblk]], tol=tol, t=t, max_iter=1000,
                                       minnorm=True, precision=prec)
        return infos[0]

    for i in range(args.warmup):
        inf = batched_step(bp, args.precision, i)
        log(f"[bench] warmup {i}: iterations {max(x.iters for x in inf)}, "
            f"max rel_res {max(x.rel_res for x in inf):.2e}")
        check(inf, "warmup")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    allinf = []
    for i in range(args.steps):
        allinf += batched_step(bp, args.precision, i)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    check(allinf, "mixed+batched")
    ms_per_step = 1e3 * elapsed / args.steps
    value = K * args.steps / elapsed
    iters = [x.iters for x in allinf]
    log(f"[bench] mixed+batched ({args.precision}, k={K}): {ms_per_step:.3f} ms per step, "
        f"{value:.1f} right-hand sides/s, iterations {min(iters)}-{max(iters)}")

    # ---- FP64 plain: one right-hand side per solve ----
    nplain = max(5, args.steps)
    for i in range(min(2, args.warmup)):
        P.cta_minnorm(pl, singles[i], tol=tol, t=t, max_iter=1000, hist_cap=64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pinf = [P.cta_minnorm(pl, singles[i % len(singles)], tol=tol, t=t, max_iter=1000,
                          hist_cap=64)[2] for i in range(nplain)]
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    check(pinf, "fp64 plain")
    plain_rate = nplain / plain_s
    log(f"[bench] FP64 plain: {1e3 * plain_s / nplain:.3f} ms per solve, {plain_rate:.1f} solves/s")

    # ---- FP64 batched, same blocks ----
    nb64 = max(3, args.steps // 4)
    batched_step(bp64, "fp64", 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b64inf = []
    for i in range(nb64):
        b64inf += batched_step(bp64, "fp64", i)
    torch.cuda.synchronize()
    b64_s = time.perf_counter() - t0
    check(b64inf, "fp64 batched")
    b64_rate = K * nb64 / b64_s
    log(f"[bench] FP64 batched (k={K}): {b64_rate:.1f} right-hand sides/s")

    # ---- dominant kernel of the headline path ----
    vb = {"fp32": 4, "bf16": 2, "fp64": 8}[args.precision]
    xb = 8 if args.precision == "fp64" else 4
    ms_a = P.batch_time_spmm(bp, K, trans=False, precision=args.precision, reps=20)
    ms_at = P.batch_time_spmm(bp, K, trans=True, precision=args.precision, reps=20)
    by_a = csr_pass_bytes(m, n, nnz, vb, 4, xb, K)
    by_at = csr_pass_bytes(n, m, nnz, vb, 4, xb, K)
    log(f"[bench] SpMM k={K} {args.precision}: A pass {ms_a * 1e3:.1f} us "
        f"({by_a / ms_a / 1e6:.0f} GB/s), A^T pass {ms_at * 1e3:.1f} us "
        f"({by_at / ms_at / 1e6:.0f} GB/s)")
    if ms_a >= ms_at:
        kname, kms, kbytes = (f"k_bspmm<{args.precision},K={K}> on A "
                              "(1e4 rows x ~600 nnz; gathers rows of the n x K block)"), ms_a, by_a
        traffic = MEASURED_TRAFFIC.get((args.precision, K, "A"))
    else:
        kname, kms, kbytes = (f"k_bspmm<{args.precision},K={K}> on A^T "
                              "(1e6 rows x ~6 nnz)"), ms_at, by_at
        traffic = MEASURED_TRAFFIC.get((args.precision, K, "AT"))
    achieved = kbytes / (kms * 1e-3) / 1e9

    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        oracle.build(force=False)
        k = max(1, args.cpu_solves)
        log(f"[bench] CPU oracle: {k} solves, 1 thread")
        c0 = time.perf_counter()
        for i in range(k):
            _, _, oi = oracle.cta_minnorm(prob.A, singles[i % len(singles)].cpu().numpy(), tol=tol,
                                          t=t, max_iter=1000, hist_cap=64)
        csec = time.perf_counter() - c0
        cpu = {"value": k / csec, "unit": "right-hand sides/s", "cores": 1, "kind": "oracle",
               "sample": f"{k} full single-right-hand-side solves of the same system (FP64, "
                         f"sequential C, {oi.iters} iterations each), {csec:.1f} s"}

    out = {
        "metric": "solves/s and HBM GB/s to rel-residual 1e-6: CTA mixed+batched vs FP64 plain",
        "value": value,
        "unit": "right-hand sides solved/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32/f64" if args.precision == "fp32" else
                 ("bf16/f32/f64" if args.precision == "bf16" else "f64"),
        "data": "synthetic",
        "config": {"workload": "lp_shaped_minnorm m=10000 n=1000000 nnz/col=6 +I slack, "
                               f"CTA t=3 y-form, mixed ({args.precision} products, FP64 "
                               f"refinement) batched k={K}, rel-res 1e-6",
                   "m": m, "n": n, "nnz": nnz, "t": t, "tol": tol, "seed": args.seed,
                   "k_per_step": K, "precision": args.precision,
                   "iterations": max(iters), "plan_ms": plan_ms,
                   "fp64_plain_solves_per_s": plain_rate,
                   "fp64_batched_rhs_per_s": b64_rate,
                   "speedup_vs_fp64_plain": value / plain_rate},
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "bytes_per_launch": kbytes, "avg_launch_us": kms * 1e3},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
