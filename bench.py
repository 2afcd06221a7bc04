#!/usr/bin/env python3
"""Throughput benchmark of the MI355X CTA solvers: mixed+batched vs FP64 plain.

Headline workload -- batched uneven systems: 256 square systems with sizes
n ~ U{1024..65536}, even-numbered ones Poisson 5-point stencils on an
nx x ny grid (nx = floor(sqrt(n))), odd-numbered ones random sparse with 7
off-diagonal N(0,1) entries per row and a diagonal of 2 x the row's absolute
sum; each system has k ~ U{1..64} right-hand sides with entries ~ U[-1, 1]
(about 8.5e3 columns, 5e7 nonzeros in all).  CTA of order t = 3 (x-form) on
every column with a budget of 400 iterations per column, stop at FP64 true
relative residual 1e-6.

A step is one batched solve of the whole set: FP32 matrix values and vectors
in the Krylov chain, FP64 Gram entries, steps, x and true-residual checks.
value = columns that reach 1e-6 (FP64 true residual), per second.  The
stencil columns do not converge within the budget (H = A A^T squares the
condition number); they run their 400 iterations inside the step and are
reported as iterations per second.

Beside it, in the same run: FP64 batched (the same call in FP64) and FP64
plain (one column per cta_solve call on a prepared operator, on a seeded
sample of columns; rate = converged columns / time of the sample).  Plans
(transposes, low-precision copies) are built before timing and reported as
plan_ms.  A secondary block measures the LP-shaped rectangular minimum-norm
system (m = 1e4, n = 1e6) the same way with 32 right-hand sides per step.

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

# HBM bytes per launch of the dominant kernel on this workload come from two
# rocprofv3 counter runs (FETCH_SIZE, then WRITE_SIZE, scaled by a 1 GiB copy
# kernel) stored in profiles/ with the hash of the kernel source they were
# taken on; the roofline's traffic is None when that source has changed since.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_bspmm_fp32_k64_batched_uneven_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2304_12168_amd", "csrc", "batched.hip")


def measured_traffic():
    """{(precision, K, pass, part): bytes} if the committed counter figures
    were taken on the current kernel source, else {}."""
    import hashlib

    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
        with open(KERNEL_SRC, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError):
        return {}
    if rec.get("kernel_source_sha256") != sha:
        return {}
    return {(e["precision"], e["K"], e["pass"], e["part"]): e["bytes_per_launch"]
            for e in rec.get("entries", [])}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def csr_pass_bytes(rows: int, cols: int, nnz: int, val_bytes: int, idx_bytes: int,
                   vec_bytes: int, k: int = 1) -> int:
    """Algorithmic HBM bytes of one Y = M X pass over a CSR matrix M (rows x
    cols) with k right-hand sides: values and column indices once, row
    pointers once, the input block once, the output block written once."""
    return (nnz * (val_bytes + idx_bytes) + (rows + 1) * 4 + cols * k * vec_bytes
            + rows * k * vec_bytes)


def group_pass_bytes(systems, ks, val_bytes: int, vec_bytes: int, K: int = 0) -> int:
    """Algorithmic HBM bytes of one pass Y = M X over the block-diagonal
    operator of `systems` (square), each system with its own k_s right-hand
    sides: every system's matrix once, its k_s input and output columns once.
    With K > 0, every system is counted at K columns instead (what a kernel
    of vector width K streams, padding included)."""
    return sum(csr_pass_bytes(a.m, a.n, a.nnz, val_bytes, 4, vec_bytes, K if K else k)
               for a, k in zip(systems, ks))


def kwidth(k: int) -> int:
    K = 1
    while K < k:
        K *= 2
    return K


def column_pieces(k: int):
    """[(K, width)]: how the batched solve splits a system's k right-hand
    sides into width groups (the widest power of two K1 <= k and the rest,
    when the rest rounds up to less than K1; else one piece of kwidth(k))."""
    if k <= 0:
        return []
    K1 = 1
    while 2 * K1 <= k:
        K1 *= 2
    if K1 == k or kwidth(k - K1) == K1:
        return [(kwidth(k), k)]
    return [(K1, K1), (kwidth(k - K1), k - K1)]


def batched_uneven_bench(args, P, torch, dev, pool=None):
    import numpy as np

    from workloads import batched_uneven

    tol, t, budget = 1e-6, 3, args.budget
    t0 = time.perf_counter()
    bt = batched_uneven(nsys=256, nmin=1024, nmax=65536, kmin=1, kmax=64, seed=args.seed)
    log(f"[bench] batched uneven: generated in {time.perf_counter() - t0:.1f} s")
    systems = [P.to_device(a) for a in bt.systems]
    # right-hand sides stored column-major (k, m) so the call makes no copy
    B = [torch.from_numpy(np.ascontiguousarray(b.T)).to(dev).t() for b in bt.B]
    ks = [b.shape[1] for b in bt.B]
    ncols = sum(ks)
    M = sum(a.m for a in bt.systems)
    nnz = sum(a.nnz for a in bt.systems)
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    bp = P.BatchPlan(systems, args.precision)
    bp64 = P.BatchPlan(systems, "fp64") if args.precision != "fp64" else bp
    torch.cuda.synchronize()
    plan_ms = 1e3 * (time.perf_counter() - t0)

    last_x = []

    def solve(plan, prec):
        X, infos = P.cta_solve_batched(plan, B, tol=tol, t=t, max_iter=budget, precision=prec)
        last_x[:] = [X]
        return infos

    def summary(infos):
        conv = iters_st = 0
        for s, inf in enumerate(infos):
            for i in inf:
                if i.stop == "residual":
                    if not i.rel_res <= tol:
                        raise SystemExit(f"column of system {s} reported converged at {i.rel_res}")
                    conv += 1
                if bt.kinds[s] == "stencil":
                    iters_st += i.iters
        return conv, iters_st

    for i in range(args.warmup):
        c, _ = summary(solve(bp, args.precision))
        log(f"[bench] warmup {i}: {c} of {ncols} columns converged")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = [solve(bp, args.precision) for _ in range(args.steps)]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    sums = [summary(r) for r in runs]
    conv = sum(c for c, _ in sums)
    value = conv / elapsed
    ms_per_step = 1e3 * elapsed / args.steps
    stencil_its = sum(s for _, s in sums) / elapsed
    rand_iters = sorted(i.iters for s, inf in enumerate(runs[-1]) for i in inf
                        if bt.kinds[s] == "random" and i.stop == "residual")
    # what per-column masks could skip: a system runs until its last column
    # stops, so each earlier-stopping column idles (max - its count) iterations
    idle = busy = 0
    for s, inf in enumerate(runs[-1]):
        if inf:
            top = max(i.iters for i in inf)
            idle += sum(top - i.iters for i in inf)
            busy += top * len(inf)
    idle_frac = idle / busy if busy else 0.0
    x_mixed = [x.cpu().numpy() for x in last_x[0]]  # the last timed step's solutions
    # bytes the step's matrix products move (algorithmic): per system, 2t passes
    # over its matrix per iteration while any column is active, and per column
    # and iteration 2t products each reading and writing one vector column
    vbs = {"fp32": 4, "bf16": 2, "fp64": 8}[args.precision]
    xbs = 8 if args.precision == "fp64" else 4
    step_bytes = 0
    for s, inf in enumerate(runs[-1]):
        a = bt.systems[s]
        c0 = 0
        for _, w in column_pieces(len(inf)):  # each piece reads the matrix on its own
            step_bytes += (max(i.iters for i in inf[c0:c0 + w]) * 2 * t *
                           (a.nnz * (vbs + 4) + 4 * (a.m + 1)))
            c0 += w
        step_bytes += sum(i.iters for i in inf) * 2 * t * 2 * a.m * xbs
    log(f"[bench] mixed+batched ({args.precision}): {ms_per_step:.1f} ms per step, "
        f"{conv // args.steps} of {ncols} columns converged per step, {value:.1f} columns/s")

    # FP64 batched, one solve
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    inf64 = solve(bp64, "fp64")
    torch.cuda.synchronize()
    b64_s = time.perf_counter() - t0
    conv64, _ = summary(inf64)
    log(f"[bench] FP64 batched: {b64_s * 1e3:.1f} ms, {conv64} columns converged")

    # BF16 products (FP32 accumulation) with FP64 refinement, one solve
    bf16 = None
    if args.precision != "bf16" and not args.no_bf16:
        bp16 = P.BatchPlan(systems, "bf16")
        solve(bp16, "bf16")  # warm-up (row-lane tuning)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        inf16 = solve(bp16, "bf16")
        torch.cuda.synchronize()
        b16_s = time.perf_counter() - t0
        conv16, _ = summary(inf16)
        bp16.close()
        bf16 = {"columns_per_s": conv16 / b16_s, "ms": b16_s * 1e3,
                "columns_converged": conv16}
        log(f"[bench] BF16 batched: {b16_s * 1e3:.1f} ms, {conv16} columns converged")

    # FP64 plain on a seeded sample of columns, one cta_solve call each
    g = np.random.default_rng([args.seed, 7])
    flat = [(s, c) for s in range(len(ks)) for c in range(ks[s])]
    pick = [flat[i] for i in g.choice(len(flat), size=args.plain_sample, replace=False)]
    plans = {s: P.plan(systems[s]) for s in sorted({s for s, _ in pick})}
    cols = [B[s][:, c].contiguous() for s, c in pick]
    P.cta_solve(plans[pick[0][0]], cols[0], tol=tol, t=t, max_iter=budget, hist_cap=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pinf = [P.cta_solve(plans[s], cols[i], tol=tol, t=t, max_iter=budget, hist_cap=1)[2]
            for i, (s, _) in enumerate(pick)]
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    plain_conv = sum(i.stop == "residual" for i in pinf)
    plain_rate = plain_conv / plain_s
    log(f"[bench] FP64 plain: {len(pick)} sampled columns in {plain_s:.2f} s, "
        f"{plain_conv} converged: {plain_rate:.1f} columns/s")

    # dominant kernel: the SpMM of the width group whose product takes longest,
    # A and A^T passes, launched as the solve launches it.  The library cuts a
    # system's columns into pieces (column_pieces) and runs a group's
    # low-precision chain in two parts, systems with at most 6 nonzeros per row
    # on average (one round of the kernel's gathers) and the rest, so each part
    # is timed on a plan over exactly its systems and a product of the group is
    # one launch of each part.  Every group is timed and listed.
    split = args.precision != "fp64"
    vb = {"fp32": 4, "bf16": 2, "fp64": 8}[args.precision]
    xb = 8 if args.precision == "fp64" else 4
    members = {}
    for s_, k in enumerate(ks):
        for K, w in column_pieces(k):
            members.setdefault(K, []).append((s_, w))
    groups = []
    for K in sorted(members, reverse=True):
        grp = members[K]
        parts = ([[(s_, w) for s_, w in grp if bt.systems[s_].nnz <= 6 * bt.systems[s_].m],
                  [(s_, w) for s_, w in grp if bt.systems[s_].nnz > 6 * bt.systems[s_].m]]
                 if split else [grp])
        part_rows = []
        for q in [q for q in parts if q]:
            gp = P.BatchPlan([systems[s_] for s_, _ in q], args.precision)
            qa = P.batch_time_spmm(gp, K, trans=False, precision=args.precision, reps=args.reps)
            qt = P.batch_time_spmm(gp, K, trans=True, precision=args.precision, reps=args.reps)
            gp.close()
            qsys = [bt.systems[s_] for s_, _ in q]
            qks = [w for _, w in q]
            qm = sum(a.m for a in qsys)
            qnnz = sum(a.nnz for a in qsys)
            part_rows.append({"systems": len(q), "rows": qm, "nnz": qnnz, "columns": sum(qks),
                              "bytes_per_launch": group_pass_bytes(qsys, qks, vb, xb),
                              "padded_bytes_per_launch": group_pass_bytes(qsys, qks, vb, xb, K=K),
                              "A_us": qa * 1e3, "AT_us": qt * 1e3})
        ms_a = sum(r["A_us"] for r in part_rows) * 1e-3
        ms_at = sum(r["AT_us"] for r in part_rows) * 1e-3
        by = sum(r["bytes_per_launch"] for r in part_rows)
        by_pad = sum(r["padded_bytes_per_launch"] for r in part_rows)
        groups.append({"K": K, "systems": len(grp), "columns": sum(w for _, w in grp),
                       "A_us": ms_a * 1e3, "AT_us": ms_at * 1e3, "bytes_per_launch": by,
                       "padded_bytes_per_launch": by_pad,
                       "frac": by / (max(ms_a, ms_at) * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       "parts": part_rows})
        log(f"[bench] SpMM K={K} {args.precision}: {len(grp)} systems, "
            f"{sum(w for _, w in grp)} columns, {len(part_rows)} launches: A {ms_a * 1e3:.1f} us, "
            f"A^T {ms_at * 1e3:.1f} us, {by / 1e9:.3f} GB algorithmic "
            f"({by_pad / 1e9:.3f} GB with padding), frac {groups[-1]['frac']:.3f}")
    dom = max(groups, key=lambda g_: max(g_["A_us"], g_["AT_us"]))
    Kd, part_rows = dom["K"], dom["parts"]
    ms_a, ms_at = dom["A_us"] * 1e-3, dom["AT_us"] * 1e-3
    by, by_pad = dom["bytes_per_launch"], dom["padded_bytes_per_launch"]
    gm = sum(r["rows"] for r in part_rows)
    gnnz = sum(r["nnz"] for r in part_rows)
    trans = ms_at > ms_a
    kms = max(ms_a, ms_at)
    orient = "AT" if trans else "A"
    mt = measured_traffic()
    traffic = None
    if all((args.precision, Kd, orient, i) in mt for i in range(len(part_rows))):
        traffic = sum(mt[(args.precision, Kd, orient, i)] for i in range(len(part_rows)))

    cpu = None
    x_err = None
    if pool is not None:
        cpu, x_err = cpu_baseline(args, bt, x_mixed, runs[-1], tol, t, budget, *pool)

    res = {
        "value": value, "ms_per_step": ms_per_step,
        "config": {
            "workload": "batched_uneven: 256 systems n~U{1024..65536}, half Poisson 5-point, half "
                        "random 8 nnz/row diag 2*rowsum, k~U{1..64} rhs ~U[-1,1]; CTA t=3 x-form, "
                        f"budget {budget} iterations/column, FP64 true rel-res 1e-6; "
                        f"{args.precision} products + FP64 refinement",
            "systems": 256, "columns": ncols, "rows": M, "nnz": nnz, "t": t, "tol": tol,
            "budget": budget, "seed": args.seed, "precision": args.precision,
            "columns_converged_per_step": conv // args.steps,
            "random_iterations_median": rand_iters[len(rand_iters) // 2] if rand_iters else None,
            "stopped_column_idle_fraction": idle_frac,
            "stencil_iterations_per_s": stencil_its, "plan_ms": plan_ms,
            "fp64_batched_columns_per_s": conv64 / b64_s,
            "bf16_batched": bf16,
            "fp64_plain_columns_per_s": plain_rate,
            "fp64_plain_sample": f"{len(pick)} columns, {plain_conv} converged, {plain_s:.2f} s",
            "speedup_vs_fp64_plain": value / plain_rate if plain_rate > 0 else None,
            "speedup_vs_fp64_batched": value / (conv64 / b64_s) if conv64 else None,
            "step_product_bytes": step_bytes,
            "step_product_GB_s": step_bytes / (ms_per_step * 1e-3) / 1e9,
            "x_rel_err_vs_fp64_oracle": x_err},
        "roofline": {
            "bound": "hbm",
            "kernel": f"k_bspmm<{args.precision}, K={Kd}> {'A^T' if trans else 'A'} product over "
                      f"the {dom['systems']} system pieces of width {Kd // 2 + 1}-{Kd} "
                      f"({gm} rows, {gnnz} nonzeros, {dom['columns']} columns), one launch per "
                      f"row-length part",
            "achieved": by / (kms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": by / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "traffic": traffic,
            "bytes_per_launch": by, "padded_bytes_per_launch": by_pad,
            "frac_with_padding": by_pad / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "avg_launch_us": kms * 1e3,
            "other_pass_us": min(ms_a, ms_at) * 1e3, "parts": part_rows,
            "groups": [{k_: v for k_, v in g_.items() if k_ != "parts"} for g_ in groups]},
        "cpu_baseline": cpu,
    }
    return res


def _oracle_column(job):
    """One sampled column solved by the CPU oracle (a worker process)."""
    import oracle

    a, b, tol, t, budget = job
    t0 = time.perf_counter()
    x, _, info = oracle.cta(a, b, tol=tol, t=t, max_iter=budget, hist_cap=1)
    return x, info.stop, time.perf_counter() - t0


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def make_cpu_pool():
    """Worker processes for the CPU baseline, forked before anything touches
    the GPU (they never do): one per host core, at most 12."""
    import multiprocessing as mp

    import oracle

    oracle.build(force=False)
    workers = max(1, min(12, os.cpu_count() or 1))
    return mp.get_context("fork").Pool(workers), workers


def cpu_baseline(args, bt, x_mixed, infos, tol, t, budget, pool, workers):
    """The oracle (sequential C, unchanged) on a seeded sample of the batch's
    columns, one column per worker process on the host's cores, and the
    relative difference between the mixed-precision x of the timed run and
    the oracle's FP64 x on every sampled column both converged."""
    import numpy as np

    g = np.random.default_rng([args.seed, 11])
    flat = [(s, c) for s in range(len(bt.B)) for c in range(bt.B[s].shape[1])]
    pick = [flat[i] for i in g.choice(len(flat), size=args.cpu_sample, replace=False)]
    jobs = [(bt.systems[s], bt.B[s][:, c], tol, t, budget) for s, c in pick]
    log(f"[bench] CPU oracle: {len(pick)} sampled columns on {workers} worker processes")
    c0 = time.perf_counter()
    res = pool.map(_oracle_column, jobs, chunksize=1)
    csec = time.perf_counter() - c0
    cconv = sum(r[1] == "residual" for r in res)
    one = sum(r[2] for r in res)
    errs = []
    for (s, c), (xo, stop, _) in zip(pick, res):
        xg = x_mixed[s][:, c]
        if stop == "residual" and infos[s][c].stop == "residual":
            errs.append(float(np.linalg.norm(xg - xo) / np.linalg.norm(xo)))
    errs.sort()
    x_err = ({"columns": len(errs), "max": errs[-1], "median": errs[len(errs) // 2],
              "note": "||x_mixed - x_oracle|| / ||x_oracle|| on sampled columns both solved"}
             if errs else None)
    if errs:
        log(f"[bench] mixed x vs FP64 oracle x on {len(errs)} columns: max {errs[-1]:.2e}, "
            f"median {errs[len(errs) // 2]:.2e}")
    cpu = {"value": cconv / csec, "unit": "columns solved to 1e-6/s", "cores": workers,
           "kind": "oracle",
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
           "single_thread_value": cconv / one if one > 0 else None,
           "sample": f"{len(pick)} seeded (system, column) pairs of the same batch, each a full "
                     f"single-column CTA-3 solve (budget {budget}) by the sequential C oracle, "
                     f"one column per process on {workers} processes; {cconv} converged; "
                     f"{csec:.1f} s wall, {one:.1f} s summed over the workers"}
    return cpu, x_err


def lp_shaped_bench(args, P, torch, dev):
    """Secondary: the LP-shaped minimum-norm system, 32 right-hand sides per
    step (mixed+batched) vs one per solve (FP64 plain)."""
    import numpy as np

    from workloads import lp_shaped

    m, n, tol, t, K = 10_000, 1_000_000, 1e-6, 3, 32
    prob = lp_shaped(m, n, per_col=6, seed=args.seed)
    A = P.to_device(prob.A)
    sp = prob.A.to_scipy()
    g = np.random.default_rng([args.seed, 99])
    blocks = [torch.from_numpy(sp @ g.standard_normal((n, K))).to(dev) for _ in range(2)]
    pl = P.plan(A)
    bp = P.BatchPlan([A], args.precision)
    torch.cuda.synchronize()

    def step(i):
        _, infos = P.cta_solve_batched(bp, [blocks[i % 2]], tol=tol, t=t, max_iter=1000,
                                       minnorm=True, precision=args.precision)
        return infos[0]

    step(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    inf = sum((step(i) for i in range(args.lp_steps)), [])
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    if any(i.stop != "residual" or not i.rel_res <= tol for i in inf):
        raise SystemExit("LP-shaped mixed+batched: a column missed the tolerance")
    singles = [blocks[0][:, i].contiguous() for i in range(args.lp_steps)]
    P.cta_minnorm(pl, singles[0], tol=tol, t=t, max_iter=1000, hist_cap=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pinf = [P.cta_minnorm(pl, b, tol=tol, t=t, max_iter=1000, hist_cap=1)[2] for b in singles]
    torch.cuda.synchronize()
    pl_s = time.perf_counter() - t0
    if any(i.stop != "residual" for i in pinf):
        raise SystemExit("LP-shaped FP64 plain: a solve missed the tolerance")
    rate, prate = K * args.lp_steps / el, len(singles) / pl_s
    log(f"[bench] LP-shaped: mixed+batched {rate:.0f} columns/s, FP64 plain {prate:.0f} solves/s")
    bp.close()
    # Algorithm 4 from an approximate solution that is not the minimum-norm one
    # (the x-form from a seeded x0), to a certified gap of 1e-4 ||x_eps||
    x0 = torch.from_numpy(0.05 * g.standard_normal(n)).to(dev)
    b0 = blocks[0][:, 0].contiguous()
    xe, _, _ = P.cta_solve(pl, b0, tol=1e-4, t=t, max_iter=100000, x0=x0, hist_cap=1)
    P.ta_minnorm(pl, b0, xe, tol=1e-2, max_iter=200000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xm, im, tests = P.ta_minnorm(pl, b0, xe, tol=1e-4, max_iter=200000)
    torch.cuda.synchronize()
    a4_s = time.perf_counter() - t0
    log(f"[bench] LP-shaped Algorithm 4: {tests} tests, {im.iters} TA iterations, {a4_s:.3f} s, "
        f"norm bracket [{im.rho_lo:.6f}, {im.rho:.6f}]")
    # LP feasibility {A x = b, x >= 0} with b = A |x*| (feasible), TA with c+
    bf = torch.from_numpy(sp @ np.abs(g.standard_normal(n))).to(dev)
    P.ta_solve(pl, bf, tol=1e-2, max_iter=200000, nonneg=True, hist_cap=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xf, _, fi = P.ta_solve(pl, bf, tol=1e-4, max_iter=200000, nonneg=True, hist_cap=1)
    torch.cuda.synchronize()
    lf_s = time.perf_counter() - t0
    log(f"[bench] LP-shaped feasibility (TA with c+): {fi.stop} after {fi.iters} iterations, "
        f"{lf_s:.3f} s, min x = {float(xf.min()):.3g}")
    return {"workload": "lp_shaped_minnorm m=10000 n=1000000 nnz/col=6 +I slack, CTA t=3 y-form, "
                        f"k={K} per step", "nnz": A.nnz,
            "mixed_batched_columns_per_s": rate, "fp64_plain_solves_per_s": prate,
            "speedup": rate / prate, "iterations": max(i.iters for i in inf),
            "algorithm4": {"tol": 1e-4, "stop": im.stop, "tests": tests, "ta_iterations": im.iters,
                           "seconds": a4_s, "rho_lo": im.rho_lo, "rho_hi": im.rho,
                           "ta_iterations_per_s": im.iters / a4_s},
            "lp_feasibility": {"tol": 1e-4, "stop": fi.stop, "iterations": fi.iters,
                               "seconds": lf_s, "rel_res": fi.rel_res}}


def diff_bench(args, P, torch, dev):
    """Secondary: the differentiable solve on the 256 x 256 perturbed stencil
    (n = 65536): FP32 forward and adjoint CTA-3 with FP64 refinement to a
    budget of 300 iterations each (they do not reach 1e-6 there), plus the
    sparse-pattern outer product of the A gradient timed alone."""
    from paper_2304_12168_amd.diff import cta_solve_diff
    from workloads import perturbed_stencil

    p = perturbed_stencil(256, sigma=0.1, seed=args.seed)
    vals = torch.tensor(p.A.val, dtype=torch.float64, device=dev, requires_grad=True)
    b = torch.tensor(p.b, dtype=torch.float64, device=dev, requires_grad=True)
    xt = torch.tensor(p.meta["x_target"], dtype=torch.float64, device=dev)
    budget = 300

    def step():
        vals.grad = None
        b.grad = None
        rec = []
        x = cta_solve_diff(p.A, vals, b, tol=1e-6, t=3, max_iter=budget, precision="fp32",
                           log=rec, allow_unconverged=True)
        ((x - xt) ** 2).sum().backward()
        return rec

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 2
    for _ in range(reps):
        solves = step()
    torch.cuda.synchronize()
    fb_ms = 1e3 * (time.perf_counter() - t0) / reps
    iters = sum(i.iters for _, i in solves)
    # one ta_csr_outer call (device CSR check, a host synchronisation, then the
    # product kernel), on the current stream
    A = P.to_device(p.A)
    u = torch.randn(p.A.m, dtype=torch.float64, device=dev)
    v = torch.randn(p.A.n, dtype=torch.float64, device=dev)
    P.csr_outer(A, u, v, -1.0)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        P.csr_outer(A, u, v, -1.0)
    e1.record()
    torch.cuda.synchronize()
    outer_ms = e0.elapsed_time(e1) / 20
    log(f"[bench] differentiable 256^2: forward+backward {fb_ms:.1f} ms ({iters} iterations), "
        f"outer-product call {outer_ms * 1e3:.1f} us")
    return {"workload": "perturbed 5-point stencil 256x256 (n=65536, sigma=0.1), loss "
                        "||x - x_target||^2, FP32 forward + adjoint CTA-3 with FP64 refinement, "
                        f"budget {budget} iterations each",
            "forward_backward_ms": fb_ms, "iterations": iters,
            "iterations_per_s": iters / (fb_ms * 1e-3),
            "outer_product_call_us": outer_ms * 1e3}


def variants_bench(args, P, torch, dev):
    """Secondary: FP64 single-right-hand-side solves to 1e-6 with the CTA
    variants -- Kac/Clement N = 10001 (fixed t = 3 as configured, and the
    order cycling 1..5..1), the same matrix with a random (inconsistent)
    right-hand side to the normal-equation tolerance 1e-6, plain and with the
    enhanced stop, and the 256 x 256 Poisson matrix (symmetric positive
    definite: H = A A^T vs H = A, fixed and cycling); first-order and t = 3
    runs with the convex-combination step at theta = 0.5 beside the plain
    ones."""
    import numpy as np

    from workloads import kac_clement, poisson5

    out = {}
    kac = kac_clement(10001, seed=args.seed)
    pois = poisson5(256)
    bp = torch.from_numpy(np.random.default_rng([args.seed, 5]).uniform(0, 1, pois.m)).to(dev)
    binc = torch.from_numpy(np.random.default_rng([args.seed, 6]).standard_normal(kac.A.m)).to(dev)
    runs = [("kac_10001_t3", kac.A, torch.from_numpy(kac.b).to(dev), dict(t=3)),
            ("kac_10001_cycle5", kac.A, torch.from_numpy(kac.b).to(dev), dict(t=5, t_cycle=True)),
            ("kac_10001_inconsistent_t3", kac.A, binc, dict(t=3, tol_normal=1e-6)),
            ("kac_10001_inconsistent_t3_enhanced", kac.A, binc,
             dict(t=3, tol_normal=1e-6, enhanced=True)),
            ("poisson_256_AAt_t3", pois, bp, dict(t=3)),
            ("poisson_256_A_t3", pois, bp, dict(t=3, h_is_a=True)),
            ("poisson_256_A_cycle5", pois, bp, dict(t=5, t_cycle=True, h_is_a=True)),
            ("kac_10001_t1", kac.A, torch.from_numpy(kac.b).to(dev), dict(t=1)),
            ("kac_10001_t1_accel0.5", kac.A, torch.from_numpy(kac.b).to(dev),
             dict(t=1, accel=0.5)),
            ("kac_10001_t3_accel0.5", kac.A, torch.from_numpy(kac.b).to(dev),
             dict(t=3, accel=0.5)),
            ("poisson_256_A_t3_accel0.5", pois, bp, dict(t=3, h_is_a=True, accel=0.5))]
    plans = {}
    for name, A, b, kw in runs:
        key = id(A)
        if key not in plans:
            plans[key] = P.plan(A)
        pl = plans[key]
        P.cta_solve(pl, b, tol=1e-6, max_iter=20000, hist_cap=1, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, info = P.cta_solve(pl, b, tol=1e-6, max_iter=20000, hist_cap=1, **kw)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        out[name] = {"stop": info.stop, "iterations": info.iters, "products": info.matvecs,
                     "seconds": sec, "rel_res": info.rel_res, "rel_normal": info.rel_normal}
        log(f"[bench] {name}: {info.stop} after {info.iters} iterations, {info.matvecs} products, "
            f"{sec * 1e3:.1f} ms")
    return out


def iteration_bytes(m, n, nnz, t, dense=False, ta=False):
    """Algorithmic FP64 bytes of one iteration: CTA-t makes t A passes and t
    A^T passes (matrix once each, input and output vectors once) and streams
    (t + 2) residual-length and (t + 2) iterate-length vectors in the update;
    TA makes one pass of each and about four vector streams."""
    mat = m * n * 8 if dense else nnz * 12 + 4 * (max(m, n) + 1)
    a_pass = mat + 8 * (m + n)
    if ta:
        return 2 * a_pass + 4 * 8 * (m + n)
    return 2 * t * a_pass + (t + 2) * 8 * (m + n)


def configs_bench(args, P, torch, dev):
    """Secondary: the dense and convection-diffusion configurations, FP64,
    one system each, run to an iteration budget (neither reaches its
    tolerance in seconds: dense Gaussian 500 x 500 needs ~1e6-1e7 CTA-2
    iterations to 1e-8, convection-diffusion 512^2 ~1e8 CTA-3 iterations to
    1e-6).  Reported: iterations/s, algorithmic GB/s (iteration_bytes), the
    relative residual reached."""
    import numpy as np

    from workloads import convection_diffusion, dense_gaussian

    out = {}
    c1 = dense_gaussian(500, seed=args.seed)
    c2 = convection_diffusion(512, seed=args.seed)
    a1 = P.to_device(np.ascontiguousarray(c1.A))
    runs = [("dense_gaussian_500_cta2", a1, c1.b, 2, False, 1e-8, 20000, (500, 500, 250000, True)),
            ("dense_gaussian_500_ta", a1, c1.b, 1, True, 1e-8, 20000, (500, 500, 250000, True)),
            ("convdiff_512_cta3", c2.A, c2.b, 3, False, 1e-6, 2000,
             (c2.A.m, c2.A.n, c2.A.nnz, False))]
    for name, A, b, t, ta, tol, budget, (m, n, nnz, dense) in runs:
        pl = P.plan(A)
        bd = torch.from_numpy(np.asarray(b)).to(dev)
        solve = (lambda: P.ta_solve(pl, bd, tol=tol, max_iter=budget, hist_cap=1)) if ta else \
            (lambda: P.cta_solve(pl, bd, tol=tol, t=t, max_iter=budget, hist_cap=1))
        solve()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, info = solve()
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        pl.close()
        ib = iteration_bytes(m, n, nnz, t, dense=dense, ta=ta)
        out[name] = {"stop": info.stop, "iterations": info.iters, "seconds": sec,
                     "iterations_per_s": info.iters / sec, "bytes_per_iteration": ib,
                     "GB_s": ib * info.iters / sec / 1e9, "rel_res": info.rel_res,
                     "tol": tol, "budget": budget}
        log(f"[bench] {name}: {info.stop} after {info.iters} iterations in {sec * 1e3:.1f} ms "
            f"({info.iters / sec:.0f} it/s, {ib * info.iters / sec / 1e9:.0f} GB/s), "
            f"rel res {info.rel_res:.3e}")
    return out


def hbm_sweep_bench(args, P, torch, dev):
    """Secondary: bandwidth of the product kernels on HBM-resident sizes --
    the LP-shaped generator at n = 1e6, 4e6, 1e7 (m = n / 100, 6 nonzeros per
    column + slack: random gathers) and the Poisson 5-point matrix at
    N^2 = 1024^2, 2048^2, 2896^2 (banded: gathers near the row's own index).
    Single-vector FP64 A and A^T passes of the solvers (the prepared
    operator's kernels) and the batched FP32 SpMM at K = 32, each timed with
    HIP events by the library's hooks; algorithmic bytes as in csr_pass_bytes.
    Past ~2e7 nonzeros the FP64 matrix (12 B per nonzero) no longer fits the
    256 MB Infinity Cache.  Then skewed rows (FP64 only): 1e6 x 1e6 with
    Pareto(1.5) row lengths of mean 8 (longest about 25000), without and with
    4 dense rows, whose A pass takes the merge-path partition."""
    import numpy as np

    from workloads import lp_shaped, poisson5, skewed_rows

    out = []
    cases = [("lp_shaped", n) for n in (1_000_000, 4_000_000, 10_000_000)]
    cases += [("poisson5", N) for N in (1024, 2048, 2896)]
    cases += [("skewed", 1_000_000), ("skewed_dense4", 1_000_000)]
    for kind, size in cases:
        t0 = time.perf_counter()
        if kind == "lp_shaped":
            Ah = lp_shaped(size // 100, size, per_col=6, seed=args.seed).A
        elif kind.startswith("skewed"):
            Ah = skewed_rows(size, size, seed=args.seed,
                             dense_rows=4 if kind == "skewed_dense4" else 0).A
        else:
            Ah = poisson5(size)
        gen_s = time.perf_counter() - t0
        m, n = Ah.m, Ah.n
        A = P.to_device(Ah)
        nnz = A.nnz
        pl = P.plan(A)
        g = np.random.default_rng([args.seed, 7])
        x = torch.from_numpy(g.standard_normal(n)).to(dev)
        u = torch.from_numpy(g.standard_normal(m)).to(dev)
        ms_a = P.time_matvec(pl, x, trans=False, reps=args.reps)
        ms_t = P.time_matvec(pl, u, trans=True, reps=args.reps)
        by_a = csr_pass_bytes(m, n, nnz, 8, 4, 8)
        by_t = csr_pass_bytes(n, m, nnz, 8, 4, 8)
        passes = [("fp64_A", by_a, ms_a), ("fp64_AT", by_t, ms_t)]
        if not kind.startswith("skewed"):
            bp = P.BatchPlan([A], "fp32")
            ms_ba = P.batch_time_spmm(bp, 32, trans=False, precision="fp32", reps=args.reps)
            ms_bt = P.batch_time_spmm(bp, 32, trans=True, precision="fp32", reps=args.reps)
            bp.close()
            passes += [("fp32_k32_A", csr_pass_bytes(m, n, nnz, 4, 4, 4, 32), ms_ba),
                       ("fp32_k32_AT", csr_pass_bytes(n, m, nnz, 4, 4, 4, 32), ms_bt)]
        row = {"matrix": kind, "size": size, "n": n, "m": m, "nnz": nnz,
               "fp64_matrix_mb": nnz * 12 / 1e6, "generated_s": gen_s,
               "format_A": pl.format(False), "format_AT": pl.format(True)}
        for key, by, ms in passes:
            gbs = by / ms / 1e6
            row[key] = {"us": ms * 1e3, "bytes": by, "GB_s": gbs, "frac": gbs / HBM_PEAK_GBS}
        out.append(row)
        msg = (f"[bench] HBM sweep {kind} {size} ({row['format_A']}, {row['format_AT']}): "
               f"FP64 A {row['fp64_A']['GB_s']:.0f} GB/s, A^T {row['fp64_AT']['GB_s']:.0f} GB/s")
        if "fp32_k32_A" in row:
            msg += (f"; FP32 K=32 A {row['fp32_k32_A']['GB_s']:.0f} GB/s, "
                    f"A^T {row['fp32_k32_AT']['GB_s']:.0f} GB/s")
        log(msg)
        del pl, A, x, u, Ah
        torch.cuda.empty_cache()
    return out


def dense_products_bench(args, P, torch, dev):
    """Secondary: the dense multi-right-hand-side products (matrix cores for
    BF16 / FP32, the compensated CSR copy for FP64) on 4 dense Gaussian
    systems of 4096^2, A pass at K = 64, 16 and 1, HIP events through the
    library's hook; bytes = the matrix in its precision plus the input and
    output blocks, flops = 2 n^2 K per system."""
    import numpy as np

    n, nsys = 4096, 4
    g = np.random.default_rng([args.seed, 4096])
    mats = [g.standard_normal((n, n)) for _ in range(nsys)]
    out = []
    for prec, vb, xb in (("bf16", 2, 4), ("fp32", 4, 4), ("fp64", 8, 8)):
        plan = P.BatchPlan(mats, prec)
        for K in (64, 16, 1):
            ms = P.batch_time_spmm(plan, K, trans=False, precision=prec, reps=args.reps)
            by = nsys * (n * n * vb + 2 * n * K * xb)
            fl = nsys * 2 * n * n * K
            out.append({"precision": prec, "K": K, "us": ms * 1e3, "TFLOP_s": fl / ms / 1e9,
                        "GB_s": by / ms / 1e6, "hbm_bound_us": by / HBM_PEAK_GBS / 1e3,
                        "frac": by / ms / 1e6 / HBM_PEAK_GBS})
            log(f"[bench] dense {nsys} x {n}^2 {prec} K={K}: {ms * 1e3:.1f} us, "
                f"{fl / ms / 1e9:.1f} TFLOP/s, {by / ms / 1e6:.0f} GB/s")
        plan.close()
        torch.cuda.empty_cache()
    return out


def traffic_record(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv):
    """Write the HBM traffic record of the dominant kernel (TRAFFIC_FILE)
    from four rocprofv3 counter collections (csv): FETCH_SIZE and WRITE_SIZE
    of this script's default run filtered to k_bspmm, and of --copy-calibration.
    The timing hook's last four runs of >= 20 back-to-back launches of the
    FP32 K = 64 kernel, in the order the script times them (part 0 A, A^T,
    part 1 A, A^T), each averaged over its last 20 (timed) launches, are
    scaled by the copy's counts per GiB; the record
    carries the SHA-256 of the kernel source, which measured_traffic checks."""
    import collections
    import csv
    import hashlib
    import statistics

    def dispatches(path):
        d = collections.OrderedDict()
        with open(path) as f:
            for r in csv.DictReader(f):
                k = int(r["Dispatch_Id"])
                e = d.setdefault(k, {"name": r["Kernel_Name"], "grid": int(r["Grid_Size"]),
                                     "val": 0.0})
                e["val"] += float(r["Counter_Value"])
        return list(d.items())

    def runs(path, name):
        items = [(k, v) for k, v in dispatches(path) if v["name"].startswith(name)]
        out, i = [], 0
        while i < len(items):
            j = i
            while (j + 1 < len(items) and items[j + 1][1]["grid"] == items[i][1]["grid"]
                   and items[j + 1][0] == items[j][0] + 1):
                j += 1
            if j - i + 1 >= 20:  # the last 20: the timed launches after tuning and warm-up
                out.append((items[i][1]["grid"],
                            statistics.mean(x[1]["val"] for x in items[j - 19:j + 1])))
            i = j + 1
        return out[-4:]  # the hook's runs come after the solve's own tuning

    def copy_kib(path):
        vals = [v["val"] for _, v in dispatches(path) if "copyBuffer" in v["name"]]
        return statistics.median(vals)

    gib = 2 ** 30 / 1024
    fcopy, wcopy = copy_kib(copy_fetch_csv), copy_kib(copy_write_csv)
    name = "void ta::bt::k_bspmm<float, float, 64, 0, 6"
    fr, wr = runs(fetch_csv, name), runs(write_csv, name)
    if len(fr) != 4 or len(wr) != 4:
        raise SystemExit(f"expected 4 timed launch runs, found {len(fr)} and {len(wr)}")
    keys = [("A", 0), ("AT", 0), ("A", 1), ("AT", 1)]
    entries = []
    for (ps, part), (grid, fk), (_, wk) in zip(keys, fr, wr):
        entries.append({"precision": "fp32", "K": 64, "pass": ps, "part": part, "grid": grid,
                        "fetch_kib": round(fk, 1), "write_kib": round(wk, 1),
                        "bytes_per_launch": int(round((fk * gib / fcopy + wk * gib / wcopy) * 1024))})
    with open(KERNEL_SRC, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    rec = {"kernel": "k_bspmm<float, float, 64, 0, 6>",
           "workload": "batched uneven systems (seed 0), K = 64 width group, one launch per "
                       "row-length part, the timing hook's 20 timed launches",
           "kernel_source": "paper_2304_12168_amd/csrc/batched.hip",
           "kernel_source_sha256": sha,
           "copy_calibration": {"fetch_kib_per_GiB": fcopy, "write_kib_per_GiB": wcopy,
                                "fetch_scale": gib / fcopy, "write_scale": gib / wcopy},
           "entries": entries}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(rec, f, indent=1)
    log(f"[bench] traffic record written: {TRAFFIC_FILE}")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--budget", type=int, default=400, help="iterations per column")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp64"])
    ap.add_argument("--plain-sample", type=int, default=24,
                    help="columns solved one at a time for the FP64 plain rate")
    ap.add_argument("--cpu-sample", type=int, default=48,
                    help="columns solved by the CPU oracle for the CPU baseline")
    ap.add_argument("--reps", type=int, default=20, help="launches per kernel timing")
    ap.add_argument("--lp-steps", type=int, default=5)
    ap.add_argument("--no-lp", action="store_true", help="skip the LP-shaped secondary block")
    ap.add_argument("--no-diff", action="store_true",
                    help="skip the differentiable-solve secondary block")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the CTA-variants secondary block")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the HBM-resident size sweep of the product kernels")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bf16", action="store_true", help="skip the BF16 batched leg")
    ap.add_argument("--sweep-only", action="store_true",
                    help="only the HBM-resident size sweep of the product kernels and the "
                         "dense products (for profiling them), printed as one JSON line")
    ap.add_argument("--traffic-record", nargs=4, metavar="CSV",
                    help="write the dominant kernel's traffic record from the FETCH_SIZE and "
                         "WRITE_SIZE counter csv files of a default run and of "
                         "--copy-calibration (in that order), and exit; needs no GPU")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB on the device three times (the reference kernel "
                         "that scales the HBM traffic counters) and exit")
    args = ap.parse_args()
    if args.traffic_record:
        traffic_record(*args.traffic_record)
        return
    if args.copy_calibration:
        import torch

        a = torch.ones(2 ** 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("[bench] copied 1 GiB three times")
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU layout is described, not built)", file=sys.stderr)
        sys.exit(2)

    # the CPU baseline's worker processes are forked first, before the GPU is
    # initialised, so that none of them holds GPU state
    pool = None if args.no_cpu_baseline else make_cpu_pool()

    import torch

    import paper_2304_12168_amd as P

    if not torch.cuda.is_available():
        log("no GPU visible")
        sys.exit(1)
    P.load_library()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.sweep_only:
        print(json.dumps({"hbm_sweep": hbm_sweep_bench(args, P, torch, dev),
                          "dense_products": dense_products_bench(args, P, torch, dev)}),
              flush=True)
        return
    res = batched_uneven_bench(args, P, torch, dev, pool)
    if pool is not None:
        pool[0].close()
        pool[0].join()
    if not args.no_lp:
        res["config"]["lp_shaped"] = lp_shaped_bench(args, P, torch, dev)
    if not args.no_diff:
        res["config"]["differentiable"] = diff_bench(args, P, torch, dev)
    if not args.no_variants:
        res["config"]["variants"] = variants_bench(args, P, torch, dev)
        res["config"]["configs"] = configs_bench(args, P, torch, dev)
    if not args.no_sweep:
        res["config"]["hbm_sweep"] = hbm_sweep_bench(args, P, torch, dev)
        res["config"]["dense_products"] = dense_products_bench(args, P, torch, dev)
    out = {
        "metric": "solves/s and HBM GB/s to rel-residual 1e-6: CTA mixed+batched vs FP64 plain",
        "value": res["value"],
        "unit": "columns solved to 1e-6 per second",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32/f64", "bf16": "bf16/f32/f64", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": res["config"],
        "roofline": res["roofline"],
        "cpu_baseline": res["cpu_baseline"],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
