#!/usr/bin/env python
"""Throughput of the MI355X EN-PT2 / CIPSI-selection sweep.

A step is one qp_pt2 call (generator ordering, per-generator preparation,
coarse filter, the batch sweep, reductions and the top-N selection) over the
seeded synthetic workload, with all inputs already resident in HBM.  The
metric is external determinants (|A|) per second.  Besides the one JSON line
on stdout, progress goes to stderr.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "external determinants/sec (PT2 fwd, fwd+bwd, batched) + achieved HBM GB/s fraction"
# MI355X: 256 CUs x 64 lanes x 2.4 GHz = one 32/64-bit lane operation per lane per clock
ALU_PEAK_OPS = 256 * 64 * 2.4e9
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_ops(stats, ns, nint):
    """Method-intrinsic lane operations of one sweep: a ban test per candidate
    cell (3), the per-state FP64 work of each external determinant (15: the
    element's phase and scaling, the diagonal update, the denominator, the
    energy and its two accumulations, the selection test) and, per connection
    to a non-generator J, the excitation analysis on 2*n_int words (12 per word)
    plus 2 FP64 per state."""
    return (3.0 * stats["n_cells"] + 15.0 * ns * stats["n_alpha"]
            + (12.0 * nint + 2.0 * ns) * stats["n_connections"])


def cpu_baseline(s, E0, n_gen):
    from oracle import oracle
    rank = oracle.generator_rank(s.dets, s.coefs)
    order = np.argsort(rank)
    pick = order[np.linspace(0, s.n_det - 1, n_gen).astype(np.int64)]
    t0 = time.perf_counter()
    r = oracle.eps_generators(s.n_orb, s.h, s.eri, s.dets, s.coefs, E0, pick)
    dt = time.perf_counter() - t0
    return dict(value=float(r.count.sum()) / dt, unit="alpha/s", cores=int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0)))),
                kind="oracle",
                sample=f"{n_gen} generators evenly spaced in generator order ({int(r.count.sum())} alpha, {dt:.1f} s)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--bwd-steps", type=int, default=2)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: this build has no multi-GPU path (see the sharding note in the "
              "design document)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1902_08154_amd import synth
    from paper_1902_08154_amd.api import Context, to_device_dets

    idx = int(args.workload[1:])
    t0 = time.perf_counter()
    s = synth.workload(idx)
    log(f"workload {s.name}: n_orb={s.n_orb} {s.n_up}+{s.n_dn} e-, n_det={s.n_det}, "
        f"states={s.n_states}, n_select={s.n_select} (generated in {time.perf_counter() - t0:.1f} s)")
    dev = torch.device("cuda", 0)
    ctx = Context(0)
    ctx.qp_set_integrals(torch.from_numpy(s.h).to(dev), torch.from_numpy(s.eri).to(dev))
    dets = to_device_dets(s.dets, dev)
    coefs = torch.from_numpy(s.coefs).to(dev)
    E0 = ctx.energy(dets, coefs)
    torch.cuda.synchronize()
    log(f"E0 = {E0.cpu().numpy()}")

    ns, nd, nint = s.n_states, s.n_det, s.n_int
    nsel = s.n_select
    e_out = torch.empty(ns, dtype=torch.float64, device=dev)
    sd = torch.empty((max(nsel, 1), 2, nint), dtype=torch.int64, device=dev)
    se = torch.empty((max(nsel, 1), ns), dtype=torch.float64, device=dev)
    nsl = torch.zeros(1, dtype=torch.int64, device=dev)
    st = torch.zeros(128, dtype=torch.uint8, device=dev)

    def step():
        ctx.qp_pt2(dets, coefs, E0, nsel, 0, e_out, sd, se, nsl, st, None)

    ctx.qp_set_timing(True)
    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i}: sweep {ctx.qp_last_timing()[0]:.2f} ms")
    sweep_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        sweep_ms.append(ctx.qp_last_timing()[0])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    from paper_1902_08154_amd.api import stats_to_dict
    stats = stats_to_dict(st, ns)
    ms_per_step = 1e3 * elapsed / args.steps
    value = stats["n_alpha"] * args.steps / elapsed
    kern_s = float(np.mean(sweep_ms)) * 1e-3
    ops = algorithmic_ops(stats, ns, nint)
    log(f"E_PT2 = {e_out.cpu().numpy()}  |A| = {stats['n_alpha']}  cells = {stats['n_cells']}  "
        f"step {ms_per_step:.2f} ms  sweep kernel {1e3 * kern_s:.2f} ms")

    # forward + backward throughput
    extra = {}
    if args.bwd_steps > 0:
        gup = torch.ones(ns, dtype=torch.float64, device=dev)
        gc = torch.empty((ns, nd), dtype=torch.float64, device=dev)
        gE = torch.empty(ns, dtype=torch.float64, device=dev)
        gh = torch.empty((s.n_orb, s.n_orb), dtype=torch.float64, device=dev)
        ctx.qp_pt2_backward(dets, coefs, E0, gup, 0, gc, gE, gh, None)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for i in range(args.bwd_steps):
            step()
            ctx.qp_pt2_backward(dets, coefs, E0, gup, 0, gc, gE, gh, None)
        torch.cuda.synchronize()
        fb = (time.perf_counter() - t1) / args.bwd_steps
        extra["fwd_bwd_alpha_per_s"] = stats["n_alpha"] / fb
        extra["fwd_bwd_ms_per_step"] = 1e3 * fb
        log(f"fwd+bwd {1e3 * fb:.2f} ms/step")

    cpu = None
    if not args.no_cpu_baseline:
        ncores = len(os.sched_getaffinity(0))
        cpu = cpu_baseline(s, E0.cpu().numpy(), max(8, min(ncores, 32)))
        log(f"cpu baseline: {cpu}")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "alpha/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": s.name, "n_orb": s.n_orb, "n_up": s.n_up, "n_dn": s.n_dn,
                   "n_det": s.n_det, "n_states": ns, "n_select": nsel, "seed": s.seed,
                   "n_alpha": stats["n_alpha"], "n_cells": stats["n_cells"]},
        "roofline": {"bound": "alu", "achieved": ops / kern_s / 1e12, "peak": ALU_PEAK_OPS / 1e12,
                     "unit": "Tops/s", "frac": ops / kern_s / ALU_PEAK_OPS, "traffic": None,
                     "kernel": "sweep_kernel", "kernel_ms": 1e3 * kern_s, "ops_per_launch": ops},
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
