#!/usr/bin/env python
"""Throughput of the MI355X EN-PT2 / CIPSI-selection sweep.

A step is one qp_pt2 call (generator ordering, per-generator preparation,
coarse filter, the batch sweep, reductions and the top-N selection) over the
seeded synthetic workload, with all inputs already resident in HBM.  The
metric is external determinants (|A|) per second.  Besides the one JSON line
on stdout, progress goes to stderr.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]

Besides the headline forward sweep it reports, in "extra": the forward +
adjoint throughput of the same workload, and the batched workload (64
independent systems, n_orb in {32,48,64,96}, 4-12 electrons per spin,
100-20,000 determinants, 1-3 states) run as one qp_pt2_batched call, forward
and forward + adjoint, against one qp_pt2 call per system on the same GPU.
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


# HBM traffic of one dense-kernel launch, from two rocprofv3 --pmc runs (FETCH_SIZE, then
# WRITE_SIZE) scaled by the same counters on a 1 GiB device copy.  Valid only for the kernel
# sources it was measured on (SHA-256 of DENSE_SOURCES); reported as null otherwise.
DENSE_SOURCES = ["qp_dev.h", "qp_fast_caps.h", "qp_fast_impl.h", "qp_fast_fwd.hip"]
MEASURED_TRAFFIC = {
    "c2_n64_10a10b_1e4det_top1000": {
        "sources_sha256": "136aac2bf4ee8ed9b10794d64b97884de7437c521ccd2e8cb316910538bdfffc",
        "bytes": 44599648000 + 46649760,
    },
}


def dense_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in DENSE_SOURCES:
        with open(os.path.join(ROOT, "paper_1902_08154_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def ops_per_alpha(stats, ns, nint):
    """Method-intrinsic lane operations per external determinant: the ban test
    (3), the per-state FP64 work (15: the element's phase and scaling, the
    diagonal update, the denominator, the energy and its two accumulations, the
    selection test) and, for each connection to a non-generator J, the
    excitation analysis on 2*n_int words (12 per word) plus 2 FP64 per state
    (connections per alpha averaged over the sweep)."""
    conn = stats["n_connections"] / max(stats["n_alpha"], 1)
    return 3.0 + 15.0 * ns + (12.0 * nint + 2.0 * ns) * conn


def cpu_baseline(s, E0, n_gen):
    from oracle import oracle
    rank = oracle.generator_rank(s.dets, s.coefs)
    order = np.argsort(rank)
    pick = order[np.linspace(0, s.n_det - 1, n_gen).astype(np.int64)]
    t0 = time.perf_counter()
    r = oracle.eps_generators(s.n_orb, s.h, s.eri, s.dets, s.coefs, E0, pick)
    dt = time.perf_counter() - t0
    return dict(value=float(r.count.sum()) / dt, unit="alpha/s",
                cores=int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0)))),
                kind="oracle",
                sample=f"{n_gen} generators evenly spaced in generator order ({int(r.count.sum())} alpha, {dt:.1f} s)")


def batched_bench(ctx, dev, steps):
    """The 64-system workload through qp_pt2_batched (forward, then forward +
    adjoint in one adjoint sweep), and the same systems as one qp_pt2 call
    each.  Integral layouts are built once, outside the timed region, as for
    the single-system workload."""
    import torch
    from paper_1902_08154_amd import synth
    from paper_1902_08154_amd.api import to_device_dets
    t0 = time.perf_counter()
    ws = synth.batched_workload()
    log(f"batched workload: {len(ws)} systems, {sum(w.n_det for w in ws)} determinants "
        f"(generated in {time.perf_counter() - t0:.1f} s)")
    ins = []
    for w in ws:
        h = torch.from_numpy(w.h).to(dev)
        eri = torch.from_numpy(w.eri).to(dev)
        ctx.qp_set_integrals(h, eri)
        dets = to_device_dets(w.dets, dev)
        coefs = torch.from_numpy(w.coefs).to(dev)
        ins.append(dict(h=h, eri_packed=eri, dets=dets, coefs=coefs, E0=ctx.energy(dets, coefs)))
    torch.cuda.synchronize()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps, r

    t_f, r_f = timed(lambda: ctx.pt2_batched(ins, reuse_integrals=True))
    n_alpha = sum(x["stats"]["n_alpha"] for x in r_f)
    n_cells = sum(x["stats"]["n_cells"] for x in r_f)
    t_fb, _ = timed(lambda: ctx.pt2_batched(ins, with_backward=True, reuse_integrals=True))

    def one_by_one():
        # one forward call per system; each system's layouts are the context's,
        # so they are rebuilt per call: that rebuild is timed on its own below
        for y in ins:
            ctx.qp_set_integrals(y["h"], y["eri_packed"])
            ctx.pt2(y["dets"], y["coefs"], y["E0"])

    def layouts_only():
        for y in ins:
            ctx.qp_set_integrals(y["h"], y["eri_packed"])

    t_seq, _ = timed(one_by_one)
    t_lay, _ = timed(layouts_only)
    out = {"workload": "c4_64sys_n32-96_4-12e_100-20000det_1-3st", "n_systems": len(ws),
           "n_det_total": int(sum(w.n_det for w in ws)), "n_alpha": n_alpha, "n_cells": n_cells,
           "fwd_ms": 1e3 * t_f, "fwd_alpha_per_s": n_alpha / t_f,
           "fwd_bwd_ms": 1e3 * t_fb, "fwd_bwd_alpha_per_s": n_alpha / t_fb,
           "one_call_per_system_fwd_ms": 1e3 * (t_seq - t_lay),
           "one_call_per_system_fwd_alpha_per_s": n_alpha / (t_seq - t_lay)}
    log(f"batched: fwd {1e3 * t_f:.1f} ms, fwd+bwd {1e3 * t_fb:.1f} ms, one call per system "
        f"{1e3 * (t_seq - t_lay):.1f} ms (+{1e3 * t_lay:.1f} ms of layout rebuilds), |A| = {n_alpha}")
    return out


def next_rows_bench(ctx, dev, s, dets, coefs, E0, steps):
    """The rows built on the sweep, on the same workload: the semi-stochastic
    E_PT2 to |dE/E| = 0.002 (against a deterministic sweep without selection),
    the sigma-build W = H U and W = S^2 U, and the Davidson diagonaliser started
    from the wave function's own coefficients."""
    import torch
    from paper_1902_08154_amd import synth

    def timed(fn):
        r = fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            r = fn()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t) / steps, r

    out = {}
    # the batched leg leaves the context's integrals at its last system's
    ctx.qp_set_integrals(torch.from_numpy(s.h).to(dev), torch.from_numpy(s.eri).to(dev))
    torch.cuda.synchronize()
    t_det, r_det = timed(lambda: ctx.pt2(dets, coefs, E0))
    u = synth.uniforms(2019, 200000)
    t_sto, g = timed(lambda: ctx.pt2_stochastic(dets, coefs, E0, u, rel_err=0.002, det_chunk=256,
                                                draws_per_round=1024))
    out["semistochastic"] = {"rel_err": 0.002, "det_chunk": 256, "draws_per_round": 1024, "ms": t_sto,
                             "deterministic_ms": t_det,
                             "n_computed": g["n_computed"], "n_det": s.n_det, "n_rounds": g["n_rounds"],
                             "e_pt2": float(g["e_pt2"][0]), "err": float(g["err"][0]),
                             "e_pt2_deterministic": float(r_det["e_pt2"][0].item())}
    log(f"semi-stochastic: {t_sto:.1f} ms ({g['n_computed']} of {s.n_det} generators, {g['n_rounds']} rounds), "
        f"deterministic {t_det:.1f} ms")
    gen = torch.Generator().manual_seed(7)
    U4 = torch.rand((4, s.n_det), generator=gen, dtype=torch.float64).to(dev)
    sig = {}
    for name, U, s2 in (("H_1vec", coefs, False), ("H_4vec", U4, False), ("S2_1vec", coefs, True)):
        sig[name + "_ms"], _ = timed(lambda: ctx.sigma(dets, U, s2=s2))
    # the same determinants again: the prepared space is reused (QP_SIGMA_REUSE)
    sig["H_1vec_reuse_ms"], _ = timed(lambda: ctx.sigma(dets, coefs, reuse=True))
    out["sigma"] = sig
    t0 = time.perf_counter()
    r = ctx.davidson(dets, n_states=1, guess=coefs, tol=1e-8, max_iter=400)
    torch.cuda.synchronize()
    out["davidson"] = {"ms": 1e3 * (time.perf_counter() - t0), "n_iter": r["n_iter"], "tol": 1e-8,
                       "E": float(r["E"][0])}
    log(f"sigma-build: {sig}; davidson {out['davidson']['ms']:.1f} ms, {r['n_iter']} iterations")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--bwd-steps", type=int, default=2)
    ap.add_argument("--batched-steps", type=int, default=2,
                    help="timed repetitions of the 64-system batched workload (0: skip it)")
    ap.add_argument("--next-steps", type=int, default=1,
                    help="timed repetitions of the semi-stochastic PT2 and the sigma-build (0: skip them)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the steps, copy MIB MiB device to device once: a transfer of known size "
                         "against which the HBM traffic counters of the sweep are scaled")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: the library has no multi-GPU path (the design notes describe how "
              "the sweep would shard over generators)", file=sys.stderr)
        sys.exit(2)

    import ctypes
    import torch
    from paper_1902_08154_amd import _lib, synth
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
    st = torch.zeros(ctypes.sizeof(_lib.Stats), dtype=torch.uint8, device=dev)

    def step():
        ctx.qp_pt2(dets, coefs, E0, nsel, 0, e_out, sd, se, nsl, st, None)

    ctx.qp_set_timing(True)
    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        tm = ctx.qp_last_timing()
        log(f"warmup {i}: dense kernel {tm[0]:.2f} ms, general kernel {tm[1]:.2f} ms, call {tm[2]:.2f} ms")
    timings = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        timings.append(ctx.qp_last_timing())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    from paper_1902_08154_amd.api import stats_to_dict
    stats = stats_to_dict(st, ns)
    ms_per_step = 1e3 * elapsed / args.steps
    value = stats["n_alpha"] * args.steps / elapsed
    # the dominant kernel: the dense sweep, timed with HIP events on its stream
    kern_s = float(np.mean([t[0] for t in timings])) * 1e-3
    gen_ms = float(np.mean([t[1] for t in timings]))
    alpha_dense = stats["n_alpha"] - stats["n_alpha_general"]
    per_alpha = ops_per_alpha(stats, ns, nint)
    ops = alpha_dense * per_alpha
    log(f"E_PT2 = {e_out.cpu().numpy()}  |A| = {stats['n_alpha']} (general kernel {stats['n_alpha_general']})  "
        f"cells = {stats['n_cells']}  step {ms_per_step:.2f} ms  dense kernel {1e3 * kern_s:.2f} ms  "
        f"general kernel {gen_ms:.2f} ms")

    # forward + backward throughput
    extra = {"general_kernel_ms": gen_ms, "alpha_general_kernel": stats["n_alpha_general"],
             "e_pt2": e_out.cpu().tolist(), "rpt2_Z": stats["Z"], "e_rpt2": stats["e_rpt2"]}
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

    if args.batched_steps > 0:
        extra["batched"] = batched_bench(ctx, dev, args.batched_steps)

    if args.next_steps > 0:
        extra["next"] = next_rows_bench(ctx, dev, s, dets, coefs, E0, args.next_steps)

    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calibration} MiB read + {args.copy_calibration} MiB written")
        del src, dst

    cpu = None
    if not args.no_cpu_baseline:
        # the oracle's OpenMP team: OMP_NUM_THREADS if set, else every CPU of the affinity mask;
        # about 12 generators per thread keep the sample near 15 s of CPU work
        threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
        cpu = cpu_baseline(s, E0.cpu().numpy(), 12 * threads)
        log(f"cpu baseline: {cpu}")

    mt = MEASURED_TRAFFIC.get(s.name)
    traffic = mt["bytes"] if mt and mt["sources_sha256"] == dense_sources_sha256() else None

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
                     "unit": "Tops/s", "frac": ops / kern_s / ALU_PEAK_OPS, "traffic": traffic,
                     "kernel": "qpfast::fast_kernel", "kernel_ms": 1e3 * kern_s, "ops_per_launch": ops,
                     "alpha_per_launch": alpha_dense, "ops_per_alpha": per_alpha},
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
