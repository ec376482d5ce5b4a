#!/usr/bin/env python
"""Throughput of the MI355X EN-PT2 / CIPSI-selection sweep.

A step is one pass of the whole hot path over the seeded synthetic workload,
with all inputs already resident in HBM: the forward sweep with its top-N
selection (qp_pt2: generator ordering, per-generator preparation, coarse
filter, the batch sweep, reductions and selection) followed by the adjoint
sweep (qp_pt2_backward: dE/dc, dE/dE0, dE/dh).  The headline workload is the
largest single-GPU one: n_orb 256 (four words per spin), 16+16 electrons,
10^6 determinants, 2 states, top-10^5.  The metric is external determinants
(|A|) per second of the step.  Besides the one JSON line on stdout, progress
goes to stderr.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c5]

In "extra": the forward sweep alone, the n_orb 64 workload (10+10 electrons,
10^4 determinants, top-1000: forward, forward + adjoint, the dense kernel's
roofline and measured traffic), the batched workload (64 independent
systems, n_orb in {32,48,64,96}, 4-12 electrons per spin, 100-20,000
determinants, 1-3 states) as one qp_pt2_batched call against one qp_pt2 call
per system, and the rows built on the sweep (semi-stochastic PT2,
sigma-build, Davidson) on the n_orb 64 workload.
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


# HBM traffic of one launch of the dominant kernel, from two rocprofv3 --pmc runs (FETCH_SIZE,
# then WRITE_SIZE) scaled by the same counters on a device copy of known size.  Valid only for
# the kernel sources it was measured on (SHA-256 of the kernel's sources); reported as null
# otherwise.  The dominant kernel is the adjoint clean-cell kernel of a split sweep, else the
# forward dense kernel.
CLEAN_SOURCES = ["qp_dev.h", "qp_lean.hip"]
DENSE_SOURCES = ["qp_dev.h", "qp_fast_caps.h", "qp_fast_impl.h", "qp_fast_fwd.hip"]
MEASURED_TRAFFIC = {
    # adjoint clean-cell launch: FETCH_SIZE 993,539,733.4 KiB x 2.000 (a 1 GiB device copy reads
    # 524,316.4 KiB) + WRITE_SIZE 77,483,339.1 KiB x 1.000 (the copy writes 1,048,576 KiB)
    "c5_n256_16a16b_1e6det_2st_top1e5": {
        "sources_sha256": "15f974cb5f8cd376b38e3e5ee54bb6500cc25d9a37eff2106afd56dab7fed85f",
        "bytes": 2114002195515.0,
    },
    # forward dense launch: FETCH_SIZE 21,773,386.3 KiB x 2.000 (the 1 GiB copy reads 524,306.5 KiB)
    # + WRITE_SIZE 45,657.3 KiB x 1.000
    "c2_n64_10a10b_1e4det_top1000": {
        "sources_sha256": "915e54199ba634a1b4f4859df8ceadf4f06b86eb5279fd1da3f206f5c4babd8c",
        "bytes": 44637074684.0,
    },
}


def clean_sources_sha256(sources=CLEAN_SOURCES):
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_1902_08154_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def clean_ops_per_alpha(ns, adjoint):
    """Method-intrinsic lane operations per external determinant that only its
    generator reaches (a clean cell): the per-state FP64 work of the forward
    sweep (15, as in ops_per_alpha; no ban test and no connection: the batch's
    filter has settled both), and for the adjoint 4 more per state (the weight
    2 g A / delta and the diagonal share g A^2 / delta^2) plus 2 (that share's
    row and column accumulation)."""
    return 15.0 * ns + ((4.0 * ns + 2.0) if adjoint else 0.0)


def cpu_baseline(s, E0, n_gen, visit_cap=0, threads=0):
    """The oracle's per-generator sweep on n_gen generators evenly spaced in
    generator order; visit_cap > 0 bounds each to its first visit_cap
    excitations (enumeration order), for workloads whose generators take
    minutes each on one core."""
    from oracle import oracle
    rank = oracle.generator_rank(s.dets, s.coefs)
    order = np.argsort(rank)
    pick = order[np.linspace(0, s.n_det - 1, n_gen).astype(np.int64)]
    t0 = time.perf_counter()
    r = oracle.eps_generators(s.n_orb, s.h, s.eri, s.dets, s.coefs, E0, pick, visit_cap=visit_cap, threads=threads)
    dt = time.perf_counter() - t0
    what = f"the first {visit_cap} excitations of each of " if visit_cap else ""
    return dict(value=float(r.count.sum()) / dt, unit="alpha/s",
                cores=threads or int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0)))),
                kind="oracle",
                sample=f"{what}{n_gen} generators evenly spaced in generator order "
                       f"({int(r.count.sum())} alpha, {dt:.1f} s)")


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
    the sigma-build W = H U and W = S^2 U, and the Davidson diagonaliser from
    its default start (the lowest root)."""
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
    # the same run selecting the top n_select alpha of its computed generators
    # on the fly, against the deterministic sweep with its selection
    t_dsel, _ = timed(lambda: ctx.pt2(dets, coefs, E0, n_select=s.n_select))
    t_ssel, gs = timed(lambda: ctx.pt2_stochastic(dets, coefs, E0, u, rel_err=0.002, det_chunk=256,
                                                  draws_per_round=1024, n_select=s.n_select))
    out["semistochastic"].update({"with_selection_ms": t_ssel, "n_select": s.n_select,
                                  "n_selected": int(gs["sel_e"].shape[0]),
                                  "deterministic_with_selection_ms": t_dsel})
    log(f"semi-stochastic: {t_sto:.1f} ms ({g['n_computed']} of {s.n_det} generators, {g['n_rounds']} rounds), "
        f"deterministic {t_det:.1f} ms; with selection of {s.n_select}: {t_ssel:.1f} ms, deterministic "
        f"{t_dsel:.1f} ms")
    gen = torch.Generator().manual_seed(7)
    U4 = torch.rand((4, s.n_det), generator=gen, dtype=torch.float64).to(dev)
    sig = {}
    for name, U, s2 in (("H_1vec", coefs, False), ("H_4vec", U4, False), ("S2_1vec", coefs, True)):
        sig[name + "_ms"], _ = timed(lambda: ctx.sigma(dets, U, s2=s2))
    # the same determinants again: the prepared space is reused (QP_SIGMA_REUSE)
    sig["H_1vec_reuse_ms"], _ = timed(lambda: ctx.sigma(dets, coefs, reuse=True))
    out["sigma"] = sig
    t0 = time.perf_counter()
    # from the default start (the unit vector of the lowest diagonal element):
    # the lowest root
    r = ctx.davidson(dets, n_states=1, guess=None, tol=1e-8, max_iter=400)
    torch.cuda.synchronize()
    out["davidson"] = {"ms": 1e3 * (time.perf_counter() - t0), "n_iter": r["n_iter"], "tol": 1e-8,
                       "start": "lowest diagonal element",
                       "E": float(r["E"][0])}
    log(f"sigma-build: {sig}; davidson {out['davidson']['ms']:.1f} ms, {r['n_iter']} iterations")
    return out


def load_workload(ctx, dev, idx):
    import torch
    from paper_1902_08154_amd import synth
    from paper_1902_08154_amd.api import to_device_dets
    t0 = time.perf_counter()
    s = synth.workload(idx)
    log(f"workload {s.name}: n_orb={s.n_orb} {s.n_up}+{s.n_dn} e-, n_det={s.n_det}, "
        f"states={s.n_states}, n_select={s.n_select} (generated in {time.perf_counter() - t0:.1f} s)")
    ctx.qp_set_integrals(torch.from_numpy(s.h).to(dev), torch.from_numpy(s.eri).to(dev))
    dets = to_device_dets(s.dets, dev)
    coefs = torch.from_numpy(s.coefs).to(dev)
    E0 = ctx.energy(dets, coefs)
    torch.cuda.synchronize()
    log(f"E0 = {E0.cpu().numpy()}")
    return s, dets, coefs, E0


class Sweep:
    """Output buffers of one workload's forward and adjoint calls, allocated
    once, outside the timed region."""

    def __init__(self, ctx, dev, s, dets, coefs, E0):
        import ctypes
        import torch
        from paper_1902_08154_amd import _lib
        self.ctx, self.s, self.dets, self.coefs, self.E0 = ctx, s, dets, coefs, E0
        ns, nd, nint, nsel = s.n_states, s.n_det, s.n_int, s.n_select
        self.e_out = torch.empty(ns, dtype=torch.float64, device=dev)
        self.sd = torch.empty((max(nsel, 1), 2, nint), dtype=torch.int64, device=dev)
        self.se = torch.empty((max(nsel, 1), ns), dtype=torch.float64, device=dev)
        self.nsl = torch.zeros(1, dtype=torch.int64, device=dev)
        self.st = torch.zeros(ctypes.sizeof(_lib.Stats), dtype=torch.uint8, device=dev)
        self.stb = torch.zeros(ctypes.sizeof(_lib.Stats), dtype=torch.uint8, device=dev)
        self.gup = torch.ones(ns, dtype=torch.float64, device=dev)
        self.gc = torch.empty((ns, nd), dtype=torch.float64, device=dev)
        self.gE = torch.empty(ns, dtype=torch.float64, device=dev)
        self.gh = torch.empty((s.n_orb, s.n_orb), dtype=torch.float64, device=dev)

    def forward(self):
        self.ctx.qp_pt2(self.dets, self.coefs, self.E0, self.s.n_select, 0, self.e_out, self.sd, self.se,
                        self.nsl, self.st, None)

    def backward(self):
        self.ctx.qp_pt2_backward(self.dets, self.coefs, self.E0, self.gup, 0, self.gc, self.gE, self.gh, self.stb)

    def stats(self, adjoint=False):
        from paper_1902_08154_amd.api import stats_to_dict
        return stats_to_dict(self.stb if adjoint else self.st, self.s.n_states)


def filter_figures(s, stats):
    """The coarse and fine filters' reductions (the paper's filtering figure):
    coarse entries per generator against |Psi|, fine entries per hole batch
    against the coarse entries per generator."""
    nel = s.n_up + s.n_dn
    batches = s.n_det * (nel + nel * (nel - 1) // 2)
    coarse = stats["n_coarse"] / s.n_det
    fine = stats["n_fine"] / batches
    return {"coarse_per_generator": coarse, "coarse_over_psi": coarse / s.n_det,
            "fine_per_batch": fine, "fine_over_coarse": fine / coarse if coarse else None,
            "clean_alpha_fraction": stats["n_alpha_clean"] / max(stats["n_alpha"], 1)}


def small_leg(ctx, dev, steps, bwd_steps):
    """The n_orb 64 workload: forward steps and forward + adjoint steps."""
    import torch
    s, dets, coefs, E0 = load_workload(ctx, dev, 2)
    w = Sweep(ctx, dev, s, dets, coefs, E0)
    w.forward()
    w.backward()
    torch.cuda.synchronize()
    tms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        w.forward()
        tms.append(ctx.qp_last_timing())
    torch.cuda.synchronize()
    tf = (time.perf_counter() - t0) / steps
    stats = w.stats()
    t1 = time.perf_counter()
    for _ in range(bwd_steps):
        w.forward()
        w.backward()
    torch.cuda.synchronize()
    tfb = (time.perf_counter() - t1) / max(bwd_steps, 1)
    out = {"workload": s.name, "n_alpha": stats["n_alpha"], "fwd_ms": 1e3 * tf,
           "fwd_alpha_per_s": stats["n_alpha"] / tf, "fwd_bwd_ms": 1e3 * tfb,
           "fwd_bwd_alpha_per_s": stats["n_alpha"] / tfb,
           "kernel_ms": {"dense": float(np.mean([t[0] for t in tms])),
                         "general": float(np.mean([t[1] for t in tms])),
                         "clean_cell": float(np.mean([t[4] for t in tms])),
                         "clean_cell_and_split_correction": float(np.mean([t[3] for t in tms]))},
           "filter": filter_figures(s, stats), "e_pt2": w.e_out.cpu().tolist()}
    log(f"{s.name}: fwd {1e3 * tf:.2f} ms, fwd+bwd {1e3 * tfb:.2f} ms, |A| = {stats['n_alpha']}")
    return out, (s, dets, coefs, E0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="c5", choices=["c1", "c2", "c3", "c5"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--small-steps", type=int, default=5,
                    help="timed forward steps of the n_orb 64 workload (0: skip it and the legs below)")
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

    import torch
    from paper_1902_08154_amd.api import Context

    dev = torch.device("cuda", 0)
    ctx = Context(0)
    s, dets, coefs, E0 = load_workload(ctx, dev, int(args.workload[1:]))
    ns, nint = s.n_states, s.n_int
    w = Sweep(ctx, dev, s, dets, coefs, E0)

    ctx.qp_set_timing(True)
    for i in range(args.warmup):
        w.forward()
        w.backward()
        torch.cuda.synchronize()
        log(f"warmup {i} done")
    tf_list, tb_list, wall_f = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ta = time.perf_counter()
        w.forward()
        tf_list.append(ctx.qp_last_timing())   # waits for the forward's last event
        wall_f.append(time.perf_counter() - ta)
        log(f"step {i}: forward {wall_f[-1]:.2f} s")
        w.backward()
        tb_list.append(ctx.qp_last_timing())
        log(f"step {i}: adjoint {tb_list[-1][2] / 1e3:.2f} s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stats = w.stats()
    ms_per_step = 1e3 * elapsed / args.steps
    value = stats["n_alpha"] * args.steps / elapsed

    # the dominant kernel: the clean-cell kernel of the adjoint, timed with HIP
    # events on the library's stream, on which it is launched
    kb = float(np.mean([t[4] for t in tb_list])) * 1e-3
    kf = float(np.mean([t[4] for t in tf_list])) * 1e-3
    alpha_clean = stats["n_alpha_clean"]
    ops_b = alpha_clean * clean_ops_per_alpha(ns, True)
    ops_f = alpha_clean * clean_ops_per_alpha(ns, False)
    log(f"E_PT2 = {w.e_out.cpu().numpy()}  |A| = {stats['n_alpha']} (clean {alpha_clean}, general kernel "
        f"{stats['n_alpha_general']})  step {ms_per_step / 1e3:.2f} s  clean-cell kernel: forward "
        f"{kf:.2f} s, adjoint {kb:.2f} s")

    def kms(tl):
        return {"dense": float(np.mean([t[0] for t in tl])), "general": float(np.mean([t[1] for t in tl])),
                "clean_cell": float(np.mean([t[4] for t in tl])),
                "split_correction": float(np.mean([t[3] - t[4] for t in tl])),
                "call": float(np.mean([t[2] for t in tl]))}

    extra = {
        "forward_ms": 1e3 * float(np.mean(wall_f)), "forward_alpha_per_s": stats["n_alpha"] / float(np.mean(wall_f)),
        "forward_kernel_ms": kms(tf_list), "adjoint_kernel_ms": kms(tb_list),
        "alpha_clean": alpha_clean, "alpha_general_kernel": stats["n_alpha_general"],
        # the adjoint hands the dense kernel's integral-plane batches (NS > 1 or
        # more than two words per spin) to the general kernel
        "adjoint_alpha_general_kernel": w.stats(adjoint=True)["n_alpha_general"],
        "adjoint_general_fraction": w.stats(adjoint=True)["n_alpha_general"] / max(stats["n_alpha"], 1),
        "clean_cell_forward_roofline": ({"achieved": ops_f / kf / 1e12, "frac": ops_f / kf / ALU_PEAK_OPS,
                                         "kernel_ms": 1e3 * kf, "ops_per_alpha": clean_ops_per_alpha(ns, False)}
                                        if alpha_clean > 0 else None),
        "filter": filter_figures(s, stats),
        "e_pt2": w.e_out.cpu().tolist(), "rpt2_Z": stats["Z"], "e_rpt2": stats["e_rpt2"],
        "n_selected": int(w.nsl.item()), "n_candidates": stats["n_candidates"],
        "dE_dE0": w.gE.cpu().tolist(),
    }

    # the issue rate the device reaches on one-instruction chains, beside the
    # derived ceiling the roofline uses (the clean-cell ops are FP64: the
    # FP64 FMA rate is the probed ceiling they are set against)
    from paper_1902_08154_amd import _lib
    probe = {name: ctx.qp_alu_probe(kind, 1 << 14) / 1e12
             for name, kind in (("f64_fma", _lib.QP_PROBE_F64_FMA), ("i32_add", _lib.QP_PROBE_I32_ADD),
                                ("mixed", _lib.QP_PROBE_MIXED))}
    extra["alu_probe_tops"] = probe
    log(f"ALU probe (T lane-ops/s): {probe}")

    cpu = None
    if not args.no_cpu_baseline:
        # the oracle's OpenMP team: OMP_NUM_THREADS if set, else every CPU of the
        # affinity mask; one generator per thread, each bounded to its first
        # 10^6 excitations (about 15 s), since a whole generator of this
        # workload takes the oracle several minutes
        threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
        cap = 1000000 if s.n_orb >= 128 else 0
        cpu = cpu_baseline(s, E0.cpu().numpy(), threads if cap else 12 * threads, visit_cap=cap)
        log(f"cpu baseline: {cpu}")
        # the same oracle on one core: one generator's first 5x10^5 excitations
        # (a whole-sweep-shaped sample takes the same time per alpha)
        extra["cpu_baseline_1core"] = cpu_baseline(s, E0.cpu().numpy(), 1, visit_cap=cap // 2 if cap else 0,
                                                   threads=1)
        log(f"cpu baseline, 1 core: {extra['cpu_baseline_1core']}")

    config = {"workload": s.name, "n_orb": s.n_orb, "n_up": s.n_up, "n_dn": s.n_dn, "n_det": s.n_det,
              "n_states": ns, "n_select": s.n_select, "seed": s.seed, "n_alpha": stats["n_alpha"],
              "n_cells": stats["n_cells"], "step": "forward with top-N selection, then adjoint"}
    del w, dets, coefs, E0
    torch.cuda.empty_cache()

    if args.small_steps > 0 and s.name != "c2_n64_10a10b_1e4det_top1000":
        extra["small"], c2 = small_leg(ctx, dev, args.small_steps, 2)
        if args.batched_steps > 0:
            extra["batched"] = batched_bench(ctx, dev, args.batched_steps)
        if args.next_steps > 0:
            extra["next"] = next_rows_bench(ctx, dev, *c2, args.next_steps)

    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calibration} MiB read + {args.copy_calibration} MiB written")
        del src, dst

    split = alpha_clean > 0
    mt = MEASURED_TRAFFIC.get(s.name)
    traffic = (mt["bytes"] if mt and mt["sources_sha256"] == clean_sources_sha256(
        CLEAN_SOURCES if split else DENSE_SOURCES) else None)
    if split:
        roof = {"kernel": "qplean::lean_kernel (adjoint)", "kernel_ms": 1e3 * kb, "ops_per_launch": ops_b,
                "alpha_per_launch": alpha_clean, "ops_per_alpha": clean_ops_per_alpha(ns, True)}
    else:
        # an unsplit sweep: the forward dense kernel, 3 + 15 per state per alpha
        # and 12 per word + 2 per state per connection
        kd = float(np.mean([t[0] for t in tf_list])) * 1e-3
        a_dense = stats["n_alpha"] - stats["n_alpha_general"]
        ops_d = a_dense * (3.0 + 15.0 * ns) + stats["n_connections"] * (12.0 * nint + 2.0 * ns)
        roof = {"kernel": "qpfast::fast_kernel (forward)", "kernel_ms": 1e3 * kd, "ops_per_launch": ops_d,
                "alpha_per_launch": a_dense, "ops_per_alpha": ops_d / max(a_dense, 1)}
    achieved = roof["ops_per_launch"] / (roof["kernel_ms"] * 1e-3) / 1e12

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
        "config": config,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_OPS / 1e12,
                     "unit": "Tops/s", "frac": achieved * 1e12 / ALU_PEAK_OPS, "traffic": traffic,
                     "peak_probed": probe["f64_fma"], "frac_of_probed": achieved / probe["f64_fma"], **roof},
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
