"""ctypes wrapper around the plain C FP64 oracle (``qp_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``.  The product library never
imports, links or calls anything here.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qp_oracle.c")
_LIB = os.path.join(_HERE, "libqp_oracle.so")

_CFLAGS = ["-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-std=c11"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no -march: identical FP results on any x86-64)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *_CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_D = ctypes.c_double


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        lib.orc_matrix_element.restype = _D
        lib.orc_matrix_element.argtypes = [_I, _I, _P, _P, _P, _P]
        lib.orc_det_fingerprint.restype = ctypes.c_uint64
        lib.orc_det_fingerprint.argtypes = [_P, _I]
        lib.orc_generator_rank.restype = _I
        lib.orc_generator_rank.argtypes = [_P, _P, _I64, _I, _I, _P]
        lib.orc_energy.restype = _I
        lib.orc_energy.argtypes = [_I, _I, _P, _P, _P, _P, _I64, _I, _P]
        lib.orc_pt2_full.restype = _I
        lib.orc_pt2_full.argtypes = [_I, _I, _P, _P, _P, _P, _I64, _I, _P, _I, _I,
                                     _P, _P, _P, _P, _P, _P, _P,
                                     _I64, _P, _P, _P, _P,
                                     _I64, _P, _P, _P, _P, _P,
                                     _P, _P, _P, _P,
                                     _P, _P, _P, _P, _P]
        lib.orc_alpha_eval.restype = _I
        lib.orc_alpha_eval.argtypes = [_I, _I, _P, _P, _P, _P, _I64, _I, _P, _P, _P, _P, _P, _P]
        lib.orc_hamiltonian.restype = _I
        lib.orc_hamiltonian.argtypes = [_I, _I, _P, _P, _P, _I64, _P]
        lib.orc_s2_matrix.restype = _I
        lib.orc_s2_matrix.argtypes = [_I, _I, _P, _I64, _P]
        lib.orc_eps_generators.restype = _I
        lib.orc_eps_generators.argtypes = [_I, _I, _P, _P, _P, _P, _I64, _I, _P, _P, _I64,
                                           _P, _P, _P, _P, _D, _I64, _P, _P, _P, _P, _I64, _I64, _I]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _nint(dets):
    return dets.shape[-1]


def hamiltonian(n_orb, h, eri, dets) -> np.ndarray:
    """Dense H over the determinant list (Slater-Condon elements)."""
    dets = _c(dets, np.uint64)
    nd = dets.shape[0]
    out = np.empty((nd, nd))
    _load().orc_hamiltonian(n_orb, _nint(dets), _ptr(_c(h, np.float64)), _ptr(_c(eri, np.float64)), _ptr(dets),
                            nd, _ptr(out))
    return out


def s2_matrix(n_orb, dets) -> np.ndarray:
    """Dense S^2 over the determinant list, by operator application."""
    dets = _c(dets, np.uint64)
    nd = dets.shape[0]
    out = np.empty((nd, nd))
    _load().orc_s2_matrix(n_orb, _nint(dets), _ptr(dets), nd, _ptr(out))
    return out


def matrix_element(n_orb, h, eri, bra, ket) -> float:
    bra = _c(bra, np.uint64); ket = _c(ket, np.uint64)
    return _load().orc_matrix_element(n_orb, _nint(bra), _ptr(_c(h, np.float64)),
                                      _ptr(_c(eri, np.float64)), _ptr(bra), _ptr(ket))


def det_fingerprint(det) -> int:
    det = _c(det, np.uint64)
    return int(_load().orc_det_fingerprint(_ptr(det), _nint(det)))


def generator_rank(dets, coefs) -> np.ndarray:
    dets = _c(dets, np.uint64); coefs = _c(np.atleast_2d(coefs), np.float64)
    rank = np.empty(dets.shape[0], dtype=np.int64)
    _load().orc_generator_rank(_ptr(dets), _ptr(coefs), dets.shape[0], coefs.shape[0],
                               _nint(dets), _ptr(rank))
    return rank


def energy(n_orb, h, eri, dets, coefs) -> np.ndarray:
    """E0_k = <Psi_k|H|Psi_k>/<Psi_k|Psi_k> (O(n_det^2) pair loop, OpenMP rows)."""
    dets = _c(dets, np.uint64); coefs = _c(np.atleast_2d(coefs), np.float64)
    ns = coefs.shape[0]
    out = np.empty(ns, dtype=np.float64)
    rc = _load().orc_energy(n_orb, _nint(dets), _ptr(_c(h, np.float64)), _ptr(_c(eri, np.float64)),
                            _ptr(dets), _ptr(coefs), dets.shape[0], ns, _ptr(out))
    if rc != 0:
        raise MemoryError("oracle energy failed")
    return out


class FullResult(dict):
    __getattr__ = dict.__getitem__


def pt2_full(n_orb, h, eri, dets, coefs, E0, n_select=0, dump_all=False, grad_up=None,
             eps_gen=False, nparts=1, part=0) -> FullResult:
    """The whole definition (see qp_oracle.c).  Keys: e_pt2, S, n_alpha, fp,
    n_conn, min_abs_delta, [eps_gen], [sel_dets, sel_e, sel_key],
    [all_dets, all_e, all_N, all_D, all_owner], [dc, dE0, dh]."""
    dets = _c(dets, np.uint64); coefs = _c(np.atleast_2d(coefs), np.float64)
    E0 = _c(np.atleast_1d(E0), np.float64)
    nd, ns, nint = dets.shape[0], coefs.shape[0], _nint(dets)
    h = _c(h, np.float64); eri = _c(eri, np.float64)
    e_pt2 = np.zeros(ns); S = np.zeros(ns)
    n_alpha = np.zeros(1, np.int64); fp = np.zeros(1, np.uint64); nconn = np.zeros(1, np.int64)
    mind = np.zeros(1)
    epsg = np.zeros((ns, nd)) if eps_gen else None
    sel_dets = sel_e = sel_key = None
    n_sel = np.zeros(1, np.int64)
    if n_select > 0:
        sel_dets = np.zeros((n_select, 2, nint), np.uint64)
        sel_e = np.zeros((n_select, ns)); sel_key = np.zeros(n_select)
    all_cap = 0
    all_dets = all_e = all_N = all_D = all_owner = None
    if dump_all:
        # bound: every single/double of every det
        from math import comb
        nup = int(sum(bin(int(x)).count("1") for x in dets[0, 0]))
        ndn = int(sum(bin(int(x)).count("1") for x in dets[0, 1]))
        vu, vd = n_orb - nup, n_orb - ndn
        per = nup * vu + ndn * vd + comb(nup, 2) * comb(vu, 2) + comb(ndn, 2) * comb(vd, 2) + nup * vu * ndn * vd
        all_cap = per * nd
        all_dets = np.zeros((all_cap, 2, nint), np.uint64)
        all_e = np.zeros((all_cap, ns)); all_N = np.zeros((all_cap, ns))
        all_D = np.zeros(all_cap); all_owner = np.zeros(all_cap, np.int64)
    dc = dE0 = dh = None
    gu = None
    if grad_up is not None:
        gu = _c(np.atleast_1d(grad_up), np.float64)
        dc = np.zeros((ns, nd)); dE0 = np.zeros(ns); dh = np.zeros((n_orb, n_orb))
    abs_e = np.zeros(ns); T = np.zeros(ns)
    S_gen = np.zeros((ns, nd)) if eps_gen else None
    abs_gen = np.zeros((ns, nd)) if eps_gen else None
    sel_D = np.zeros(n_select) if n_select > 0 else None
    rc = _load().orc_pt2_full(n_orb, nint, _ptr(h), _ptr(eri), _ptr(dets), _ptr(coefs), nd, ns,
                              _ptr(E0), nparts, part,
                              _ptr(e_pt2), _ptr(S), _ptr(n_alpha), _ptr(fp), _ptr(nconn), _ptr(mind),
                              _ptr(epsg), n_select, _ptr(sel_dets), _ptr(sel_e), _ptr(sel_key),
                              _ptr(n_sel), all_cap, _ptr(all_dets), _ptr(all_e), _ptr(all_N),
                              _ptr(all_D), _ptr(all_owner), _ptr(gu), _ptr(dc), _ptr(dE0), _ptr(dh),
                              _ptr(abs_e), _ptr(T), _ptr(S_gen), _ptr(abs_gen), _ptr(sel_D))
    if rc != 0:
        raise MemoryError("oracle pt2_full failed")
    r = FullResult(e_pt2=e_pt2, S=S, n_alpha=int(n_alpha[0]), fp=int(fp[0]), n_conn=int(nconn[0]),
                   min_abs_delta=float(mind[0]), abs_e=abs_e, T=T, E0=E0)
    if eps_gen:
        r.update(eps_gen=epsg, S_gen=S_gen, abs_gen=abs_gen)
    if n_select > 0:
        m = int(n_sel[0])
        r.update(sel_dets=sel_dets[:m], sel_e=sel_e[:m], sel_key=sel_key[:m], sel_D=sel_D[:m])
    if dump_all:
        m = r["n_alpha"]
        r.update(all_dets=all_dets[:m], all_e=all_e[:m], all_N=all_N[:m], all_D=all_D[:m],
                 all_owner=all_owner[:m])
    if grad_up is not None:
        r.update(dc=dc, dE0=dE0, dh=dh)
    return r


def rpt2(E0, e_pt2, S):
    """Renormalised PT2 (sec. "Renormalized PT2", eq. Z): the self-energy
    Sigma[E] = sum_alpha <alpha|H|Psi>^2 / (E - H_aa) is linearised about E0,
    where Sigma[E0] = E_PT2 and dSigma/dE = -S; solving E = E0 + Sigma[E] then
    gives E = E0 + Z E_PT2 with Z = 1 / (1 - dSigma/dE) = 1 / (1 + S).
    Per state k.  Returns (Z, E0 + Z E_PT2)."""
    E0 = np.atleast_1d(np.asarray(E0, dtype=np.float64))
    e = np.atleast_1d(np.asarray(e_pt2, dtype=np.float64))
    S = np.atleast_1d(np.asarray(S, dtype=np.float64))
    Z = 1.0 / (1.0 + S)
    return Z, E0 + Z * e


def semistochastic(eps_of_ranks, w, uniforms, rel_err, det_chunk, draws_per_round):
    """Semi-stochastic E_PT2 (sec. "CIPSI selection and PT2 energy", the hybrid
    deterministic/stochastic scheme), written from the paper's description.

    Generators are taken in generator order (rank r).  E_PT2 = sum_I eps_I is
    split into a deterministic part D, the first d ranks, and a stochastic part
    S, the rest.  Each round, D grows by det_chunk ranks and draws_per_round
    ranks are drawn with probability w_r / W (w_r = sum_k c_rk^2); a drawn
    rank's eps is computed once and remembered.  A draw is the first rank r
    whose running weight sum exceeds u W, for the next number u of
    `uniforms`.  The draws that fall in S are a sample of S with probability
    w_r / W_S (W_S the weight of S), so sum_S eps is estimated by the mean of
    W_S eps_r / w_r over them, with the standard error of that mean.  The
    run stops when every state's error is at most rel_err |estimate|, when D
    covers every rank (exact), or when the uniforms run out.

    eps_of_ranks(list of ranks) -> array [len][ns] gives eps for ranks.
    Returns (estimate[ns], error[ns], number of ranks evaluated, rounds)."""
    w = np.asarray(w, dtype=np.float64)
    n = w.size
    cum = np.empty(n)
    run = 0.0
    for r in range(n):
        run += w[r]
        cum[r] = run
    tail = np.zeros(n + 1)
    for r in range(n - 1, -1, -1):
        tail[r] = tail[r + 1] + w[r]
    W = run
    memo = {}
    draws = []
    d = 0
    nu = 0
    rounds = 0
    ns = None
    det_sum = None
    est = err = None
    while True:
        d_new = min(n, d + det_chunk)
        todo = [r for r in range(d, d_new) if r not in memo]
        drawn = 0
        while drawn < draws_per_round and nu < len(uniforms) and W > 0.0:
            t = uniforms[nu] * W
            nu += 1
            r = min(int(np.searchsorted(cum, t, side="right")), n - 1)
            draws.append(r)
            drawn += 1
            if r >= d_new and r not in memo and r not in todo:
                todo.append(r)
        if todo:
            vals = np.atleast_2d(np.asarray(eps_of_ranks(todo), dtype=np.float64))
            for r, v in zip(todo, vals):
                memo[r] = v
        if ns is None:
            ns = len(next(iter(memo.values()))) if memo else 1
            det_sum = np.zeros(ns)
        for r in range(d, d_new):
            det_sum = det_sum + memo[r]
        d = d_new
        rounds += 1
        est = np.zeros(ns)
        err = np.zeros(ns)
        converged = True
        if d == n:
            est = det_sum.copy()
        else:
            WS = tail[d]
            inS = [r for r in draws if r >= d]
            for k in range(ns):
                mean = 0.0
                m2 = 0.0
                for j, r in enumerate(inS, start=1):
                    y = WS * memo[r][k] / w[r]
                    dl = y - mean
                    mean += dl / j
                    m2 += dl * (y - mean)
                m = len(inS)
                est[k] = det_sum[k] + (mean if m > 0 else 0.0)
                err[k] = np.sqrt(m2 / (m - 1) / m) if m > 1 else np.inf
                if not (m > 1 and err[k] <= rel_err * abs(est[k])):
                    converged = False
        if d == n or converged:
            break
        if draws_per_round > 0 and nu >= len(uniforms):
            break
    return est, err, len(memo), rounds


def alpha_eval(n_orb, h, eri, dets, coefs, rank, alpha):
    """(N[ns], D, owner_rank, internal) for one determinant alpha, scanning all of Psi."""
    dets = _c(dets, np.uint64); coefs = _c(np.atleast_2d(coefs), np.float64)
    alpha = _c(alpha, np.uint64); rank = _c(rank, np.int64)
    ns = coefs.shape[0]
    N = np.zeros(ns); D = np.zeros(1); own = np.zeros(1, np.int64); internal = np.zeros(1, np.int32)
    _load().orc_alpha_eval(n_orb, _nint(dets), _ptr(_c(h, np.float64)), _ptr(_c(eri, np.float64)),
                           _ptr(dets), _ptr(coefs), dets.shape[0], ns, _ptr(rank), _ptr(alpha),
                           _ptr(N), _ptr(D), _ptr(own), _ptr(internal))
    return N, float(D[0]), int(own[0]), bool(internal[0])


def eps_generators(n_orb, h, eri, dets, coefs, E0, gens, dump_thr=None, dump_cap=0, visit_cap=0, threads=0,
                   visit_start=0):
    """Per-generator eps_I [n_gen][ns], S, |A_I|, fingerprint sums, and optional
    dumps of owned alpha with |e~| >= dump_thr.  visit_start and visit_cap > 0
    restrict each generator to its excitations [visit_start, visit_start +
    visit_cap) in enumeration order (a timing sample, or one slice of a
    generator whose slices the caller sums); threads > 0 sets the OpenMP
    team's size."""
    dets = _c(dets, np.uint64); coefs = _c(np.atleast_2d(coefs), np.float64)
    E0 = _c(np.atleast_1d(E0), np.float64)
    gens = _c(np.atleast_1d(gens), np.int64)
    ng, ns, nint = gens.size, coefs.shape[0], _nint(dets)
    eps = np.zeros((ng, ns)); S = np.zeros((ng, ns))
    count = np.zeros(ng, np.int64); fp = np.zeros(ng, np.uint64)
    dd = de = dk = dn = None
    if dump_cap > 0:
        dd = np.zeros((ng, dump_cap, 2, nint), np.uint64)
        de = np.zeros((ng, dump_cap, ns)); dk = np.zeros((ng, dump_cap)); dn = np.zeros(ng, np.int64)
    rc = _load().orc_eps_generators(n_orb, nint, _ptr(_c(h, np.float64)), _ptr(_c(eri, np.float64)),
                                    _ptr(dets), _ptr(coefs), dets.shape[0], ns, _ptr(E0),
                                    _ptr(gens), ng, _ptr(eps), _ptr(S), _ptr(count), _ptr(fp),
                                    float(dump_thr if dump_thr is not None else np.inf), dump_cap,
                                    _ptr(dd), _ptr(de), _ptr(dk), _ptr(dn), int(visit_start), int(visit_cap),
                                    int(threads))
    if rc != 0:
        raise MemoryError("oracle eps_generators failed")
    out = FullResult(eps=eps, S=S, count=count, fp=fp)
    if dump_cap > 0:
        out.update(dump_dets=dd, dump_e=de, dump_key=dk, dump_n=dn)
    return out
