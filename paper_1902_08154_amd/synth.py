"""Seeded synthetic inputs for the Epstein-Nesbet PT2 / CIPSI-selection sweep.

This module only *draws* inputs: one-electron integrals, packed two-electron
integrals, determinant lists and coefficient vectors.  It contains none of the
method's arithmetic (no Slater-Condon element, no energy, no excitation degree
beyond picking random holes and particles).  Both the CPU oracle (test side)
and the HIP library (product side) consume what it returns.

Bit-for-bit reproducibility across machines is a design goal, because stored
expected values are keyed to these inputs:

* normal deviates come from ``numpy.random.default_rng(seed)`` (scalar C code);
* exponential decays use hard-coded IEEE constants raised to integer powers by
  repeated multiplication (no libm / SIMD ``exp``);
* Cholesky factors are rounded to multiples of 2^-20, so every product and
  partial sum in the GEMM that forms (pq|rs) is exact and the result does not
  depend on the BLAS kernel or its summation order;
* norms and dot products use ``math.fsum`` (correctly rounded).

Conventions (the boundary's layout, see the C header):

* a determinant is ``uint64[2][n_int]`` -- spin-up string then spin-down string;
  bit ``b`` of word ``w`` is spatial orbital ``64*w + b`` (0-based);
* ``n_int = (n_orb - 1) // 64 + 1``;
* two-electron integrals are chemist-notation (pq|rs), real, 8-fold symmetric,
  packed at ``tri(tri(p,q), tri(r,s))`` with ``tri(a,b) = M(M+1)/2 + m``,
  ``M = max(a,b)``, ``m = min(a,b)``.  With 1-based indices this is the
  integral "hash" of the paper's Algorithm 1 minus one (a bijection onto
  ``[0, P(P+1)/2)``, ``P = n(n+1)/2``).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

# exp(-1/3), exp(-1/10), exp(-1/2000) as exact IEEE doubles.
_DECAY_3 = float.fromhex("0x1.6edd3122f2ea5p-1")
_DECAY_10 = float.fromhex("0x1.cf46d99d52b3ap-1")
_DECAY_2000 = float.fromhex("0x1.ffbe7afa4452ep-1")

_CHOL_GRID = 2.0 ** 20


def n_int_for(n_orb: int) -> int:
    return (n_orb - 1) // 64 + 1


def _powers(base: float, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.float64)
    v = 1.0
    for i in range(count):
        out[i] = v
        v = v * base
    return out


def _sym_decay(rng: np.random.Generator, n: int, decay: np.ndarray) -> np.ndarray:
    """Symmetric n x n matrix, entries N(0,1) * decay[|p-q|] (upper triangle drawn)."""
    z = rng.standard_normal((n, n))
    dist = np.abs(np.subtract.outer(np.arange(n), np.arange(n)))
    m = z * decay[dist]
    iu = np.triu_indices(n, 1)
    m[(iu[1], iu[0])] = m[iu]
    return m


def pair_index(n: int):
    """(p, q) arrays with p >= q, ordered by tri(p, q) = p(p+1)/2 + q."""
    p, q = np.tril_indices(n)
    return p, q


def make_integrals(rng: np.random.Generator, n_orb: int, n_chol: int):
    """One-electron h and packed 8-fold-symmetric ERIs from seeded Cholesky factors.

    h_pq = h_qp ~ N(0,1) exp(-|p-q|/3), then h_pp += p.
    L^k_pq = L^k_qp ~ N(0,1) exp(-|p-q|/3) / sqrt(n_chol), rounded to 2^-20.
    (pq|rs) = sum_k L^k_pq L^k_rs  (positive semidefinite, 8-fold symmetric).
    """
    n = n_orb
    decay = _powers(_DECAY_3, n)
    h = _sym_decay(rng, n, decay)
    h[np.arange(n), np.arange(n)] += np.arange(n, dtype=np.float64)

    scale = 1.0 / math.sqrt(n_chol)
    pp, qq = pair_index(n)
    npair = pp.size
    lp = np.empty((n_chol, npair), dtype=np.float64)
    for k in range(n_chol):
        lk = _sym_decay(rng, n, decay) * scale
        lk = np.rint(lk * _CHOL_GRID) / _CHOL_GRID
        lp[k] = lk[pp, qq]

    eri = np.empty(npair * (npair + 1) // 2, dtype=np.float64)
    # Row blocks of the lower triangle of Lp^T Lp; every product and partial sum
    # is a multiple of 2^-40 well below 2^12, hence exact in any order.
    block = max(1, min(npair, (1 << 24) // max(npair, 1)))
    for a in range(0, npair, block):
        b = min(npair, a + block)
        v = lp[:, a:b].T @ lp[:, :b]
        for t in range(a, b):
            base = t * (t + 1) // 2
            eri[base:base + t + 1] = v[t - a, :t + 1]
    return h, eri


# --------------------------------------------------------------------------
# determinants
# --------------------------------------------------------------------------

def det_from_orbitals(n_orb: int, up, dn) -> np.ndarray:
    nint = n_int_for(n_orb)
    d = np.zeros((2, nint), dtype=np.uint64)
    for s, occ in enumerate((up, dn)):
        for o in occ:
            d[s, o // 64] |= np.uint64(1) << np.uint64(o % 64)
    return d


def hf_det(n_orb: int, n_up: int, n_dn: int) -> np.ndarray:
    return det_from_orbitals(n_orb, range(n_up), range(n_dn))


def _occ_lists(det_tuple, n_orb, nint):
    occ = ([], [])
    for s in range(2):
        for w in range(nint):
            x = det_tuple[s * nint + w]
            while x:
                low = x & -x
                occ[s].append(64 * w + low.bit_length() - 1)
                x ^= low
    return occ


def _excitation_count(n_orb, nup, ndn):
    vu, vd = n_orb - nup, n_orb - ndn
    return (nup * vu, ndn * vd, math.comb(nup, 2) * math.comb(vu, 2),
            math.comb(ndn, 2) * math.comb(vd, 2), nup * vu * ndn * vd)


def _unrank_pair(idx, m):
    """idx-th pair (i<j) of range(m) in lexicographic order."""
    i = 0
    while idx >= m - 1 - i:
        idx -= m - 1 - i
        i += 1
    return i, i + 1 + idx


def _apply_excitation(det_tuple, n_orb, nint, index):
    """Apply the index-th single/double excitation (uniform enumeration) to a det.

    Enumeration order: up singles, down singles, up-up doubles, down-down
    doubles, up-down doubles.  Works on Python ints (one per 64-bit word).
    """
    occ = _occ_lists(det_tuple, n_orb, nint)
    virt = tuple(sorted(set(range(n_orb)) - set(o)) for o in occ)
    counts = _excitation_count(n_orb, len(occ[0]), len(occ[1]))
    words = list(det_tuple)

    def flip(spin, orb):
        words[spin * nint + orb // 64] ^= 1 << (orb % 64)

    cat = 0
    while index >= counts[cat]:
        index -= counts[cat]
        cat += 1
    if cat in (0, 1):
        s = cat
        nv = len(virt[s])
        h, p = occ[s][index // nv], virt[s][index % nv]
        flip(s, h)
        flip(s, p)
    elif cat in (2, 3):
        s = cat - 2
        nvp = math.comb(len(virt[s]), 2)
        hi, pi = index // nvp, index % nvp
        h1, h2 = _unrank_pair(hi, len(occ[s]))
        p1, p2 = _unrank_pair(pi, len(virt[s]))
        for o in (occ[s][h1], occ[s][h2], virt[s][p1], virt[s][p2]):
            flip(s, o)
    else:
        nu = len(occ[0]) * len(virt[0])
        iu, idn = index // (len(occ[1]) * len(virt[1])), index % (len(occ[1]) * len(virt[1]))
        del nu
        nvu, nvd = len(virt[0]), len(virt[1])
        flip(0, occ[0][iu // nvu])
        flip(0, virt[0][iu % nvu])
        flip(1, occ[1][idn // nvd])
        flip(1, virt[1][idn % nvd])
    return tuple(words)


def _to_tuple(det: np.ndarray):
    return tuple(int(x) for x in det.reshape(-1))


def _from_tuples(tuples, nint):
    arr = np.array(tuples, dtype=np.uint64)
    return arr.reshape(len(tuples), 2, nint)


def excitations_of_hf_sample(rng, n_orb, nup, ndn, count):
    """HF plus `count` distinct random singles/doubles of HF (uniform, no replacement)."""
    nint = n_int_for(n_orb)
    hf = _to_tuple(hf_det(n_orb, nup, ndn))
    total = sum(_excitation_count(n_orb, nup, ndn))
    picks = rng.choice(total, size=count, replace=False)
    dets = [hf] + [_apply_excitation(hf, n_orb, nint, int(i)) for i in picks]
    return _from_tuples(dets, nint)


def grow_wavefunction(rng, n_orb, nup, ndn, n_det):
    """Grow a determinant set from HF: pick an existing det uniformly, apply a
    uniformly random single/double, insert it if new; repeat until n_det.
    Returns dets in insertion order (rank r = insertion index)."""
    nint = n_int_for(n_orb)
    hf = _to_tuple(hf_det(n_orb, nup, ndn))
    total = sum(_excitation_count(n_orb, nup, ndn))
    dets = [hf]
    seen = {hf}
    while len(dets) < n_det:
        src = dets[int(rng.integers(len(dets)))]
        new = _apply_excitation(src, n_orb, nint, int(rng.integers(total)))
        if new not in seen:
            seen.add(new)
            dets.append(new)
    return _from_tuples(dets, nint)


# --------------------------------------------------------------------------
# coefficients
# --------------------------------------------------------------------------

def _normalise(v: np.ndarray) -> np.ndarray:
    nrm = math.sqrt(math.fsum(float(x) * float(x) for x in v))
    return v / nrm


def _dot(a: np.ndarray, b: np.ndarray) -> float:
    return math.fsum((a * b).tolist())


def decaying_coefficients(rng, n_det, n_states, tau_pow=_DECAY_2000):
    """c_r = s_r * exp(-r/2000) (r = insertion rank), s_0 = +1 for state 0, other
    signs random; states >= 1 draw independent signs.  Gram-Schmidt
    orthonormalised (state 0 stays HF-dominated)."""
    mag = _powers(tau_pow, n_det)
    out = np.empty((n_states, n_det), dtype=np.float64)
    for k in range(n_states):
        s = rng.choice(np.array([-1.0, 1.0]), size=n_det)
        if k == 0:
            s[0] = 1.0
        v = s * mag
        for j in range(k):
            v = v - _dot(v, out[j]) * out[j]
        out[k] = _normalise(v)
    return out


def hf_dominated_coefficients(rng, n_det):
    """c_0 = 0.95, c_i = 0.1 N(0,1) exp(-i/10); normalised (one state)."""
    mag = _powers(_DECAY_10, n_det)
    v = 0.1 * rng.standard_normal(n_det) * mag
    v[0] = 0.95
    return _normalise(v)[None, :]


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

@dataclass
class System:
    name: str
    seed: int
    n_orb: int
    n_up: int
    n_dn: int
    h: np.ndarray
    eri: np.ndarray
    dets: np.ndarray          # uint64 [n_det][2][n_int]
    coefs: np.ndarray         # float64 [n_states][n_det]
    n_select: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n_int(self) -> int:
        return n_int_for(self.n_orb)

    @property
    def n_det(self) -> int:
        return self.dets.shape[0]

    @property
    def n_states(self) -> int:
        return self.coefs.shape[0]


def make_system(name, seed, n_orb, n_up, n_dn, n_det, n_states=1, n_chol=None,
                n_select=0, style="grown"):
    """Generic seeded system: Cholesky integrals (k = 2n unless given) and a grown
    determinant set with decaying coefficients ("grown"), or HF + random
    excitations of HF with an HF-dominated vector ("hf")."""
    rng = np.random.default_rng(seed)
    h, eri = make_integrals(rng, n_orb, n_chol if n_chol else 2 * n_orb)
    if style == "hf":
        dets = excitations_of_hf_sample(rng, n_orb, n_up, n_dn, n_det - 1)
        coefs = hf_dominated_coefficients(rng, n_det)
        if n_states > 1:
            raise ValueError("style 'hf' is single-state")
    else:
        dets = grow_wavefunction(rng, n_orb, n_up, n_dn, n_det)
        coefs = decaying_coefficients(rng, n_det, n_states)
    return System(name, seed, n_orb, n_up, n_dn, h, eri, dets, coefs, n_select)


# The five workloads (seed = 1000 + index).
WORKLOADS = {
    1: dict(name="c1_n12_3a3b_50det", n_orb=12, n_up=3, n_dn=3, n_det=50,
            n_states=1, n_chol=24, n_select=100, style="hf"),
    2: dict(name="c2_n64_10a10b_1e4det_top1000", n_orb=64, n_up=10, n_dn=10,
            n_det=10_000, n_states=1, n_chol=128, n_select=1000),
    3: dict(name="c3_n128_14a14b_1e5det", n_orb=128, n_up=14, n_dn=14,
            n_det=100_000, n_states=1, n_chol=256, n_select=1000),
    5: dict(name="c5_n256_16a16b_1e6det_2st_top1e5", n_orb=256, n_up=16, n_dn=16,
            n_det=1_000_000, n_states=2, n_chol=512, n_select=100_000),
}


def workload(index: int, n_det: Optional[int] = None) -> System:
    """Workload `index` (1, 2, 3 or 5); `n_det` overrides the determinant count
    (the same seed, so a prefix-grown smaller instance)."""
    spec = dict(WORKLOADS[index])
    if n_det is not None:
        spec["n_det"] = n_det
    name = spec.pop("name")
    return make_system(name, 1000 + index, **spec)


def batched_workload(n_sys: int = 64, seed: int = 1004,
                     det_range=(100, 20_000)) -> List[System]:
    """64 independent systems: n_orb in {32,48,64,96}, 4-12 electrons per spin
    (independently), n_det log-uniform in det_range, 1-3 orthonormal states."""
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(n_sys):
        n_orb = int(rng.choice([32, 48, 64, 96]))
        nup = int(rng.integers(4, 13))
        ndn = int(rng.integers(4, 13))
        lo, hi = math.log(det_range[0]), math.log(det_range[1])
        nd = int(round(math.exp(lo + (hi - lo) * float(rng.random()))))
        ns = int(rng.integers(1, 4))
        specs.append((n_orb, nup, ndn, nd, ns, int(rng.integers(1 << 31))))
    out = []
    for i, (n_orb, nup, ndn, nd, ns, sseed) in enumerate(specs):
        out.append(make_system(f"c4_sys{i}", sseed, n_orb, nup, ndn, nd,
                               n_states=ns, n_select=0))
    return out


def uniforms(seed: int, count: int) -> np.ndarray:
    """Seeded random numbers in [0, 1), e.g. the draws of a stochastic estimate."""
    return np.random.default_rng(seed).random(count)
