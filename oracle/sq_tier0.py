"""Tier-0 brute force by second quantisation, for tiny orbital spaces.

TEST INFRASTRUCTURE ONLY.  Independent of the C oracle: it never evaluates a
Slater-Condon rule.  The Hamiltonian (sec. "Matrix elements of the
Hamiltonian": one-electron integrals (p|h|q) and chemist ERIs (pq|rs), real
orbitals) is applied term by term,

    H = sum_{pq,s} h_pq a+_{ps} a_{qs}
        + 1/2 sum_{pqrs} sum_{s,s'} (pq|rs) a+_{ps} a+_{rs'} a_{s's'} a_{qs},

to canonically ordered determinants (up spin-orbitals before down ones,
increasing index inside each spin -- sec. "Internal representation of
determinants"); each operator contributes (-1)^(number of occupied
spin-orbitals before it).

A determinant is a Python int over 2n spin-orbital bits: bit p = (p, up),
bit n+p = (p, down).
"""
from __future__ import annotations

import itertools
from typing import Dict, Iterable, List

import numpy as np


def eri_from_packed(eri_packed: np.ndarray, n: int) -> np.ndarray:
    """Dense (pq|rs) from the packed layout.  Written with its own index formula
    (max*(max+1)/2 + min, applied to orbital pairs, then to pair indices)."""
    def tri(a, b):
        hi, lo = max(a, b), min(a, b)
        return hi * (hi + 1) // 2 + lo
    g = np.empty((n, n, n, n))
    for p, q, r, s in itertools.product(range(n), repeat=4):
        g[p, q, r, s] = eri_packed[tri(tri(p, q), tri(r, s))]
    return g


class PackedERI:
    """Lazy (pq|rs) accessor over the packed array (same index formula as
    eri_from_packed), for orbital spaces too large for a dense n^4 array."""

    def __init__(self, eri_packed: np.ndarray):
        self.eri = eri_packed

    def __getitem__(self, idx):
        p, q, r, s = (int(x) for x in idx)

        def tri(a, b):
            hi, lo = max(a, b), min(a, b)
            return hi * (hi + 1) // 2 + lo
        return float(self.eri[tri(tri(p, q), tri(r, s))])


def _annihilate(det: int, so: int):
    if not (det >> so) & 1:
        return 0, 0
    sign = -1 if bin(det & ((1 << so) - 1)).count("1") & 1 else 1
    return sign, det & ~(1 << so)


def _create(det: int, so: int):
    if (det >> so) & 1:
        return 0, 0
    sign = -1 if bin(det & ((1 << so) - 1)).count("1") & 1 else 1
    return sign, det | (1 << so)


def apply_hamiltonian(n: int, h: np.ndarray, g: np.ndarray, det: int) -> Dict[int, float]:
    """H|det> as {det': coefficient}; g is the dense (pq|rs) array."""
    out: Dict[int, float] = {}
    occ = [so for so in range(2 * n) if (det >> so) & 1]
    # one-electron part
    for qso in occ:
        s1, d1 = _annihilate(det, qso)
        spin, q = divmod(qso, n)
        for p in range(n):
            s2, d2 = _create(d1, spin * n + p)
            if s2 == 0:
                continue
            out[d2] = out.get(d2, 0.0) + s1 * s2 * h[p, q]
    # two-electron part: a+_p(s) a+_r(s') a_s(s') a_q(s); annihilate q first
    for qso in occ:
        sq_, d1 = _annihilate(det, qso)
        spin_q, q = divmod(qso, n)
        for sso in occ:
            if sso == qso:
                continue
            ss_, d2 = _annihilate(d1, sso)
            spin_s, s = divmod(sso, n)
            for r in range(n):
                sr_, d3 = _create(d2, spin_s * n + r)
                if sr_ == 0:
                    continue
                for p in range(n):
                    sp_, d4 = _create(d3, spin_q * n + p)
                    if sp_ == 0:
                        continue
                    v = 0.5 * g[p, q, r, s] * sq_ * ss_ * sr_ * sp_
                    out[d4] = out.get(d4, 0.0) + v
    return out


def diagonal_element(n: int, h: np.ndarray, g: np.ndarray, det: int) -> float:
    """<det|H|det> by second quantisation, keeping only operator strings that
    return det itself (the others cannot contribute to this coefficient)."""
    val = 0.0
    occ = [so for so in range(2 * n) if (det >> so) & 1]
    for qso in occ:
        val += h[qso % n, qso % n]
    for qso in occ:
        sq_, d1 = _annihilate(det, qso)
        for sso in occ:
            if sso == qso:
                continue
            ss_, d2 = _annihilate(d1, sso)
            # a+_p a+_r must recreate {qso, sso}: (r=s, p=q) or (r=q, p=s) when spins allow
            for (pso, rso) in ((qso, sso), (sso, qso)):
                if pso // n != qso // n or rso // n != sso // n:
                    continue
                sr_, d3 = _create(d2, rso)
                sp_, d4 = _create(d3, pso)
                if sr_ == 0 or sp_ == 0 or d4 != det:
                    continue
                val += 0.5 * g[pso % n, qso % n, rso % n, sso % n] * sq_ * ss_ * sr_ * sp_
    return val


def fci_space(n: int, nup: int, ndn: int) -> List[int]:
    dets = []
    for up in itertools.combinations(range(n), nup):
        for dn in itertools.combinations(range(n), ndn):
            m = 0
            for p in up:
                m |= 1 << p
            for p in dn:
                m |= 1 << (n + p)
            dets.append(m)
    return dets


def dense_hamiltonian(n: int, h: np.ndarray, g: np.ndarray, basis: List[int]) -> np.ndarray:
    index = {d: i for i, d in enumerate(basis)}
    H = np.zeros((len(basis), len(basis)))
    for j, d in enumerate(basis):
        for d2, v in apply_hamiltonian(n, h, g, d).items():
            H[index[d2], j] += v
    return H


def to_words(det: int, n: int) -> np.ndarray:
    """int spin-orbital mask -> uint64[2][n_int] boundary layout."""
    nint = (n - 1) // 64 + 1
    out = np.zeros((2, nint), dtype=np.uint64)
    up, dn = det & ((1 << n) - 1), det >> n
    for s, m in enumerate((up, dn)):
        for w in range(nint):
            out[s, w] = np.uint64((m >> (64 * w)) & 0xFFFFFFFFFFFFFFFF)
    return out


def from_words(words: np.ndarray, n: int) -> int:
    words = np.asarray(words, dtype=np.uint64).reshape(2, -1)
    up = sum(int(x) << (64 * w) for w, x in enumerate(words[0]))
    dn = sum(int(x) << (64 * w) for w, x in enumerate(words[1]))
    return up | (dn << n)


def degree(a: int, b: int) -> int:
    return bin(a ^ b).count("1") // 2


def pt2_bruteforce(n: int, h: np.ndarray, g: np.ndarray, psi: List[int], coefs: np.ndarray,
                   E0: Iterable[float]):
    """Brute-force E_PT2 over the external set: H applied to every internal det
    gives the exact columns H[:, Psi]; alpha runs over the determinants those
    columns reach (plus structurally connected ones with a zero element).
    Returns (E_PT2[ns], {alpha: (N[ns], H_aa)})."""
    coefs = np.atleast_2d(coefs)
    ns = coefs.shape[0]
    E0 = np.atleast_1d(np.asarray(E0, dtype=float))
    inpsi = set(psi)
    num: Dict[int, np.ndarray] = {}
    for j, d in enumerate(psi):
        for a, v in apply_hamiltonian(n, h, g, d).items():
            if a in inpsi:
                continue
            num.setdefault(a, np.zeros(ns))
            num[a] += coefs[:, j] * v
    # every structurally connected alpha is a key above (zero-valued terms are
    # accumulated too), so the keys are exactly A
    out = {}
    e = np.zeros(ns)
    for a in sorted(num):
        if not any(1 <= degree(a, d) <= 2 for d in psi):
            continue
        haa = diagonal_element(n, h, g, a)
        out[a] = (num[a], haa)
        e += num[a] ** 2 / (E0 - haa)
    return e, out
