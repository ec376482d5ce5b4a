// qp_sweep.hip -- the per-generator EN-PT2 / selection sweep (forward and
// adjoint) for gfx950.
//
// Work decomposition (sec. "CIPSI selection and PT2 energy", appendix on the
// selection implementation): generators I in order of decreasing sum_k c_Ik^2;
// for each I the external determinants alpha = I - H + P are enumerated by
// hole set H (|H| = 1 or 2, the exact holes) and particle set P (virtual
// orbitals of I with matching spins), so each (I, alpha) pair appears once.
// A batch is one hole set; its cells are the particle sets.
//
// One workgroup is one wavefront.  A work item is (generator, q): every Q-th
// batch of the generator starting at q.  Inside a batch the cells form a
// row x column grid (opposite spins: the two virtual lists; same spin: the
// triangle p1 < p2 folded into rows of full width; singles: one row).  Lanes
// run over the contiguous column index and the loop runs over rows, so
// row-dependent quantities are wavefront-uniform and every integral read is a
// coalesced row of a per-hole-pair block.
//
// Per cell:  <I|H|alpha> = phase * block element (or a Fock element of I for
// singles); H_alpha,alpha = E(I - H) + F(p1) + F(p2) + pair(p1, p2), the
// Fock-diagonal update of the same appendix; e_k = A_k^2 / (E0_k - D).
//
// Other internal determinants J within degree 4 of I (coarse list) pass the
// fine filter m = |(I - H) \ J| <= 2 and touch only cells with
// |P \ J| <= 2 - m.  They are corrections: a J earlier in generator order
// bans the cell (alpha belongs to an earlier generator), J = alpha bans it,
// otherwise c_J <J|H|alpha> is added.  Their elements are evaluated with all
// lanes busy: m = 2 cells in a per-batch list, the column part of m = 1 in a
// per-batch column buffer (lanes over rows); the row part of m = 1 and m = 0
// entries are evaluated while their row is processed ("inline").
#include "qp_dev.h"

namespace {

constexpr int WAVE = 64;
constexpr int FCAP = 64;     // fine entries kept per batch
constexpr int L2CAP = 64;    // m = 2 cells per batch
constexpr int CSCAP = 2;     // column segments per batch
constexpr int ICAP = 16;     // inline entries per batch

struct FineE {
    int32_t j;
    uint8_t m, earlier, ner, nec;   // ner / nec: particles of E on the row / column spin
    uint32_t er;                    // row-spin virtual indices of E = J \ I, one per byte
    uint32_t ec;                    // column-spin virtual indices of E (opposite spins)
};

struct Batch {
    int type;        // BT_*
    int s1, h1, s2, h2;
    int rs, cs;      // row / column spins
    int nr, nc;      // OS: rows, columns; SS and SINGLE: V
    int sH;          // hole part of the phase
    double D0;       // energy of I - H
    const double *blk;
};

__device__ __forceinline__ double fast_rcp(double d)
{
    // reciprocal to about one ulp: hardware estimate and two Newton steps
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    return d == 0.0 ? copysign(__builtin_inf(), d) : r;
}


__device__ __forceinline__ void tri_decode(int c, int &i1, int &i2)
{
    int t = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)c)) * 0.5f);
    while (t * (t - 1) / 2 > c) --t;
    while ((t + 1) * t / 2 <= c) ++t;
    i2 = t;
    i1 = c - t * (t - 1) / 2;
}

// carve a typed array out of the dynamic LDS block: offset arithmetic only,
// so the compiler keeps the LDS address space (ds_* instead of flat_*)
template <typename T>
__device__ __forceinline__ T *carve(unsigned char *base, unsigned &off, int count)
{
    off = (off + 15u) & ~15u;
    T *r = reinterpret_cast<T *>(base + off);
    off += (unsigned)(sizeof(T) * (unsigned)count);
    return r;
}

// is x among the first nv bytes of v
__device__ __forceinline__ bool has(uint32_t v, int nv, int x)
{
    bool r = false;
#pragma unroll
    for (int t = 0; t < 4; ++t) r |= (t < nv) && ((int)((v >> (8 * t)) & 255u) == x);
    return r;
}
__device__ __forceinline__ int byte_at(uint32_t v, int t) { return (int)((v >> (8 * t)) & 255u); }

__device__ __forceinline__ double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

}  // namespace

// generic <J|H|alpha>, alpha = I with the holes removed and the particles
// added
template <int NINT, class Ints>
__device__ __forceinline__ double corr_element(const Ints &I, const uint64_t *Ibits, int h0, int h1c, int pa,
                                            int sa, int pb, int sb, const uint64_t *J, int *deg, int *sgl)
{
    uint64_t al[2 * NINT];
#pragma unroll
    for (int w = 0; w < 2 * NINT; ++w) al[w] = alpha_word<NINT>(Ibits, w, h0, h1c, pa, sa, pb, sb);
    uint64_t Jb[2 * NINT];
#pragma unroll
    for (int w = 0; w < 2 * NINT; ++w) Jb[w] = J[w];
    return sc_offdiag<NINT>(I, al, Jb, deg, sgl);
}

template <int NINT, int NS, bool BWD>
__global__ __launch_bounds__(WAVE) void sweep_kernel(const SweepArgs *__restrict__ sys,
                                                    const int64_t *__restrict__ item_end, int n_sys)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const int lane = threadIdx.x;
    // the items of all systems, system after system, are dealt round-robin
    // over the persistent grid (no shared counter); item_end[s] is the end of
    // system s's items
    const int64_t total = item_end[n_sys - 1];
    int sid = 0;
    int64_t ibase = 0;
    for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
        while (it >= item_end[sid]) ibase = item_end[sid++];
        ConstSys &a = ((ConstSys *)sys)[sid];
        const int64_t item = it - ibase;
        const int n = a.n;
        const int64_t n2 = (int64_t)n * n;
        const int P2 = n * (n - 1) / 2;
        const int nel = a.nel;
        const int nb = nel + nel * (nel - 1) / 2;
        const int Q = a.q_per_gen;
        const bool want_fp = (a.flags & 1) != 0;
        const bool want_sel = a.n_select > 0;

        // ----------------------------------------------------------- LDS layout
        unsigned lo_ = 0;
        double *sF = carve<double>(lds_raw, lo_, 2 * n);                   // Fock diagonal of I [spin][p]
        double *sRG = carve<double>(lds_raw, lo_, QPD_MAX_ORB);            // row vector: diagonal offset
        double *sCB = carve<double>(lds_raw, lo_, CSCAP * QPD_MAX_ORB);    // column-segment elements
        double *sFC = carve<double>(lds_raw, lo_, FCAP * NS);              // c_Jk of fine entries
        double *sL2H = carve<double>(lds_raw, lo_, L2CAP);                 // m = 2 cell elements
        double *sDCF = carve<double>(lds_raw, lo_, BWD ? FCAP * NS : 1);   // adjoint: dE/dc_J per entry
        double *sDHD = carve<double>(lds_raw, lo_, BWD ? n : 1);           // adjoint: diagonal of dE/dh
        uint64_t *sI = carve<uint64_t>(lds_raw, lo_, 2 * NINT);
        FineE *sFine = carve<FineE>(lds_raw, lo_, FCAP);
        uint32_t *sL2 = carve<uint32_t>(lds_raw, lo_, L2CAP);              // i1 | i2 << 8 | fine << 16 | ban << 24
        int32_t *sCS = carve<int32_t>(lds_raw, lo_, CSCAP);                // fine | col << 8
        uint8_t *sIL = carve<uint8_t>(lds_raw, lo_, ICAP);                 // inline fine entries
        uint16_t *sVidx = carve<uint16_t>(lds_raw, lo_, 2 * n);
        uint8_t *sOcc = carve<uint8_t>(lds_raw, lo_, 2 * QPD_MAX_ORB);
        uint8_t *sVirt = carve<uint8_t>(lds_raw, lo_, 2 * QPD_MAX_ORB);
        uint8_t *sCnt = carve<uint8_t>(lds_raw, lo_, 2 * n);
        uint8_t *sRS = carve<uint8_t>(lds_raw, lo_, QPD_MAX_ORB);          // row vector: phase bit
        uint64_t *sRowBits = carve<uint64_t>(lds_raw, lo_, 4);             // rows holding m = 2 cells
        uint32_t *sSplit = carve<uint32_t>(lds_raw, lo_, 16);              // split sweep: row, column flags

        double E0[NS], gup[NS], cI[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) { E0[k] = a.E0[k]; gup[k] = BWD ? a.gup[k] : 0.0; }

        int q, bstride, part = 0, nparts = 1;
        int64_t g, slot;
        if (a.def_mode) {
            // one part of one listed batch per item: its rows rr = part mod
            // nparts, so that a large batch does not rest on one wave; partials
            // go to the item's own slot
            nparts = a.def_parts;
            const int64_t de = item / nparts;
            part = (int)(item - de * nparts);
            g = a.def_g[de];
            q = (int)a.def_b[de];
            bstride = nb;
            slot = item;
        } else {
            q = (int)(item / a.n_gen);
            const int64_t gi = item - (int64_t)q * a.n_gen;
            g = a.gen_list ? (int64_t)a.gen_list[gi] : gi;
            bstride = Q;
            slot = gi * Q + q;
        }
        const int det = a.perm[g];

        // ------------------------------------------------------ generator data
        uint64_t Ib[2 * NINT];
#pragma unroll
        for (int w = 0; w < 2 * NINT; ++w) Ib[w] = a.dets[(int64_t)det * 2 * NINT + w];
        if (lane < 2 * NINT) sI[lane] = a.dets[(int64_t)det * 2 * NINT + lane];
        for (int x = lane; x < 2 * n; x += WAVE) {
            const int s = x >= n ? 1 : 0, p = x - s * n;
            int c = 0;
#pragma unroll
            for (int qq = 0; qq < NINT; ++qq) {
                const uint64_t wv = s ? Ib[NINT + qq] : Ib[qq];
                if (64 * qq + 63 < p) c += popc64(wv);
                else if (64 * qq <= p) c += popc64(wv & ((1ull << (p - 64 * qq)) - 1ull));
            }
            const bool occ = occ_bit<NINT>(Ib, s, p) != 0;
            sCnt[x] = (uint8_t)c;
            if (occ) { sOcc[s * QPD_MAX_ORB + c] = (uint8_t)p; sVidx[x] = 0xFFFF; }
            else { sVirt[s * QPD_MAX_ORB + p - c] = (uint8_t)p; sVidx[x] = (uint16_t)(p - c); }
            sF[x] = a.F[(g * 2) * n + x];
            if (BWD && s == 0) sDHD[p] = 0.0;
        }
#pragma unroll
        for (int k = 0; k < NS; ++k) cI[k] = a.coefs[(int64_t)k * a.n_det + det];
        const double HII = a.HII[g];
        const int64_t cbeg = a.coff[g], cend = a.coff[g + 1];
        __syncthreads();

        const int nup = a.nup;
        const int nv0 = n - a.nup, nv1 = n - a.ndn;

        double esum[NS], ssum[NS], dcI[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) { esum[k] = 0.0; ssum[k] = 0.0; dcI[k] = 0.0; }
        uint32_t cnt = 0, conn = 0;
        uint64_t fpsum = 0;
        double mind = __builtin_inf();
        double vtot = 0.0;

        for (int b = q; b < nb; b += bstride) {
            // ---------------------------------------------------- batch setup
            Batch B;
            {
                int i1, i2 = -1;
                if (b < nel) i1 = b;
                else tri_decode(b - nel, i1, i2);
                B.s1 = i1 < nup ? 0 : 1;
                B.h1 = i1 < nup ? sOcc[i1] : sOcc[QPD_MAX_ORB + i1 - nup];
                if (i2 < 0) {
                    B.type = BT_SINGLE; B.s2 = -1; B.h2 = -1;
                    B.rs = B.cs = B.s1; B.nr = B.nc = B.s1 == 0 ? nv0 : nv1;
                    B.sH = 0; B.D0 = HII - sF[B.s1 * n + B.h1]; B.blk = nullptr;
                } else {
                    B.s2 = i2 < nup ? 0 : 1;
                    B.h2 = i2 < nup ? sOcc[i2] : sOcc[QPD_MAX_ORB + i2 - nup];
                    if (B.s2 == B.s1) {
                        B.type = BT_SS;
                        B.rs = B.cs = B.s1; B.nr = B.nc = B.s1 == 0 ? nv0 : nv1;
                        B.sH = (sCnt[B.s1 * n + B.h1] + sCnt[B.s1 * n + B.h2] - 1) & 1;
                        B.D0 = HII - sF[B.s1 * n + B.h1] - sF[B.s1 * n + B.h2] + a.I.JK[B.h1 * n + B.h2];
                        B.blk = a.I.Y + qtris(B.h1, B.h2) * (int64_t)P2;
                    } else {
                        B.type = BT_OS;   // h1 up, h2 down
                        if (B.h1 <= B.h2) { B.rs = 0; B.cs = 1; B.blk = a.I.X + qtri(B.h1, B.h2) * n2; }
                        else { B.rs = 1; B.cs = 0; B.blk = a.I.X + qtri(B.h2, B.h1) * n2; }
                        B.nr = B.rs == 0 ? nv0 : nv1; B.nc = B.cs == 0 ? nv0 : nv1;
                        B.sH = (sCnt[B.h1] + sCnt[n + B.h2]) & 1;
                        B.D0 = HII - sF[B.h1] - sF[n + B.h2] + a.I.Jm[B.h1 * n + B.h2];
                    }
                }
            }
            const int hc0 = (B.s1 << 8) | B.h1;
            const int hc1 = B.type == BT_SINGLE ? -1 : ((B.s2 << 8) | B.h2);
            const uint8_t *rvirt = sVirt + B.rs * QPD_MAX_ORB;
            const uint8_t *cvirt = sVirt + B.cs * QPD_MAX_ORB;
            // same-spin and other-spin hole of the row spin
            const int hrs = B.type == BT_OS ? (B.rs == 0 ? B.h1 : B.h2) : B.h1;
            const int hro = B.type == BT_OS ? (B.rs == 0 ? B.h2 : B.h1) : (B.type == BT_SS ? B.h2 : -1);

            // split sweep: a hole-pair batch handed over by the split-correction
            // kernel (more fine entries than it holds) has its clean cells taken by
            // the clean-cell kernel; this kernel then keeps the flagged rows and
            // columns only
            bool skipc = false;
            if (a.split && B.type != BT_SINGLE) {
                if (lane < 16) sSplit[lane] = 0u;
                __syncthreads();
                skipc = split_flags(a, g, n, a.nup, a.ndn, B.type == BT_OS, B.rs, hc0, hc1, sVidx, sSplit,
                                    sSplit + 8, lane);
                __syncthreads();
            }
            auto flagged = [&](const uint32_t *m, int i) -> bool { return (m[i >> 5] >> (i & 31)) & 1u; };

            // row vector: phase bit and diagonal offset per row-spin particle
            for (int i = lane; i < B.nr; i += WAVE) {
                const int p = rvirt[i];
                int par = sCnt[B.rs * n + p] - (hrs < p);
                double gv = sF[B.rs * n + p] - a.I.JK[hrs * n + p];
                if (B.type == BT_SINGLE) par += sCnt[B.rs * n + B.h1];
                else if (B.type == BT_SS) { par -= (hro < p); gv -= a.I.JK[hro * n + p]; }
                else gv -= a.I.Jm[hro * n + p];
                sRS[i] = (uint8_t)(par & 1);
                sRG[i] = gv;
            }

            // ------------------------------------------------- fine filter
            int nfine = 0;
            for (int64_t base = cbeg; base < cend; base += WAVE) {
                const int64_t e = base + lane;
                bool keep = false;
                CoarseEnt ce;
                int m = 0;
                if (e < cend) {
                    ce = a.cent[e];
                    int dc = 0, in = 0;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int d = ce.D[t];
                        if (d == 0xFFFF) continue;
                        dc++;
                        in += (d == hc0) || (d == hc1);
                    }
                    m = dc - in;
                    keep = m <= 2;
                }
                const uint64_t mask = __ballot(keep);
                const int pos = nfine + __popcll(mask & ((1ull << lane) - 1ull));
                if (keep && pos < FCAP) {
                    FineE f;
                    f.j = ce.j; f.m = (uint8_t)m; f.earlier = (uint8_t)(ce.flags & 1);
                    int ner = 0, nec = 0;
                    uint32_t er = 0xFFFFFFFFu, ec = 0xFFFFFFFFu;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int ecode = ce.E[t];
                        if (ecode == 0xFFFF) continue;
                        const int es = ecode >> 8, ep = ecode & 255;
                        if (ep >= n) continue;
                        const int vi = sVidx[es * n + ep];
                        if (vi >= (es == 0 ? nv0 : nv1)) continue;
                        if (es == B.rs) {
                            er = (er & ~(255u << (8 * ner))) | ((uint32_t)vi << (8 * ner));
                            ner++;
                        } else if (B.type == BT_OS) {
                            ec = (ec & ~(255u << (8 * nec))) | ((uint32_t)vi << (8 * nec));
                            nec++;
                        }
                    }
                    f.ner = (uint8_t)ner; f.nec = (uint8_t)nec; f.er = er; f.ec = ec;
                    sFine[pos] = f;
#pragma unroll
                    for (int k = 0; k < NS; ++k) sFC[pos * NS + k] = a.coefs[(int64_t)k * a.n_det + ce.j];
                }
                nfine += __popcll(mask);
            }
            const bool fine_overflow = nfine > FCAP;
            if (fine_overflow) nfine = FCAP;
            __syncthreads();

            // ----------- classify: m = 2 cells, column segments, inline entries
            int nl2 = 0, ncs = 0, nil = 0;
            bool slow = fine_overflow;
            if (lane < 4) sRowBits[lane] = 0ull;
            for (int f = 0; f < nfine; ++f) {
                const FineE fe = sFine[f];
                bool inl = false;
                if (B.type == BT_SINGLE || fe.m == 0) inl = true;
                else if (fe.m == 2) {
                    if (B.type == BT_OS) {
                        for (int x = 0; x < fe.ner; ++x)
                            for (int y = 0; y < fe.nec; ++y) {
                                if (nl2 < L2CAP && lane == 0)
                                    sL2[nl2] = byte_at(fe.er, x) | (byte_at(fe.ec, y) << 8) | (f << 16) | ((uint32_t)fe.earlier << 24);
                                nl2++;
                            }
                    } else {
                        for (int x = 0; x < fe.ner; ++x)
                            for (int y = x + 1; y < fe.ner; ++y) {
                                const int i1 = byte_at(fe.er, x) < byte_at(fe.er, y) ? byte_at(fe.er, x) : byte_at(fe.er, y);
                                const int i2 = byte_at(fe.er, x) < byte_at(fe.er, y) ? byte_at(fe.er, y) : byte_at(fe.er, x);
                                if (nl2 < L2CAP && lane == 0)
                                    sL2[nl2] = i1 | (i2 << 8) | (f << 16) | ((uint32_t)fe.earlier << 24);
                                nl2++;
                            }
                    }
                } else {   // m == 1: column part -> segments; row part -> inline
                    const int nseg = B.type == BT_OS ? fe.nec : fe.ner;
                    for (int x = 0; x < nseg; ++x) {
                        const int col = B.type == BT_OS ? byte_at(fe.ec, x) : byte_at(fe.er, x);
                        if (ncs < CSCAP && lane == 0) sCS[ncs] = f | (col << 8);
                        ncs++;
                    }
                    inl = fe.ner > 0;
                }
                if (inl) {
                    if (nil < ICAP && lane == 0) sIL[nil] = (uint8_t)f;
                    nil++;
                }
            }
            if (nl2 > L2CAP || ncs > CSCAP || nil > ICAP) slow = true;
            if (slow) {
                // everything inline, touch rule evaluated per cell
                nl2 = 0; ncs = 0;
                nil = nfine;
            }
            __syncthreads();
            if (!slow) {
                // m = 2 cells: one lane each
                if (lane < nl2) {
                    const uint32_t e = sL2[lane];
                    const int i1 = e & 255, i2 = (e >> 8) & 255, f = (e >> 16) & 255;
                    double v = 0.0;
                    if (!((e >> 24) & 1)) {
                        int pa, sa, pb, sb;
                        if (B.type == BT_OS) { pa = rvirt[i1]; sa = B.rs; pb = cvirt[i2]; sb = B.cs; }
                        else { pa = rvirt[i1]; pb = rvirt[i2]; sa = sb = B.rs; }
                        int deg;
                        v = corr_element<NINT>(a.I, sI, hc0, hc1, pa, sa, pb, sb,
                                               a.dets + (int64_t)sFine[f].j * 2 * NINT, &deg, nullptr);
                        if (deg == 0) sL2[lane] = e | (1u << 24);   // alpha is internal
                    }
                    sL2H[lane] = v;
                    const int br = B.type == BT_SS ? (i2 <= B.nr / 2 ? i2 : B.nr - i2) : i1;
                    atomicOr((unsigned long long *)&sRowBits[br >> 6], 1ull << (br & 63));
                }
                // column segments: lanes over the rows of the segment
                for (int s = 0; s < ncs; ++s) {
                    const int f = sCS[s] & 255, col = sCS[s] >> 8;
                    const FineE fe = sFine[f];
                    if (fe.earlier) continue;
                    for (int r = lane; r < B.nr; r += WAVE) {
                        double v = 0.0;
                        const bool use = B.type == BT_OS ? !has(fe.er, fe.ner, r) : (r > col && !has(fe.er, fe.ner, r));
                        if (use) {
                            int pa, sa, pb, sb;
                            if (B.type == BT_OS) { pa = rvirt[r]; sa = B.rs; pb = cvirt[col]; sb = B.cs; }
                            else { pa = rvirt[col]; pb = rvirt[r]; sa = sb = B.rs; }
                            int deg;
                            v = corr_element<NINT>(a.I, sI, hc0, hc1, pa, sa, pb, sb,
                                                   a.dets + (int64_t)fe.j * 2 * NINT, &deg, nullptr);
                        }
                        sCB[s * QPD_MAX_ORB + r] = v;
                    }
                }
            }
            if (BWD) for (int x = lane; x < FCAP * NS; x += WAVE) sDCF[x] = 0.0;
            __syncthreads();

            const uint64_t tau_key = want_sel ? bin_edge(__atomic_load_n(a.tau_bin, __ATOMIC_RELAXED)) : 0ull;
            const double tau_val = __longlong_as_double((long long)tau_key) * (1.0 - 1e-12);
            bool appended = false;
            double vbatch = 0.0;

            // touch rule of an inline entry for the cell (i1, i2)
            auto inline_touch = [&](const FineE &fe, int i1, int i2) -> bool {
                if (B.type == BT_SINGLE) return fe.m <= 1 || has(fe.er, fe.ner, i1);
                if (fe.m == 0) return true;
                if (B.type == BT_OS) {
                    const bool inR = has(fe.er, fe.ner, i1), inC = has(fe.ec, fe.nec, i2);
                    if (fe.m == 1) return slow ? (inR || inC) : inR;
                    return slow && inR && inC;
                }
                const bool in1 = has(fe.er, fe.ner, i1), in2 = has(fe.er, fe.ner, i2);
                if (fe.m == 1) return slow ? (in1 || in2) : in2;
                return slow && in1 && in2;
            };

            // --------------------------------------------------- dense pass
            const int nrow = B.type == BT_OS ? B.nr : (B.type == BT_SS ? B.nr / 2 : 1);
            const int ncolv = B.type == BT_OS ? B.nc : B.nr;
            for (int c0 = 0; c0 < ncolv; c0 += WAVE) {
                const int l = c0 + lane;
                const bool lane_ok = l < ncolv;
                int pcol = 0, csg = 0;
                double cbase = 0.0, colacc = 0.0;
                if (B.type == BT_OS && lane_ok) {
                    pcol = cvirt[l];
                    const int hcs = B.cs == 0 ? B.h1 : B.h2, hco = B.cs == 0 ? B.h2 : B.h1;
                    csg = (B.sH + sCnt[B.cs * n + pcol] - (hcs < pcol)) & 1;
                    cbase = B.D0 + sF[B.cs * n + pcol] - a.I.JK[hcs * n + pcol] - a.I.Jm[hco * n + pcol];
                }
                for (int rr = part; rr < nrow; rr += nparts) {
                    const int r = B.type == BT_SS ? rr + 1 : rr;
                    bool act = lane_ok;
                    int i1, i2;
                    int pa = 0, sa = B.rs, pb = -1, sb = B.cs;
                    double Hval = 0.0, D = 0.0;
                    if (B.type == BT_OS) {
                        i1 = r; i2 = l;
                        pa = rvirt[r]; pb = pcol;
                        if (skipc) act = act && (flagged(sSplit, r) || flagged(sSplit + 8, l));
                        if (act) {
                            const double x = B.blk[(int64_t)pa * n + pb];
                            const double jj = a.I.Jm[(int64_t)pa * n + pb];
                            Hval = (csg ^ sRS[r]) ? -x : x;
                            D = cbase + sRG[r] + jj;
                        }
                    } else if (B.type == BT_SS) {
                        const bool partA = l < r;
                        i1 = partA ? l : l - r;
                        i2 = partA ? r : B.nr - r;
                        act = act && (partA || (B.nr - r > r));
                        if (skipc) act = act && (flagged(sSplit, i2) || flagged(sSplit + 8, i1));
                        pa = rvirt[act ? i1 : 0]; pb = rvirt[act ? i2 : 0]; sb = B.rs;
                        if (act) {
                            const double x = B.blk[qtris(pa, pb)];
                            const double jk = a.I.JK[(int64_t)pb * n + pa];
                            Hval = (B.sH ^ sRS[i1] ^ sRS[i2]) ? -x : x;
                            D = B.D0 + sRG[i1] + sRG[i2] + jk;
                        }
                    } else {
                        i1 = l; i2 = 0;
                        pa = rvirt[act ? l : 0];
                        if (act) {
                            const double f = fock_offdiag<NINT>(a.I, Ib, B.s1, B.h1, pa);
                            Hval = sRS[l] ? -f : f;
                            D = B.D0 + sRG[l];
                        }
                    }
                    // split sweep: a row with no flagged cell has nothing here
                    if (skipc && __ballot(act) == 0ull) continue;
                    double A[NS];
#pragma unroll
                    for (int k = 0; k < NS; ++k) A[k] = cI[k] * Hval;
                    bool banned = false;
                    int ncorr = 0;

                    // ---------------------------------------- corrections
                    const bool rowhit = nl2 > 0 && ((sRowBits[r >> 6] >> (r & 63)) & 1ull);
                    if (rowhit) {
                        for (int t = 0; t < nl2; ++t) {
                            const uint32_t e = sL2[t];
                            if (act && (int)(e & 255) == i1 && (int)((e >> 8) & 255) == i2) {
                                if ((e >> 24) & 1) banned = true;
                                else {
                                    const int f = (e >> 16) & 255;
                                    ncorr++;
#pragma unroll
                                    for (int k = 0; k < NS; ++k) A[k] += sFC[f * NS + k] * sL2H[t];
                                }
                            }
                        }
                    }
                    for (int s = 0; s < ncs; ++s) {
                        const int f = sCS[s] & 255, col = sCS[s] >> 8;
                        const FineE fe = sFine[f];
                        const int rowi = B.type == BT_OS ? i1 : i2;
                        const bool hit = act && (B.type == BT_OS ? i2 : i1) == col && !has(fe.er, fe.ner, rowi);
                        if (hit) {
                            if (fe.earlier) banned = true;
                            else {
                                ncorr++;
                                const double v = sCB[s * QPD_MAX_ORB + rowi];
#pragma unroll
                                for (int k = 0; k < NS; ++k) A[k] += sFC[f * NS + k] * v;
                            }
                        }
                    }
                    for (int t = 0; t < nil; ++t) {
                        const int f = slow ? t : sIL[t];
                        const FineE fe = sFine[f];
                        const bool touch = act && inline_touch(fe, i1, i2);
                        if (__ballot(touch) == 0ull) continue;
                        if (touch) {
                            if (fe.earlier) banned = true;
                            else {
                                int deg;
                                const double v = corr_element<NINT>(a.I, sI, hc0, hc1, pa, sa, pb, sb,
                                                                    a.dets + (int64_t)fe.j * 2 * NINT, &deg, nullptr);
                                if (deg == 0) banned = true;
                                else {
                                    ncorr++;
#pragma unroll
                                    for (int k = 0; k < NS; ++k) A[k] += sFC[f * NS + k] * v;
                                }
                            }
                        }
                    }
                    if (fine_overflow) {
                        // coarse entries beyond the first FCAP fine ones
                        int seen = 0;
                        for (int64_t e = cbeg; e < cend; ++e) {
                            const CoarseEnt ce = a.cent[e];
                            int dc = 0, in = 0;
                            for (int t = 0; t < 4; ++t) {
                                const int d = ce.D[t];
                                if (d == 0xFFFF) continue;
                                dc++;
                                in += (d == hc0) || (d == hc1);
                            }
                            if (dc - in > 2) continue;
                            if (seen++ < FCAP) continue;
                            if (!act) continue;
                            int deg;
                            const double v = corr_element<NINT>(a.I, sI, hc0, hc1, pa, sa, pb, sb,
                                                                a.dets + (int64_t)ce.j * 2 * NINT, &deg, nullptr);
                            if (deg > 2) continue;
                            if ((ce.flags & 1) || deg == 0) { banned = true; continue; }
                            ncorr++;
#pragma unroll
                            for (int k = 0; k < NS; ++k) A[k] += a.coefs[(int64_t)k * a.n_det + ce.j] * v;
                        }
                    }

                    // ------------------------------------------------ finalise
                    const bool live = act && !banned;
                    double ek[NS], rk[NS];
                    double tsel = 0.0, vsum = 0.0;
#pragma unroll
                    for (int k = 0; k < NS; ++k) {
                        const double delta = E0[k] - D;
                        const double rc = fast_rcp(delta);
                        const double e = (A[k] * A[k]) * rc;
                        ek[k] = e; rk[k] = rc;
                        if (live) {
                            esum[k] += e;
                            ssum[k] = fma(e, rc, ssum[k]);
                            mind = fmin(mind, fabs(delta));
                            tsel = fma(e, a.inv_maxc2[k], tsel);
                            if (BWD) vsum += gup[k] * e * rc;
                        }
                    }
                    if (live) {
                        cnt++;
                        conn += ncorr;
                        if (want_fp) {
                            uint64_t al[2 * NINT];
#pragma unroll
                            for (int w = 0; w < 2 * NINT; ++w) al[w] = alpha_word<NINT>(Ib, w, hc0, hc1, pa, sa, pb, sb);
                            fpsum += det_fold<NINT>(al);
                        }
                    }
                    if (want_sel) {
                        bool cand = live && fabs(tsel) >= tau_val;
                        uint64_t key = 0;
                        if (cand) {
                            double t = 0.0;
#pragma unroll
                            for (int k = 0; k < NS; ++k) t += ek[k] / a.maxc2[k];
                            key = (uint64_t)__double_as_longlong(fabs(t));
                            cand = key >= tau_key;
                        }
                        const uint64_t mask = __ballot(cand);
                        if (mask) {
                            const int leader = ctz64(mask);
                            unsigned long long base = 0;
                            if (lane == leader) base = atomicAdd(a.cand_count, (unsigned long long)__popcll(mask));
                            base = __shfl(base, leader);
                            appended = true;
                            if (cand) {
                                const unsigned long long sc = base + __popcll(mask & ((1ull << lane) - 1ull));
                                atomicAdd(&a.hist[key_bin(key)], 1u);
                                if ((int64_t)sc < a.cand_cap) {
                                    Cand cd;
                                    cd.key = key;
                                    const int up = (B.type == BT_OS) ? (sa == 0 ? pa : pb) : pa;
                                    const int dn = (B.type == BT_OS) ? (sa == 0 ? pb : pa) : (pb < 0 ? 0 : pb);
                                    cd.code = pack_code(B.type, B.s1, B.h1, B.h2 < 0 ? 0 : B.h2, up, dn);
                                    cd.g = (uint32_t)g;
                                    cd.pad = 0;
#pragma unroll
                                    for (int k = 0; k < QPD_MAX_STATES; ++k) cd.e[k] = k < NS ? ek[k] : 0.0;
                                    a.cand[sc] = cd;
                                } else {
                                    atomicOr(a.overflow, 1ull);
                                }
                            }
                        }
                    }

                    // ------------------------------------------------ adjoint
                    if (BWD) {
                        double w[NS];
#pragma unroll
                        for (int k = 0; k < NS; ++k) {
                            w[k] = live ? 2.0 * gup[k] * A[k] * rk[k] : 0.0;
                            dcI[k] += w[k] * Hval;
                        }
                        const double v = live ? vsum : 0.0;
                        vbatch += v;
                        // diagonal of dE/dh from the particles' occupations
                        if (B.type == BT_OS) {
                            const double rsum = wave_sum(v);
                            if (lane == 0 && rsum != 0.0) sDHD[rvirt[r]] += rsum;
                            colacc += v;
                        } else if (B.type == BT_SS) {
                            // part A shares i2 = r, part B shares i2 = V - r
                            const bool partA = l < r;
                            const double sA = wave_sum(partA ? v : 0.0), sB = wave_sum(partA ? 0.0 : v);
                            if (lane == 0) {
                                if (sA != 0.0) sDHD[rvirt[r]] += sA;
                                if (sB != 0.0 && B.nr - r > r) sDHD[rvirt[B.nr - r]] += sB;
                            }
                            if (v != 0.0) atomicAdd(&sDHD[pa], v);
                        } else if (live) {
                            atomicAdd(&sDHD[pa], v);
                            // single excitation of I: d<I|H|alpha>/dh_{h p} = phase
                            double gs = 0.0;
#pragma unroll
                            for (int k = 0; k < NS; ++k) gs += w[k] * cI[k];
                            if (a.dh && gs != 0.0) {
                                const double gg = 0.5 * (sRS[l] ? -gs : gs);
                                atomicAdd(&a.dh[(int64_t)B.h1 * n + pa], gg);
                                atomicAdd(&a.dh[(int64_t)pa * n + B.h1], gg);
                            }
                        }
                        // corrections: dE/dc_J += w <J|H|alpha>; single
                        // excitations J -> alpha also feed dE/dh
                        if (rowhit && live) {
                            for (int t = 0; t < nl2; ++t) {
                                const uint32_t e = sL2[t];
                                if ((int)(e & 255) == i1 && (int)((e >> 8) & 255) == i2 && !((e >> 24) & 1)) {
                                    const int f = (e >> 16) & 255;
#pragma unroll
                                    for (int k = 0; k < NS; ++k) atomicAdd(&sDCF[f * NS + k], w[k] * sL2H[t]);
                                }
                            }
                        }
                        for (int s = 0; s < ncs; ++s) {
                            const int f = sCS[s] & 255, col = sCS[s] >> 8;
                            const FineE fe = sFine[f];
                            if (fe.earlier) continue;
                            const int rowi = B.type == BT_OS ? i1 : i2;
                            const bool hit = live && (B.type == BT_OS ? i2 : i1) == col && !has(fe.er, fe.ner, rowi);
                            if (hit) {
                                const double hv = sCB[s * QPD_MAX_ORB + rowi];
#pragma unroll
                                for (int k = 0; k < NS; ++k) atomicAdd(&sDCF[f * NS + k], w[k] * hv);
                            }
                        }
                        for (int t = 0; t < nil; ++t) {
                            const int f = slow ? t : sIL[t];
                            const FineE fe = sFine[f];
                            if (fe.earlier) continue;
                            const bool touch = live && inline_touch(fe, i1, i2);
                            if (__ballot(touch) == 0ull) continue;
                            double hv = 0.0;
                            int deg = 0, sgl[4] = {-1, -1, 0, 0};
                            if (touch)
                                hv = corr_element<NINT>(a.I, sI, hc0, hc1, pa, sa, pb, sb,
                                                        a.dets + (int64_t)fe.j * 2 * NINT, &deg, sgl);
                            const bool ok = touch && deg >= 1 && deg <= 2;
#pragma unroll
                            for (int k = 0; k < NS; ++k) {
                                const double s_ = wave_sum(ok ? w[k] * hv : 0.0);
                                if (lane == 0 && s_ != 0.0) sDCF[f * NS + k] += s_;
                            }
                            if (ok && deg == 1 && a.dh) {
                                double gs = 0.0;
#pragma unroll
                                for (int k = 0; k < NS; ++k) gs += w[k] * sFC[f * NS + k];
                                const double gg = 0.5 * gs * sgl[3];
                                atomicAdd(&a.dh[(int64_t)sgl[0] * n + sgl[1]], gg);
                                atomicAdd(&a.dh[(int64_t)sgl[1] * n + sgl[0]], gg);
                            }
                        }
                        if (fine_overflow && live) {
                            int seen = 0;
                            for (int64_t e = cbeg; e < cend; ++e) {
                                const CoarseEnt ce = a.cent[e];
                                int dc = 0, in = 0;
                                for (int t = 0; t < 4; ++t) {
                                    const int d = ce.D[t];
                                    if (d == 0xFFFF) continue;
                                    dc++;
                                    in += (d == hc0) || (d == hc1);
                                }
                                if (dc - in > 2) continue;
                                if (seen++ < FCAP) continue;
                                if (ce.flags & 1) continue;
                                int deg, sgl[4];
                                const double hv = corr_element<NINT>(a.I, sI, hc0, hc1, pa, sa, pb, sb,
                                                                     a.dets + (int64_t)ce.j * 2 * NINT, &deg, sgl);
                                if (deg < 1 || deg > 2) continue;
                                double gs = 0.0;
#pragma unroll
                                for (int k = 0; k < NS; ++k) {
                                    const double cj = a.coefs[(int64_t)k * a.n_det + ce.j];
                                    if (a.dc) atomicAdd(&a.dc[(int64_t)k * a.n_det + ce.j], w[k] * hv);
                                    gs += w[k] * cj;
                                }
                                if (deg == 1 && a.dh) {
                                    const double gg = 0.5 * gs * sgl[3];
                                    atomicAdd(&a.dh[(int64_t)sgl[0] * n + sgl[1]], gg);
                                    atomicAdd(&a.dh[(int64_t)sgl[1] * n + sgl[0]], gg);
                                }
                            }
                        }
                    }
                }  // rows
                if (BWD && B.type == BT_OS && lane_ok && colacc != 0.0) atomicAdd(&sDHD[pcol], colacc);
            }  // column chunks

            if (want_sel && __ballot(appended)) {
                // raise the global threshold from the candidate histogram: the
                // highest bin b with at least n_select candidates at or above b
                constexpr int PER = QP_HIST_BINS / WAVE;
                uint32_t loc[PER];
                uint64_t tot = 0;
#pragma unroll
                for (int t = 0; t < PER; ++t) {
                    loc[t] = __atomic_load_n(&a.hist[lane * PER + t], __ATOMIC_RELAXED);
                    tot += loc[t];
                }
                uint64_t incl = tot;   // sum over lanes >= this lane
                for (int off = 1; off < WAVE; off <<= 1) {
                    const uint64_t v = __shfl_down(incl, off);
                    if (lane + off < WAVE) incl += v;
                }
                uint64_t cum = incl - tot;
                int best = -1;
                for (int t = PER - 1; t >= 0; --t) {
                    cum += loc[t];
                    if (cum >= (uint64_t)a.n_select) { best = lane * PER + t; break; }
                }
                for (int off = 32; off > 0; off >>= 1) {
                    const int o = __shfl_xor(best, off);
                    best = o > best ? o : best;
                }
                if (lane == 0 && best > 0) atomicMax(a.tau_bin, best);
            }
            if (BWD) {
                // holes: n_p(I - H) = n_p(I) - [p in H]
                const double vb = wave_sum(vbatch);
                __syncthreads();
                if (lane == 0) {
                    sDHD[B.h1] -= vb;
                    if (B.type != BT_SINGLE) sDHD[B.h2] -= vb;
                }
                vtot += vbatch;
                __syncthreads();
                for (int x = lane; x < nfine * NS; x += WAVE) {
                    const double v = sDCF[x];
                    if (v != 0.0 && a.dc) atomicAdd(&a.dc[(int64_t)(x % NS) * a.n_det + sFine[x / NS].j], v);
                }
            }
            __syncthreads();
        }  // batch

        // ------------------------------------------------- item reduction
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            esum[k] = wave_sum(esum[k]);
            ssum[k] = wave_sum(ssum[k]);
            if (BWD) dcI[k] = wave_sum(dcI[k]);
        }
        uint64_t cc = cnt, ff = fpsum, cn = conn;
        for (int off = 32; off > 0; off >>= 1) {
            cc += __shfl_xor(cc, off);
            ff += __shfl_xor(ff, off);
            cn += __shfl_xor(cn, off);
            mind = fmin(mind, __shfl_xor(mind, off));
        }
        vtot = wave_sum(vtot);
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                a.eps_item[slot * NS + k] = esum[k];
                a.S_item[slot * NS + k] = ssum[k];
                if (BWD) a.dc_item[slot * NS + k] = dcI[k];
            }
            a.cnt_item[slot] = (uint32_t)cc;
            if (a.fp_item) a.fp_item[slot] = ff;
            a.conn_item[slot] = (uint32_t)cn;
            // non-negative doubles order like their bit patterns; most items
            // cannot lower the minimum, so read before the atomic
            const unsigned long long mb = (unsigned long long)__double_as_longlong(mind);
            if (mb < __atomic_load_n(a.min_delta_bits, __ATOMIC_RELAXED)) atomicMin(a.min_delta_bits, mb);
        }
        if (BWD && a.dh) {
            __syncthreads();
            for (int x = lane; x < n; x += WAVE) {
                const int np = occ_bit<NINT>(Ib, 0, x) + occ_bit<NINT>(Ib, 1, x);
                const double v = sDHD[x] + np * vtot;
                if (v != 0.0) atomicAdd(&a.dh[(int64_t)x * n + x], v);
            }
        }
        __syncthreads();
    }
}

size_t sweep_lds_bytes(int n, int ns, bool bwd)
{
    size_t b = 0;
    auto add = [&](size_t bytes) { b = ((b + 15) & ~(size_t)15) + bytes; };
    add(8 * 2 * n); add(8 * QPD_MAX_ORB); add(8 * CSCAP * QPD_MAX_ORB); add(8 * FCAP * ns); add(8 * L2CAP);
    add(8 * (bwd ? FCAP * ns : 1)); add(8 * (bwd ? n : 1)); add(8 * 2 * QPD_MAX_NINT); add(sizeof(FineE) * FCAP);
    add(4 * L2CAP); add(4 * CSCAP); add(ICAP); add(2 * 2 * n); add(2 * QPD_MAX_ORB); add(2 * QPD_MAX_ORB); add(2 * n);
    add(QPD_MAX_ORB); add(8 * 4); add(4 * 16);
    return b + 16;
}

template <int NINT, int NS, bool BWD>
void launch_sweep(const SweepArgs *sys, const int64_t *item_end, int n_sys, size_t lds, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((sweep_kernel<NINT, NS, BWD>), dim3(grid), dim3(WAVE), lds, st, sys, item_end, n_sys);
}

template <int NINT, int NS, bool BWD>
int sweep_occupancy(size_t lds)
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, sweep_kernel<NINT, NS, BWD>, WAVE, lds) != hipSuccess)
        return 8;
    return blocks > 0 ? blocks : 1;
}

#define QP_INST(NI, NS)                                                                                         \
    template void launch_sweep<NI, NS, false>(const SweepArgs *, const int64_t *, int, size_t, int, hipStream_t); \
    template void launch_sweep<NI, NS, true>(const SweepArgs *, const int64_t *, int, size_t, int, hipStream_t);  \
    template int sweep_occupancy<NI, NS, false>(size_t);                                                       \
    template int sweep_occupancy<NI, NS, true>(size_t);
QP_INST(1, 1) QP_INST(1, 2) QP_INST(1, 3) QP_INST(1, 4)
QP_INST(2, 1) QP_INST(2, 2) QP_INST(2, 3) QP_INST(2, 4)
QP_INST(3, 1) QP_INST(3, 2) QP_INST(3, 3) QP_INST(3, 4)
QP_INST(4, 1) QP_INST(4, 2) QP_INST(4, 3) QP_INST(4, 4)
