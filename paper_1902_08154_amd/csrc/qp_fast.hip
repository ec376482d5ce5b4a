// qp_fast.hip -- the dense EN-PT2 / selection sweep for gfx950 (forward and
// adjoint): the kernel that handles almost every (generator, hole set) batch.
//
// Same decomposition and per-cell arithmetic as the general kernel
// (qp_sweep.hip): generators in order of decreasing sum_k c_Ik^2, batches by
// exact hole set, cells by particle set, <I|H|alpha> from one coalesced row of
// a per-hole-pair integral block, H_alpha,alpha by the Fock-diagonal update.
// What differs is how the other connected determinants J (the corrections)
// are handled: every correction element of a batch is evaluated first, with
// all lanes busy, into small LDS buffers --
//   * m = 2 entries: single cells (a list);
//   * m = 1 entries: whole rows (row buffers, lanes over columns) and whole
//     columns (column buffers, lanes over rows);
// -- and the dense pass only reads those buffers.  Batches that need more
// (an m = 0 entry, whose J touches every cell and may equal alpha, or more
// corrections than the buffers hold) are appended to a deferred list and
// processed afterwards by the general kernel; the per-generator reduction
// adds them in batch order, so results stay deterministic.
//
// Rows are processed in groups of ROWG: all integral reads of a group are
// issued before any is used, so their latency overlaps.
#include "qp_dev.h"

namespace {

constexpr int WAVE = 64;
constexpr int FCAP = 32;     // fine entries per batch
constexpr int L2CAP = 64;    // m = 2 cells per batch
constexpr int ROWG = 8;      // rows per prefetch group

struct FE {
    int32_t j;
    uint8_t m, earlier, ner, nec;
    uint32_t er;   // row-spin virtual indices of E = J \ I (one per byte)
    uint32_t ec;   // column-spin virtual indices of E
};

__device__ __forceinline__ double frcp(double d)
{
    // reciprocal to about one ulp: hardware estimate and two Newton steps
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    return d == 0.0 ? copysign(__builtin_inf(), d) : r;
}

__device__ __forceinline__ void tdec(int c, int &i1, int &i2)
{
    int t = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)c)) * 0.5f);
    while (t * (t - 1) / 2 > c) --t;
    while ((t + 1) * t / 2 <= c) ++t;
    i2 = t;
    i1 = c - t * (t - 1) / 2;
}

template <typename T>
__device__ __forceinline__ T *carve(unsigned char *base, unsigned &off, int count)
{
    off = (off + 15u) & ~15u;
    T *r = reinterpret_cast<T *>(base + off);
    off += (unsigned)(sizeof(T) * (unsigned)count);
    return r;
}

__device__ __forceinline__ int bat(uint32_t v, int t) { return (int)((v >> (8 * t)) & 255u); }
__device__ __forceinline__ bool has(uint32_t v, int nv, int x)
{
    bool r = false;
#pragma unroll
    for (int t = 0; t < 4; ++t) r |= (t < nv) && (bat(v, t) == x);
    return r;
}
__device__ __forceinline__ double wsum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// <J|H|alpha> for alpha = I - holes + particles (generic Slater-Condon)
template <int NINT>
__device__ __forceinline__ double celem(const DevInts &I, const uint64_t *Ib, int hc0, int hc1, int pa, int sa,
                                        int pb, int sb, const uint64_t *J, int *deg, int *sgl)
{
    uint64_t al[2 * NINT], jb[2 * NINT];
#pragma unroll
    for (int w = 0; w < 2 * NINT; ++w) {
        uint64_t x = Ib[w];
        const int base = 64 * (w % NINT), sp = w / NINT;
        if ((hc0 >> 8) == sp && (hc0 & 255) - base >= 0 && (hc0 & 255) - base < 64) x ^= 1ull << ((hc0 & 255) - base);
        if (hc1 >= 0 && (hc1 >> 8) == sp && (hc1 & 255) - base >= 0 && (hc1 & 255) - base < 64)
            x ^= 1ull << ((hc1 & 255) - base);
        if (sa == sp && pa - base >= 0 && pa - base < 64) x ^= 1ull << (pa - base);
        if (pb >= 0 && sb == sp && pb - base >= 0 && pb - base < 64) x ^= 1ull << (pb - base);
        al[w] = x;
        jb[w] = J[w];
    }
    return sc_offdiag<NINT>(I, al, jb, deg, sgl);
}

}  // namespace

size_t fast_lds_bytes(int n, int ns, bool bwd, int rscap, int cscap)
{
    size_t b = 0;
    auto add = [&](size_t bytes) { b = ((b + 15) & ~(size_t)15) + bytes; };
    add(8 * 2 * n);                 // F
    add(8 * n);                     // row vector G
    add(8 * rscap * n);             // row buffers
    add(4 * rscap * n);             // row buffer single-excitation info (adjoint)
    add(8 * cscap * n);             // column buffers
    add(8 * FCAP * ns);             // fine coefficients
    add(8 * L2CAP);                 // list values
    add(8 * (bwd ? FCAP * ns : 1)); // adjoint per-entry accumulators
    add(8 * (bwd ? n : 1));         // adjoint diagonal of dE/dh
    add(sizeof(FE) * FCAP);
    add(4 * L2CAP);
    add(4 * rscap);
    add(4 * cscap);
    add(2 * 2 * n);                 // vidx
    add(2 * QPD_MAX_ORB);           // occ
    add(2 * QPD_MAX_ORB);           // virt
    add(2 * n);                     // cnt
    add(n);                         // row vector phase bits
    add(8 * 4);                     // list row bits
    return b + 16;
}

template <int NINT, int NS, bool BWD>
__global__ __launch_bounds__(WAVE) void fast_kernel(SweepArgs a)
{
    extern __shared__ __align__(16) unsigned char lds[];
    const int n = a.n;
    const int lane = threadIdx.x;
    const int64_t n2 = (int64_t)n * n;
    const int P2 = n * (n - 1) / 2;
    const int nel = a.nel;
    const int nb = nel + nel * (nel - 1) / 2;
    const int Q = a.q_per_gen;
    const int RSCAP = a.rscap, CSCAP = a.cscap;
    const bool want_fp = (a.flags & 1) != 0;
    const bool want_sel = a.n_select > 0;

    unsigned off = 0;
    double *sF = carve<double>(lds, off, 2 * n);
    double *sRG = carve<double>(lds, off, n);
    double *sRB = carve<double>(lds, off, RSCAP * n);
    uint32_t *sRI = carve<uint32_t>(lds, off, RSCAP * n);
    double *sCB = carve<double>(lds, off, CSCAP * n);
    double *sFC = carve<double>(lds, off, FCAP * NS);
    double *sLH = carve<double>(lds, off, L2CAP);
    double *sDCF = carve<double>(lds, off, BWD ? FCAP * NS : 1);
    double *sDHD = carve<double>(lds, off, BWD ? n : 1);
    FE *sFine = carve<FE>(lds, off, FCAP);
    uint32_t *sL = carve<uint32_t>(lds, off, L2CAP);   // i1 | i2 << 8 | f << 16 | ban << 24
    uint32_t *sRSg = carve<uint32_t>(lds, off, RSCAP); // row | f << 16 | ban << 24
    uint32_t *sCSg = carve<uint32_t>(lds, off, CSCAP); // col | f << 16 | ban << 24
    uint16_t *sVidx = carve<uint16_t>(lds, off, 2 * n);
    uint8_t *sOcc = carve<uint8_t>(lds, off, 2 * QPD_MAX_ORB);
    uint8_t *sVirt = carve<uint8_t>(lds, off, 2 * QPD_MAX_ORB);
    uint8_t *sCnt = carve<uint8_t>(lds, off, 2 * n);
    uint8_t *sRS = carve<uint8_t>(lds, off, n);
    uint64_t *sLB = carve<uint64_t>(lds, off, 4);

    double E0[NS], gup[NS], cI[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) { E0[k] = a.E0[k]; gup[k] = BWD ? a.gup[k] : 0.0; }

    for (;;) {
        int it0 = 0;
        if (lane == 0) it0 = (int)atomicAdd(a.item_counter, 1u);
        const int64_t item = (int64_t)(unsigned)__builtin_amdgcn_readlane(it0, 0);
        if (item >= a.n_items) break;
        const int q = (int)(item / a.n_det);
        const int64_t g = item - (int64_t)q * a.n_det;
        const int64_t slot = g * Q + q;
        const int det = a.perm[g];

        uint64_t Ib[2 * NINT];
#pragma unroll
        for (int w = 0; w < 2 * NINT; ++w) Ib[w] = a.dets[(int64_t)det * 2 * NINT + w];
        for (int x = lane; x < 2 * n; x += WAVE) {
            const int s = x >= n ? 1 : 0, p = x - s * n;
            int c = 0;
#pragma unroll
            for (int qq = 0; qq < NINT; ++qq) {
                const uint64_t wv = Ib[s * NINT + qq];
                if (64 * qq + 63 < p) c += popc64(wv);
                else if (64 * qq <= p) c += popc64(wv & ((1ull << (p - 64 * qq)) - 1ull));
            }
            const bool occ = (Ib[s * NINT + (p >> 6)] >> (p & 63)) & 1ull;
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

        for (int b = q; b < nb; b += Q) {
            // ---------------------------------------------------- batch
            int type, s1, h1, s2 = -1, h2 = -1, rs, cs, nr, nc, sH;
            double D0;
            const double *blk = nullptr;
            {
                int i1, i2 = -1;
                if (b < nel) i1 = b;
                else tdec(b - nel, i1, i2);
                s1 = i1 < nup ? 0 : 1;
                h1 = i1 < nup ? sOcc[i1] : sOcc[QPD_MAX_ORB + i1 - nup];
                if (i2 < 0) {
                    type = BT_SINGLE; rs = cs = s1; nr = nc = s1 == 0 ? nv0 : nv1; sH = 0;
                    D0 = HII - sF[s1 * n + h1];
                } else {
                    s2 = i2 < nup ? 0 : 1;
                    h2 = i2 < nup ? sOcc[i2] : sOcc[QPD_MAX_ORB + i2 - nup];
                    if (s2 == s1) {
                        type = BT_SS; rs = cs = s1; nr = nc = s1 == 0 ? nv0 : nv1;
                        sH = (sCnt[s1 * n + h1] + sCnt[s1 * n + h2] - 1) & 1;
                        D0 = HII - sF[s1 * n + h1] - sF[s1 * n + h2] + a.I.JK[h1 * n + h2];
                        blk = a.I.Y + qtris(h1, h2) * (int64_t)P2;
                    } else {
                        type = BT_OS;
                        if (h1 <= h2) { rs = 0; cs = 1; blk = a.I.X + qtri(h1, h2) * n2; }
                        else { rs = 1; cs = 0; blk = a.I.X + qtri(h2, h1) * n2; }
                        nr = rs == 0 ? nv0 : nv1; nc = cs == 0 ? nv0 : nv1;
                        sH = (sCnt[h1] + sCnt[n + h2]) & 1;
                        D0 = HII - sF[h1] - sF[n + h2] + a.I.Jm[h1 * n + h2];
                    }
                }
            }
            const int hc0 = (s1 << 8) | h1;
            const int hc1 = type == BT_SINGLE ? -1 : ((s2 << 8) | h2);
            const uint8_t *rvirt = sVirt + rs * QPD_MAX_ORB;
            const uint8_t *cvirt = sVirt + cs * QPD_MAX_ORB;
            const int hrs = type == BT_OS ? (rs == 0 ? h1 : h2) : h1;
            const int hro = type == BT_OS ? (rs == 0 ? h2 : h1) : (type == BT_SS ? h2 : -1);

            for (int i = lane; i < nr; i += WAVE) {
                const int p = rvirt[i];
                int par = sCnt[rs * n + p] - (hrs < p);
                double gv = sF[rs * n + p] - a.I.JK[hrs * n + p];
                if (type == BT_SINGLE) par += sCnt[rs * n + h1];
                else if (type == BT_SS) { par -= (hro < p); gv -= a.I.JK[hro * n + p]; }
                else gv -= a.I.Jm[hro * n + p];
                sRS[i] = (uint8_t)(par & 1);
                sRG[i] = gv;
            }

            // ------------------------------------------------- fine filter
            int nfine = 0;
            bool slow = false;
            for (int64_t base = cbeg; base < cend; base += WAVE) {
                const int64_t e = base + lane;
                bool keep = false, m0 = false;
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
                    m0 = m == 0;
                }
                const uint64_t mask = __ballot(keep);
                if (__ballot(m0)) slow = true;
                const int pos = nfine + __popcll(mask & ((1ull << lane) - 1ull));
                if (keep && pos < FCAP) {
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
                        if (es == rs) { er = (er & ~(255u << (8 * ner))) | ((uint32_t)vi << (8 * ner)); ner++; }
                        else if (type == BT_OS) { ec = (ec & ~(255u << (8 * nec))) | ((uint32_t)vi << (8 * nec)); nec++; }
                    }
                    FE f;
                    f.j = ce.j; f.m = (uint8_t)m; f.earlier = (uint8_t)(ce.flags & 1);
                    f.ner = (uint8_t)ner; f.nec = (uint8_t)nec; f.er = er; f.ec = ec;
                    sFine[pos] = f;
#pragma unroll
                    for (int k = 0; k < NS; ++k) sFC[pos * NS + k] = a.coefs[(int64_t)k * a.n_det + ce.j];
                }
                nfine += __popcll(mask);
            }
            if (nfine > FCAP) slow = true;
            __syncthreads();

            // ------------------------------------------ classify corrections
            int nl = 0, nrs = 0, ncs = 0;
            if (!slow) {
                if (lane < 4) sLB[lane] = 0ull;
                for (int f = 0; f < nfine; ++f) {
                    const FE fe = sFine[f];
                    const uint32_t ban = fe.earlier ? (1u << 24) : 0u;
                    if (type == BT_SINGLE) {
                        if (fe.m <= 1) {
                            if (nrs < RSCAP && lane == 0) sRSg[nrs] = 0u | (f << 16) | ban;
                            nrs++;
                        } else {
                            for (int x = 0; x < fe.ner; ++x) {
                                if (nl < L2CAP && lane == 0) sL[nl] = bat(fe.er, x) | (f << 16) | ban;
                                nl++;
                            }
                        }
                    } else if (type == BT_OS) {
                        if (fe.m == 2) {
                            for (int x = 0; x < fe.ner; ++x)
                                for (int y = 0; y < fe.nec; ++y) {
                                    if (nl < L2CAP && lane == 0) sL[nl] = bat(fe.er, x) | (bat(fe.ec, y) << 8) | (f << 16) | ban;
                                    nl++;
                                }
                        } else {
                            for (int x = 0; x < fe.ner; ++x) {
                                if (nrs < RSCAP && lane == 0) sRSg[nrs] = bat(fe.er, x) | (f << 16) | ban;
                                nrs++;
                            }
                            for (int y = 0; y < fe.nec; ++y) {
                                if (ncs < CSCAP && lane == 0) sCSg[ncs] = bat(fe.ec, y) | (f << 16) | ban;
                                ncs++;
                            }
                        }
                    } else {   // BT_SS
                        if (fe.m == 2) {
                            for (int x = 0; x < fe.ner; ++x)
                                for (int y = x + 1; y < fe.ner; ++y) {
                                    const int u = bat(fe.er, x), v = bat(fe.er, y);
                                    if (nl < L2CAP && lane == 0)
                                        sL[nl] = (u < v ? u : v) | ((u < v ? v : u) << 8) | (f << 16) | ban;
                                    nl++;
                                }
                        } else {
                            for (int x = 0; x < fe.ner; ++x) {
                                const int ie = bat(fe.er, x);
                                if (nrs < RSCAP && lane == 0) sRSg[nrs] = ie | (f << 16) | ban;
                                nrs++;
                                if (ncs < CSCAP && lane == 0) sCSg[ncs] = ie | (f << 16) | ban;
                                ncs++;
                            }
                        }
                    }
                }
                if (nl > L2CAP || nrs > RSCAP || ncs > CSCAP) slow = true;
            }
            if (slow) {
                // the general kernel takes this batch
                if (lane == 0) {
                    const unsigned long long d = atomicAdd(a.def_count, 1ull);
                    if ((int64_t)d < a.def_cap) {
                        a.def_g[d] = (uint32_t)g;
                        a.def_b[d] = (uint32_t)b;
                        a.def_next[d] = atomicExch(&a.def_head[g], (int)d);
                    } else {
                        atomicOr(a.overflow, 2ull);
                    }
                }
                __syncthreads();
                continue;
            }
            __syncthreads();

            // --------------------------------- evaluate correction elements
            if (lane < nl) {
                const uint32_t e = sL[lane];
                double v = 0.0;
                if (!((e >> 24) & 1)) {
                    const int i1 = e & 255, i2 = (e >> 8) & 255, f = (e >> 16) & 255;
                    int pa, sa, pb = -1, sb = cs;
                    if (type == BT_OS) { pa = rvirt[i1]; sa = rs; pb = cvirt[i2]; }
                    else if (type == BT_SS) { pa = rvirt[i1]; pb = rvirt[i2]; sa = sb = rs; }
                    else { pa = rvirt[i1]; sa = rs; }
                    int deg;
                    v = celem<NINT>(a.I, Ib, hc0, hc1, pa, sa, pb, sb, a.dets + (int64_t)sFine[f].j * 2 * NINT,
                                    &deg, nullptr);
                }
                sLH[lane] = v;
                const int i1 = e & 255, i2 = (e >> 8) & 255;
                const int br = type == BT_SS ? (i2 <= nr / 2 ? i2 : nr - i2) : (type == BT_OS ? i1 : 0);
                atomicOr((unsigned long long *)&sLB[br >> 6], 1ull << (br & 63));
            }
            for (int s = 0; s < nrs; ++s) {
                const uint32_t sg = sRSg[s];
                if ((sg >> 24) & 1) continue;
                const int row = sg & 0xFFFF, f = (sg >> 16) & 255;
                const uint64_t *Jb = a.dets + (int64_t)sFine[f].j * 2 * NINT;
                // cells of the row: OS (row, c) for all c; SS (i1, row) for i1 < row;
                // SINGLE: every particle
                const int len = type == BT_OS ? nc : (type == BT_SS ? row : nr);
                for (int x = lane; x < len; x += WAVE) {
                    int pa, sa, pb = -1, sb = cs;
                    if (type == BT_OS) { pa = rvirt[row]; sa = rs; pb = cvirt[x]; }
                    else if (type == BT_SS) { pa = rvirt[x]; pb = rvirt[row]; sa = sb = rs; }
                    else { pa = rvirt[x]; sa = rs; }
                    int deg, sgl[4] = {-1, -1, 0, 0};
                    const double v = celem<NINT>(a.I, Ib, hc0, hc1, pa, sa, pb, sb, Jb, &deg, BWD ? sgl : nullptr);
                    sRB[s * n + x] = v;
                    if (BWD) sRI[s * n + x] = deg == 1 ? (uint32_t)(sgl[0] | (sgl[1] << 8) | ((sgl[3] < 0) << 16) | (1u << 17)) : 0u;
                }
            }
            for (int s = 0; s < ncs; ++s) {
                const uint32_t sg = sCSg[s];
                if ((sg >> 24) & 1) continue;
                const int col = sg & 0xFFFF, f = (sg >> 16) & 255;
                const FE fe = sFine[f];
                const uint64_t *Jb = a.dets + (int64_t)fe.j * 2 * NINT;
                for (int r = lane; r < nr; r += WAVE) {
                    double v = 0.0;
                    // OS: cells (r, col), r not in E_r; SS: cells (col, r), r > col, r not in E
                    const bool use = !has(fe.er, fe.ner, r) && (type == BT_OS || r > col);
                    if (use) {
                        int pa, sa, pb, sb;
                        if (type == BT_OS) { pa = rvirt[r]; sa = rs; pb = cvirt[col]; sb = cs; }
                        else { pa = rvirt[col]; pb = rvirt[r]; sa = sb = rs; }
                        int deg;
                        v = celem<NINT>(a.I, Ib, hc0, hc1, pa, sa, pb, sb, Jb, &deg, nullptr);
                    }
                    sCB[s * n + r] = v;
                }
            }
            if (BWD) for (int x = lane; x < FCAP * NS; x += WAVE) sDCF[x] = 0.0;
            __syncthreads();

            const uint64_t tau_key = want_sel ? bin_edge(__atomic_load_n(a.tau_bin, __ATOMIC_RELAXED)) : 0ull;
            const double tau_val = __longlong_as_double((long long)tau_key) * (1.0 - 1e-12);
            bool appended = false;
            double vbatch = 0.0;

            // --------------------------------------------------- dense pass
            const int nrow = type == BT_OS ? nr : (type == BT_SS ? nr / 2 : 1);
            const int ncolv = type == BT_OS ? nc : nr;
            for (int c0 = 0; c0 < ncolv; c0 += WAVE) {
                const int l = c0 + lane;
                const bool lok = l < ncolv;
                int pcol = 0, csg = 0;
                double cbase = 0.0, colacc = 0.0;
                if (type == BT_OS && lok) {
                    pcol = cvirt[l];
                    const int hcs = cs == 0 ? h1 : h2, hco = cs == 0 ? h2 : h1;
                    csg = (sH + sCnt[cs * n + pcol] - (hcs < pcol)) & 1;
                    cbase = D0 + sF[cs * n + pcol] - a.I.JK[hcs * n + pcol] - a.I.Jm[hco * n + pcol];
                }
                for (int g0 = 0; g0 < nrow; g0 += ROWG) {
                    // issue the group's integral reads first
                    double px[ROWG], pj[ROWG];
#pragma unroll
                    for (int u = 0; u < ROWG; ++u) {
                        px[u] = 0.0; pj[u] = 0.0;
                        const int rr = g0 + u;
                        if (rr >= nrow || !lok) continue;
                        if (type == BT_OS) {
                            const int pa = rvirt[rr];
                            px[u] = blk[(int64_t)pa * n + pcol];
                            pj[u] = a.I.Jm[(int64_t)pa * n + pcol];
                        } else if (type == BT_SS) {
                            const int r = rr + 1;
                            const bool pA = l < r;
                            if (pA || nr - r > r) {
                                const int i1 = pA ? l : l - r, i2 = pA ? r : nr - r;
                                const int pa = rvirt[i1], pb = rvirt[i2];
                                px[u] = blk[qtris(pa, pb)];
                                pj[u] = a.I.JK[(int64_t)pb * n + pa];
                            }
                        }
                    }
                    const int gend = (g0 + ROWG < nrow) ? ROWG : nrow - g0;
                    for (int u = 0; u < gend; ++u) {
                        // select the prefetched values without dynamic register indexing
                        double x = 0.0, xj = 0.0;
#pragma unroll
                        for (int t = 0; t < ROWG; ++t) if (t == u) { x = px[t]; xj = pj[t]; }
                        const int rr = g0 + u;
                        const int r = type == BT_SS ? rr + 1 : rr;
                        bool act = lok;
                        int i1, i2, pa = 0, pb = -1;
                        double Hv = 0.0, D = 0.0;
                        if (type == BT_OS) {
                            i1 = r; i2 = l; pa = rvirt[r]; pb = pcol;
                            Hv = (csg ^ sRS[r]) ? -x : x;
                            D = cbase + sRG[r] + xj;
                        } else if (type == BT_SS) {
                            const bool pA = l < r;
                            i1 = pA ? l : l - r;
                            i2 = pA ? r : nr - r;
                            act = act && (pA || nr - r > r);
                            if (act) {
                                pa = rvirt[i1]; pb = rvirt[i2];
                                Hv = (sH ^ sRS[i1] ^ sRS[i2]) ? -x : x;
                                D = D0 + sRG[i1] + sRG[i2] + xj;
                            }
                        } else {
                            i1 = l; i2 = 0;
                            if (act) {
                                pa = rvirt[l];
                                const double fv = fock_offdiag<NINT>(a.I, Ib, s1, h1, pa);
                                Hv = sRS[l] ? -fv : fv;
                                D = D0 + sRG[l];
                            }
                        }
                        double A[NS];
#pragma unroll
                        for (int k = 0; k < NS; ++k) A[k] = cI[k] * Hv;
                        bool banned = false;
                        int ncorr = 0;
                        // row buffers
                        for (int s = 0; s < nrs; ++s) {
                            const uint32_t sg = sRSg[s];
                            const int row = sg & 0xFFFF;
                            bool hit;
                            int x_;
                            if (type == BT_OS) { hit = row == i1; x_ = i2; }
                            else if (type == BT_SS) { hit = row == i2; x_ = i1; }
                            else { hit = true; x_ = i1; }
                            if (hit && act) {
                                if ((sg >> 24) & 1) banned = true;
                                else {
                                    const int f = (sg >> 16) & 255;
                                    const double v = sRB[s * n + x_];
                                    ncorr++;
#pragma unroll
                                    for (int k = 0; k < NS; ++k) A[k] += sFC[f * NS + k] * v;
                                }
                            }
                        }
                        // column buffers
                        for (int s = 0; s < ncs; ++s) {
                            const uint32_t sg = sCSg[s];
                            const int col = sg & 0xFFFF, f = (sg >> 16) & 255;
                            const int rowi = type == BT_OS ? i1 : i2;
                            const bool hit = act && (type == BT_OS ? i2 : i1) == col &&
                                             !has(sFine[f].er, sFine[f].ner, rowi);
                            if (hit) {
                                if ((sg >> 24) & 1) banned = true;
                                else {
                                    const double v = sCB[s * n + rowi];
                                    ncorr++;
#pragma unroll
                                    for (int k = 0; k < NS; ++k) A[k] += sFC[f * NS + k] * v;
                                }
                            }
                        }
                        // m = 2 cells
                        const bool lrow = nl > 0 && ((sLB[r >> 6] >> (r & 63)) & 1ull);
                        if (lrow) {
                            for (int t = 0; t < nl; ++t) {
                                const uint32_t e = sL[t];
                                if (act && (int)(e & 255) == i1 && (int)((e >> 8) & 255) == i2) {
                                    if ((e >> 24) & 1) banned = true;
                                    else {
                                        const int f = (e >> 16) & 255;
                                        ncorr++;
#pragma unroll
                                        for (int k = 0; k < NS; ++k) A[k] += sFC[f * NS + k] * sLH[t];
                                    }
                                }
                            }
                        }

                        // ------------------------------------------ finalise
                        const bool live = act && !banned;
                        double ek[NS], rk[NS], tsel = 0.0, vsum = 0.0;
#pragma unroll
                        for (int k = 0; k < NS; ++k) {
                            const double delta = E0[k] - D;
                            const double rc = frcp(delta);
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
                                for (int w = 0; w < 2 * NINT; ++w) al[w] = Ib[w];
                                al[(hc0 >> 8) * NINT + ((hc0 & 255) >> 6)] ^= 1ull << (hc0 & 63);
                                if (hc1 >= 0) al[(hc1 >> 8) * NINT + ((hc1 & 255) >> 6)] ^= 1ull << (hc1 & 63);
                                al[rs * NINT + (pa >> 6)] ^= 1ull << (pa & 63);
                                if (pb >= 0) al[(type == BT_OS ? cs : rs) * NINT + (pb >> 6)] ^= 1ull << (pb & 63);
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
                                        const int up = type == BT_OS ? (rs == 0 ? pa : pb) : pa;
                                        const int dn = type == BT_OS ? (rs == 0 ? pb : pa) : (pb < 0 ? 0 : pb);
                                        cd.code = pack_code(type, s1, h1, h2 < 0 ? 0 : h2, up, dn);
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

                        // ------------------------------------------- adjoint
                        if (BWD) {
                            double w[NS];
#pragma unroll
                            for (int k = 0; k < NS; ++k) {
                                w[k] = live ? 2.0 * gup[k] * A[k] * rk[k] : 0.0;
                                dcI[k] += w[k] * Hv;
                            }
                            const double v = live ? vsum : 0.0;
                            vbatch += v;
                            if (type == BT_OS) {
                                const double rsum = wsum(v);
                                if (lane == 0 && rsum != 0.0) sDHD[rvirt[r]] += rsum;
                                colacc += v;
                            } else if (type == BT_SS) {
                                const bool pA = l < r;
                                const double sA = wsum(pA ? v : 0.0), sB = wsum(pA ? 0.0 : v);
                                if (lane == 0) {
                                    if (sA != 0.0) sDHD[rvirt[r]] += sA;
                                    if (sB != 0.0 && nr - r > r) sDHD[rvirt[nr - r]] += sB;
                                }
                                if (v != 0.0) atomicAdd(&sDHD[pa], v);
                            } else if (live) {
                                atomicAdd(&sDHD[pa], v);
                                double gs = 0.0;
#pragma unroll
                                for (int k = 0; k < NS; ++k) gs += w[k] * cI[k];
                                if (a.dh && gs != 0.0) {
                                    const double gg = 0.5 * (sRS[l] ? -gs : gs);
                                    atomicAdd(&a.dh[(int64_t)h1 * n + pa], gg);
                                    atomicAdd(&a.dh[(int64_t)pa * n + h1], gg);
                                }
                            }
                            // corrections: dE/dc_J += w <J|H|alpha>
                            for (int s = 0; s < nrs; ++s) {
                                const uint32_t sg = sRSg[s];
                                if ((sg >> 24) & 1) continue;
                                const int row = sg & 0xFFFF, f = (sg >> 16) & 255;
                                bool hit;
                                int x_;
                                if (type == BT_OS) { hit = row == i1; x_ = i2; }
                                else if (type == BT_SS) { hit = row == i2; x_ = i1; }
                                else { hit = true; x_ = i1; }
                                hit = hit && live;
                                if (__ballot(hit) == 0ull) continue;
                                const double hv = hit ? sRB[s * n + x_] : 0.0;
#pragma unroll
                                for (int k = 0; k < NS; ++k) {
                                    const double t_ = wsum(w[k] * hv);
                                    if (lane == 0 && t_ != 0.0) sDCF[f * NS + k] += t_;
                                }
                                const uint32_t inf = hit ? sRI[s * n + x_] : 0u;
                                if ((inf >> 17) & 1u) {
                                    double gs = 0.0;
#pragma unroll
                                    for (int k = 0; k < NS; ++k) gs += w[k] * sFC[f * NS + k];
                                    const double gg = 0.5 * (((inf >> 16) & 1u) ? -gs : gs);
                                    const int hh = inf & 255, pp = (inf >> 8) & 255;
                                    if (a.dh) {
                                        atomicAdd(&a.dh[(int64_t)hh * n + pp], gg);
                                        atomicAdd(&a.dh[(int64_t)pp * n + hh], gg);
                                    }
                                }
                            }
                            for (int s = 0; s < ncs; ++s) {
                                const uint32_t sg = sCSg[s];
                                if ((sg >> 24) & 1) continue;
                                const int col = sg & 0xFFFF, f = (sg >> 16) & 255;
                                const int rowi = type == BT_OS ? i1 : i2;
                                const bool hit = live && (type == BT_OS ? i2 : i1) == col &&
                                                 !has(sFine[f].er, sFine[f].ner, rowi);
                                if (hit) {
                                    const double hv = sCB[s * n + rowi];
#pragma unroll
                                    for (int k = 0; k < NS; ++k) atomicAdd(&sDCF[f * NS + k], w[k] * hv);
                                }
                            }
                            if (lrow && live) {
                                for (int t = 0; t < nl; ++t) {
                                    const uint32_t e = sL[t];
                                    if ((int)(e & 255) == i1 && (int)((e >> 8) & 255) == i2 && !((e >> 24) & 1)) {
                                        const int f = (e >> 16) & 255;
#pragma unroll
                                        for (int k = 0; k < NS; ++k) atomicAdd(&sDCF[f * NS + k], w[k] * sLH[t]);
                                    }
                                }
                            }
                        }
                    }  // rows of the group
                }  // row groups
                if (BWD && type == BT_OS && lok && colacc != 0.0) atomicAdd(&sDHD[pcol], colacc);
            }  // column chunks

            if (want_sel && __ballot(appended)) {
                constexpr int PER = QP_HIST_BINS / WAVE;
                uint64_t tot = 0;
#pragma unroll
                for (int t = 0; t < PER; ++t) tot += __atomic_load_n(&a.hist[lane * PER + t], __ATOMIC_RELAXED);
                uint64_t incl = tot;
                for (int o = 1; o < WAVE; o <<= 1) {
                    const uint64_t v = __shfl_down(incl, o);
                    if (lane + o < WAVE) incl += v;
                }
                uint64_t cum = incl - tot;
                int best = -1;
                for (int t = PER - 1; t >= 0; --t) {
                    cum += __atomic_load_n(&a.hist[lane * PER + t], __ATOMIC_RELAXED);
                    if (cum >= (uint64_t)a.n_select) { best = lane * PER + t; break; }
                }
                for (int o = 32; o > 0; o >>= 1) {
                    const int ob = __shfl_xor(best, o);
                    best = ob > best ? ob : best;
                }
                if (lane == 0 && best > 0) atomicMax(a.tau_bin, best);
            }
            if (BWD) {
                const double vb = wsum(vbatch);
                __syncthreads();
                if (lane == 0) {
                    sDHD[h1] -= vb;
                    if (type != BT_SINGLE) sDHD[h2] -= vb;
                }
                vtot += vbatch;
                __syncthreads();
                for (int x = lane; x < nfine * NS; x += WAVE) {
                    const double v = sDCF[x];
                    if (v != 0.0 && a.dc) atomicAdd(&a.dc[(int64_t)(x % NS) * a.n_det + sFine[x / NS].j], v);
                }
            }
            __syncthreads();
        }  // batches

#pragma unroll
        for (int k = 0; k < NS; ++k) {
            esum[k] = wsum(esum[k]);
            ssum[k] = wsum(ssum[k]);
            if (BWD) dcI[k] = wsum(dcI[k]);
        }
        uint64_t cc = cnt, ff = fpsum, cn = conn;
        for (int o = 32; o > 0; o >>= 1) {
            cc += __shfl_xor(cc, o);
            ff += __shfl_xor(ff, o);
            cn += __shfl_xor(cn, o);
            mind = fmin(mind, __shfl_xor(mind, o));
        }
        vtot = wsum(vtot);
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                a.eps_item[slot * NS + k] = esum[k];
                a.S_item[slot * NS + k] = ssum[k];
                if (BWD) a.dc_item[slot * NS + k] = dcI[k];
            }
            a.cnt_item[slot] = (uint32_t)cc;
            if (a.fp_item) a.fp_item[slot] = ff;
            if (cn) atomicAdd((unsigned long long *)a.conn_total, (unsigned long long)cn);
            atomicMin(a.min_delta_bits, (unsigned long long)__double_as_longlong(mind));
        }
        if (BWD && a.dh) {
            __syncthreads();
            for (int x = lane; x < n; x += WAVE) {
                const int np = (int)((Ib[x >> 6] >> (x & 63)) & 1ull) + (int)((Ib[NINT + (x >> 6)] >> (x & 63)) & 1ull);
                const double v = sDHD[x] + np * vtot;
                if (v != 0.0) atomicAdd(&a.dh[(int64_t)x * n + x], v);
            }
        }
        __syncthreads();
    }
}

template <int NINT, int NS, bool BWD>
void launch_fast(const SweepArgs &a, int grid, hipStream_t st)
{
    const size_t lds = fast_lds_bytes(a.n, NS, BWD, a.rscap, a.cscap);
    hipLaunchKernelGGL((fast_kernel<NINT, NS, BWD>), dim3(grid), dim3(WAVE), lds, st, a);
}

template <int NINT, int NS, bool BWD>
int fast_occupancy(int n, int rscap, int cscap)
{
    int blocks = 0;
    const size_t lds = fast_lds_bytes(n, NS, BWD, rscap, cscap);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fast_kernel<NINT, NS, BWD>, WAVE, lds) != hipSuccess)
        return 8;
    return blocks > 0 ? blocks : 1;
}

#define QPF_INST(NI, NS)                                                            \
    template void launch_fast<NI, NS, false>(const SweepArgs &, int, hipStream_t);  \
    template void launch_fast<NI, NS, true>(const SweepArgs &, int, hipStream_t);   \
    template int fast_occupancy<NI, NS, false>(int, int, int);                      \
    template int fast_occupancy<NI, NS, true>(int, int, int);
QPF_INST(1, 1) QPF_INST(1, 2) QPF_INST(1, 3) QPF_INST(1, 4)
QPF_INST(2, 1) QPF_INST(2, 2) QPF_INST(2, 3) QPF_INST(2, 4)
QPF_INST(3, 1) QPF_INST(3, 2) QPF_INST(3, 3) QPF_INST(3, 4)
QPF_INST(4, 1) QPF_INST(4, 2) QPF_INST(4, 3) QPF_INST(4, 4)
