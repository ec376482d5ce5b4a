// qp_sweep.hip -- the per-generator EN-PT2 / selection sweep (forward and
// adjoint) for gfx950.
//
// Work decomposition (sec. "CIPSI selection and PT2 energy", appendix on the
// selection implementation): generators I in order of decreasing sum_k c_Ik^2;
// for each I the external determinants alpha = I - H + P are enumerated by
// hole set H (|H| = 1 or 2, exact holes) and particle set P (virtual orbitals
// of I of matching spins), so each (I, alpha) pair appears exactly once.  A
// batch is one hole set; its cells are the particle sets.  A work item is
// (generator, first hole h1): the single batch {h1} plus every double batch
// {h1, h2} with h2 after h1 in spin-orbital order.  A persistent grid takes
// items from an atomic counter.
//
// Per batch:
//   * the generator's own element <I|H|alpha> is a closed form per cell: a
//     separable phase (hole part x row part x column part) times one coalesced
//     read of the per-hole-pair integral block (X for opposite spins, Y for
//     same spin) or a Fock element of I (singles);
//   * the diagonal <alpha|H|alpha> is the ionised-determinant energy plus two
//     per-particle Fock terms plus one pair term (Fock-diagonal update of the
//     same appendix);
//   * other internal determinants J within degree 4 of I (coarse list) that
//     pass the fine filter m = |(I-H) \ J| <= 2 touch only the cells with
//     |P \ J| <= 2 - m: all cells (m = 0), rows/columns (m = 1) or a few
//     cells (m = 2).  They are scattered into an LDS tile: J earlier in the
//     generator order bans the cell (alpha belongs to an earlier generator),
//     J = alpha bans it (alpha is internal), otherwise c_J <J|H|alpha> is
//     added.  Batches without such J skip the tile entirely.
//   * finalise: e_k = A_k^2 / (E0_k - D), partial sums, selection candidates
//     above the running global threshold.
#include "qp_dev.h"

namespace {

struct FineEnt {
    int j;
    int m;
    int earlier;
    uint16_t E[4];
};

#define FCAP 64

struct Batch {
    int type;       // BT_*
    int s1, h1;     // first hole (spin, orbital)
    int s2, h2;     // second hole (double batches)
    int rs, cs;     // row / column spin (OS); SS and SINGLE use rs only
    int nr, nc;     // rows / columns (OS); V for SS and SINGLE
    int64_t ncell;
    int sH;         // hole part of the phase (0/1)
    double D0;      // energy of the ionised determinant I - H
    const double *blk;  // integral block base (X or Y row)
};

__device__ __forceinline__ void wg_barrier() { __syncthreads(); }

// decode SS triangle index c -> (i1 < i2), c = i2(i2-1)/2 + i1
__device__ __forceinline__ void tri_decode(int64_t c, int &i1, int &i2)
{
    int t = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)c)) * 0.5f);
    while ((int64_t)t * (t - 1) / 2 > c) --t;
    while ((int64_t)(t + 1) * t / 2 <= c) ++t;
    i2 = t;
    i1 = (int)(c - (int64_t)t * (t - 1) / 2);
}

}  // namespace

template <int NINT, int NS, bool BWD>
__global__ __launch_bounds__(QPD_WG) void sweep_kernel(SweepArgs a)
{
    constexpr int SLAB = (BWD ? 2048 : 3072) / NS;
    constexpr int NWAVE = QPD_WG / 64;

    __shared__ double s_F[2][QPD_MAX_ORB];
    __shared__ double s_G[2][QPD_MAX_ORB];
    __shared__ uint8_t s_sg[2][QPD_MAX_ORB];
    __shared__ uint8_t s_occ[2][QPD_MAX_ORB];
    __shared__ uint8_t s_virt[2][QPD_MAX_ORB];
    __shared__ uint8_t s_cnt[2][QPD_MAX_ORB];
    __shared__ uint16_t s_vidx[2][QPD_MAX_ORB];
    __shared__ uint64_t s_I[2 * NINT];
    __shared__ double s_tile[NS * SLAB];
    __shared__ double s_vt[BWD ? SLAB : 1];
    __shared__ double s_dhd[BWD ? QPD_MAX_ORB : 1];
    __shared__ double s_dhrow[BWD ? QPD_MAX_ORB : 1];
    __shared__ uint32_t s_ban[(SLAB + 31) / 32];
    __shared__ FineEnt s_fine[FCAP];
    __shared__ double s_fc[FCAP][NS];
    __shared__ int s_nfine;
    __shared__ int64_t s_fpos;
    __shared__ int s_item_ok;
    __shared__ unsigned int s_item;
    __shared__ int s_appended;
    __shared__ uint64_t s_tau_key;
    __shared__ double s_red[NWAVE][2 * NS + 2];
    __shared__ uint64_t s_redu[NWAVE][3];
    __shared__ double s_HII;
    __shared__ double s_vtot;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int n = a.n;
    const int64_t n2 = (int64_t)n * n;
    const int nel = a.nel;
    const int P2 = n * (n - 1) / 2;
    const bool want_fp = (a.flags & 1) != 0;
    const bool want_sel = a.n_select > 0;

    double cI[NS], E0[NS], gup[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) { E0[k] = a.E0[k]; gup[k] = BWD ? a.gup[k] : 0.0; }

    for (;;) {
        if (tid == 0) s_item = atomicAdd(a.item_counter, 1u);
        wg_barrier();
        const int64_t item = s_item;
        if (item >= a.n_items) break;
        const int ih = (int)(item / a.n_det);
        const int64_t g = item - (int64_t)ih * a.n_det;
        const int64_t slot = g * nel + ih;
        const int det = a.perm[g];

        // ---------------------------------------------------------- generator
        if (tid < 2 * NINT) s_I[tid] = a.dets[(int64_t)det * 2 * NINT + tid];
        if (tid == 0) { s_HII = a.HII[g]; s_appended = 0; }
        wg_barrier();
        for (int x = tid; x < 2 * n; x += QPD_WG) {
            int s = x / n, p = x - s * n;
            const uint64_t *w = s_I + s * NINT;
            int c = 0;
#pragma unroll
            for (int q = 0; q < NINT; ++q) {
                if (64 * q + 63 < p) c += popc64(w[q]);
                else if (64 * q <= p) c += popc64(w[q] & ((1ull << (p - 64 * q)) - 1ull));
            }
            int occ = (int)((w[p >> 6] >> (p & 63)) & 1ull);
            s_cnt[s][p] = (uint8_t)c;
            if (occ) { s_occ[s][c] = (uint8_t)p; s_vidx[s][p] = 0xFFFF; }
            else { s_virt[s][p - c] = (uint8_t)p; s_vidx[s][p] = (uint16_t)(p - c); }
            s_F[s][p] = a.F[(g * 2 + s) * n + p];
            if (BWD) { if (s == 0) s_dhd[p] = 0.0; }
        }
#pragma unroll
        for (int k = 0; k < NS; ++k) cI[k] = a.coefs[(int64_t)k * a.n_det + det];
        wg_barrier();

        const int nup = a.nup, ndn = a.ndn;
        const int nv0 = n - nup, nv1 = n - ndn;
        const int s1 = ih < nup ? 0 : 1;
        const int h1 = ih < nup ? s_occ[0][ih] : s_occ[1][ih - nup];
        const int64_t cbeg = a.coff[g], cend = a.coff[g + 1];

        double esum[NS], ssum[NS], dcI[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) { esum[k] = 0.0; ssum[k] = 0.0; dcI[k] = 0.0; }
        uint32_t cnt = 0, conn = 0;
        uint64_t fpsum = 0;
        double mind = __longlong_as_double(0x7ff0000000000000ll);
        double vtot = 0.0;   // BWD: sum over the item's alpha of v (for n_p(I))

        const int nb = nel - ih;
        for (int b = 0; b < nb; ++b) {
            // ------------------------------------------------------ batch setup
            Batch B;
            B.s1 = s1; B.h1 = h1;
            if (b == 0) {
                B.type = BT_SINGLE; B.s2 = -1; B.h2 = -1;
                B.rs = s1; B.cs = s1;
                B.nr = s1 == 0 ? nv0 : nv1; B.nc = 1;
                B.ncell = B.nr;
                B.sH = 0;
                B.D0 = s_HII - s_F[s1][h1];
                B.blk = nullptr;
            } else {
                int i2 = ih + b;
                B.s2 = i2 < nup ? 0 : 1;
                B.h2 = i2 < nup ? s_occ[0][i2] : s_occ[1][i2 - nup];
                if (B.s2 == s1) {
                    B.type = BT_SS;
                    B.rs = s1; B.cs = s1;
                    B.nr = s1 == 0 ? nv0 : nv1; B.nc = B.nr;
                    B.ncell = (int64_t)B.nr * (B.nr - 1) / 2;
                    B.sH = (s_cnt[s1][B.h1] + s_cnt[s1][B.h2] - 1) & 1;
                    B.D0 = s_HII - s_F[s1][B.h1] - s_F[s1][B.h2] + a.I.Jm[B.h1 * n + B.h2] -
                           a.I.Km[B.h1 * n + B.h2];
                    B.blk = a.I.Y + qtris(B.h1, B.h2) * (int64_t)P2;
                } else {
                    B.type = BT_OS;  // s1 = up, s2 = down
                    if (B.h1 <= B.h2) { B.rs = 0; B.cs = 1; B.blk = a.I.X + qtri(B.h1, B.h2) * n2; }
                    else { B.rs = 1; B.cs = 0; B.blk = a.I.X + qtri(B.h2, B.h1) * n2; }
                    B.nr = B.rs == 0 ? nv0 : nv1;
                    B.nc = B.cs == 0 ? nv0 : nv1;
                    B.ncell = (int64_t)B.nr * B.nc;
                    B.sH = (s_cnt[0][B.h1] + s_cnt[1][B.h2]) & 1;
                    B.D0 = s_HII - s_F[0][B.h1] - s_F[1][B.h2] + a.I.Jm[B.h1 * n + B.h2];
                }
            }
            // per-particle vectors: index 0 = row spin, 1 = column spin
            {
                const int nvec = (B.type == BT_OS) ? 2 : 1;
                for (int x = tid; x < nvec * QPD_MAX_ORB; x += QPD_WG) {
                    int v = x / QPD_MAX_ORB, i = x - v * QPD_MAX_ORB;
                    int sp = v == 0 ? B.rs : B.cs;
                    int nvs = sp == 0 ? nv0 : nv1;
                    if (i >= nvs) continue;
                    int p = s_virt[sp][i];
                    int par;
                    double gv = s_F[sp][p];
                    if (B.type == BT_SINGLE) {
                        par = (s_cnt[sp][B.h1] + s_cnt[sp][p] - (B.h1 < p)) & 1;
                        gv -= a.I.Jm[B.h1 * n + p] - a.I.Km[B.h1 * n + p];
                    } else if (B.type == BT_SS) {
                        par = (s_cnt[sp][p] - (B.h1 < p) - (B.h2 < p)) & 1;
                        gv -= a.I.Jm[B.h1 * n + p] - a.I.Km[B.h1 * n + p];
                        gv -= a.I.Jm[B.h2 * n + p] - a.I.Km[B.h2 * n + p];
                    } else {
                        int hs = sp == 0 ? B.h1 : B.h2;   // same-spin hole
                        int ho = sp == 0 ? B.h2 : B.h1;   // opposite-spin hole
                        par = (s_cnt[sp][p] - (hs < p)) & 1;
                        gv -= a.I.Jm[hs * n + p] - a.I.Km[hs * n + p];
                        gv -= a.I.Jm[ho * n + p];
                    }
                    s_sg[v][i] = (uint8_t)par;
                    s_G[v][i] = gv;
                }
                if (BWD && B.type == BT_SINGLE)
                    for (int x = tid; x < n; x += QPD_WG) s_dhrow[x] = 0.0;
            }
            if (want_sel && tid == 0) s_tau_key = bin_edge(__atomic_load_n(a.tau_bin, __ATOMIC_RELAXED));
            wg_barrier();

            const int rvs = B.rs, cvs = B.cs;
            const uint8_t *rvirt = s_virt[rvs];
            const uint8_t *cvirt = s_virt[cvs];

            // particle orbitals (spin, orbital) of cell c
            auto particles = [&](int64_t c, int &pa, int &sa, int &pb, int &sb, int &ra, int &rb) {
                if (B.type == BT_SINGLE) {
                    ra = (int)c; rb = -1;
                    pa = rvirt[ra]; sa = rvs; pb = -1; sb = -1;
                } else if (B.type == BT_SS) {
                    int i1, i2;
                    tri_decode(c, i1, i2);
                    ra = i1; rb = i2;
                    pa = rvirt[i1]; pb = rvirt[i2]; sa = rvs; sb = rvs;
                } else {
                    int r = (int)(c / B.nc);
                    int col = (int)(c - (int64_t)r * B.nc);
                    ra = r; rb = col;
                    pa = rvirt[r]; sa = rvs; pb = cvirt[col]; sb = cvs;
                }
            };
            // alpha bits of cell c
            auto alpha_bits = [&](int pa, int sa, int pb, int sb, uint64_t *al) {
#pragma unroll
                for (int w = 0; w < 2 * NINT; ++w) al[w] = s_I[w];
                al[B.s1 * NINT + (B.h1 >> 6)] ^= 1ull << (B.h1 & 63);
                if (B.type != BT_SINGLE) al[B.s2 * NINT + (B.h2 >> 6)] ^= 1ull << (B.h2 & 63);
                al[sa * NINT + (pa >> 6)] ^= 1ull << (pa & 63);
                if (pb >= 0) al[sb * NINT + (pb >> 6)] ^= 1ull << (pb & 63);
            };

            // ---------------------------------------------- fine-filter round
            // wave 0 fills s_fine with up to FCAP entries of the coarse list
            // starting at s_fpos that pass m <= 2 for this hole set.
            auto fine_round = [&](int64_t start) {
                if (wave == 0) {
                    int nf = 0;
                    int64_t pos = start;
                    while (pos < cend && nf < FCAP) {
                        int64_t e = pos + lane;
                        int keep = 0, m = 0;
                        CoarseEnt ce;
                        if (e < cend) {
                            ce = a.cent[e];
                            int dcount = 0, inH = 0;
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                uint16_t d = ce.D[q];
                                if (d == 0xFFFF) continue;
                                dcount++;
                                int ds = d >> 8, dp = d & 255;
                                if (ds == B.s1 && dp == B.h1) inH++;
                                else if (B.type != BT_SINGLE && ds == B.s2 && dp == B.h2) inH++;
                            }
                            m = dcount - inH;
                            keep = m <= 2;
                        }
                        uint64_t mask = __ballot(keep);
                        int before = __popcll(mask & ((1ull << lane) - 1ull));
                        int tot = __popcll(mask);
                        // take entries only while they fit
                        int take = (nf + tot <= FCAP) ? tot : (FCAP - nf);
                        // last lane index consumed
                        int64_t consumed = 64;
                        if (take < tot) {
                            // find lane of the (take)-th kept entry: consume up to it
                            uint64_t mm = mask;
                            for (int q = 0; q < take; ++q) mm &= mm - 1;
                            consumed = ctz64(mm);
                        }
                        if (keep && before < take) {
                            FineEnt f;
                            f.j = ce.j; f.m = m; f.earlier = ce.flags & 1;
#pragma unroll
                            for (int q = 0; q < 4; ++q) f.E[q] = ce.E[q];
                            s_fine[nf + before] = f;
#pragma unroll
                            for (int k = 0; k < NS; ++k) s_fc[nf + before][k] = a.coefs[(int64_t)k * a.n_det + ce.j];
                        }
                        nf += take;
                        pos += consumed < 64 ? consumed : 64;
                        if (pos > cend) pos = cend;
                    }
                    if (lane == 0) { s_nfine = nf; s_fpos = pos; }
                }
            };

            // enumerate touched cells of fine entry f in [lo, hi) with all threads
            // and call fn(c) for each
            auto for_touched = [&](const FineEnt &f, int64_t lo, int64_t hi, auto &&fn) {
                int er[4], ec[4], ner = 0, nec = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    uint16_t e = f.E[q];
                    if (e == 0xFFFF) continue;
                    int es = e >> 8, ep = e & 255;
                    int vi = s_vidx[es][ep];
                    if (ep >= n || vi >= (es == 0 ? nv0 : nv1)) continue;   // not a particle of I
                    if (es == rvs) er[ner++] = vi;
                    else if (B.type == BT_OS && es == cvs) ec[nec++] = vi;
                }
                bool all = (f.m == 0) || (B.type == BT_SINGLE && f.m == 1);
                if (all) {
                    for (int64_t c = lo + tid; c < hi; c += QPD_WG) fn(c);
                    return;
                }
                if (f.m == 2) {
                    // cells with P subset of E
                    int64_t list[6];
                    int nl = 0;
                    if (B.type == BT_SINGLE) {
                        for (int q = 0; q < ner; ++q) list[nl++] = er[q];
                    } else if (B.type == BT_SS) {
                        for (int q = 0; q < ner; ++q)
                            for (int r = q + 1; r < ner; ++r) {
                                int x = er[q] < er[r] ? er[q] : er[r], y = er[q] < er[r] ? er[r] : er[q];
                                list[nl++] = (int64_t)y * (y - 1) / 2 + x;
                            }
                    } else {
                        for (int q = 0; q < ner; ++q)
                            for (int r = 0; r < nec; ++r) list[nl++] = (int64_t)er[q] * B.nc + ec[r];
                    }
                    for (int q = tid; q < nl; q += QPD_WG)
                        if (list[q] >= lo && list[q] < hi) fn(list[q]);
                    return;
                }
                // m == 1
                if (B.type == BT_OS) {
                    int64_t nrow = (int64_t)ner * B.nc, tot = nrow + (int64_t)nec * B.nr;
                    for (int64_t t = tid; t < tot; t += QPD_WG) {
                        int64_t c;
                        if (t < nrow) {
                            int q = (int)(t / B.nc);
                            c = (int64_t)er[q] * B.nc + (t - (int64_t)q * B.nc);
                        } else {
                            int64_t u = t - nrow;
                            int q = (int)(u / B.nr);
                            int r = (int)(u - (int64_t)q * B.nr);
                            bool dup = false;
                            for (int z = 0; z < ner; ++z) dup |= (er[z] == r);
                            if (dup) continue;
                            c = (int64_t)r * B.nc + ec[q];
                        }
                        if (c >= lo && c < hi) fn(c);
                    }
                } else {  // BT_SS
                    int V = B.nr;
                    int64_t tot = (int64_t)ner * (V - 1);
                    for (int64_t t = tid; t < tot; t += QPD_WG) {
                        int q = (int)(t / (V - 1));
                        int x = (int)(t - (int64_t)q * (V - 1));
                        if (x >= er[q]) x++;
                        bool dup = false;
                        for (int z = 0; z < q; ++z) dup |= (er[z] == x);
                        if (dup) continue;
                        int i1 = x < er[q] ? x : er[q], i2 = x < er[q] ? er[q] : x;
                        int64_t c = (int64_t)i2 * (i2 - 1) / 2 + i1;
                        if (c >= lo && c < hi) fn(c);
                    }
                }
            };

            // does this batch have any fine entry?
            fine_round(cbeg);
            wg_barrier();
            const bool has_tile = BWD ? true : (s_nfine > 0);
            const bool any_fine = s_nfine > 0;

            for (int64_t lo = 0; lo < B.ncell; lo += SLAB) {
                const int64_t hi = (lo + SLAB < B.ncell) ? lo + SLAB : B.ncell;
                const int sn = (int)(hi - lo);
                if (has_tile) {
                    for (int x = tid; x < NS * SLAB; x += QPD_WG) s_tile[x] = 0.0;
                    for (int x = tid; x < (SLAB + 31) / 32; x += QPD_WG) s_ban[x] = 0u;
                    if (lo > 0 && any_fine) {  // refill the first fine round for this slab
                        wg_barrier();
                        fine_round(cbeg);
                    }
                    wg_barrier();
                    if (any_fine) {
                        for (;;) {
                            const int nf = s_nfine;
                            for (int fi = 0; fi < nf; ++fi) {
                                const FineEnt f = s_fine[fi];
                                uint64_t Jb[2 * NINT];
#pragma unroll
                                for (int w = 0; w < 2 * NINT; ++w) Jb[w] = a.dets[(int64_t)f.j * 2 * NINT + w];
                                for_touched(f, lo, hi, [&](int64_t c) {
                                    int loc = (int)(c - lo);
                                    if (f.earlier) { atomicOr(&s_ban[loc >> 5], 1u << (loc & 31)); return; }
                                    int pa, sa, pb, sb, ra, rb;
                                    particles(c, pa, sa, pb, sb, ra, rb);
                                    uint64_t al[2 * NINT];
                                    alpha_bits(pa, sa, pb, sb, al);
                                    int deg;
                                    double v = sc_offdiag<NINT>(a.I, al, Jb, &deg, nullptr);
                                    if (deg == 0) { atomicOr(&s_ban[loc >> 5], 1u << (loc & 31)); return; }
                                    conn++;
#pragma unroll
                                    for (int k = 0; k < NS; ++k) s_tile[k * SLAB + loc] += s_fc[fi][k] * v;
                                });
                                wg_barrier();
                            }
                            if (s_fpos >= cend) break;
                            wg_barrier();
                            fine_round(s_fpos);
                            wg_barrier();
                        }
                    }
                }

                // ------------------------------------------------ cell pass
                const int iters = (sn + QPD_WG - 1) / QPD_WG;
                for (int it = 0; it < iters; ++it) {
                    const int loc = it * QPD_WG + tid;
                    const bool active = loc < sn;
                    const int64_t c = lo + loc;
                    double Hval = 0.0, D = 0.0;
                    int pa = -1, pb = -1, sa = 0, sb = 0, ra = 0, rb = 0;
                    bool banned = false;
                    if (active) {
                        particles(c, pa, sa, pb, sb, ra, rb);
                        if (B.type == BT_SINGLE) {
                            double f = fock_offdiag<NINT>(a.I, s_I, B.s1, B.h1, pa);
                            Hval = s_sg[0][ra] ? -f : f;
                            D = B.D0 + s_G[0][ra];
                        } else if (B.type == BT_SS) {
                            double x = B.blk[qtris(pa, pb)];
                            Hval = (B.sH ^ s_sg[0][ra] ^ s_sg[0][rb]) ? -x : x;
                            D = B.D0 + s_G[0][ra] + s_G[0][rb] + a.I.Jm[pa * n + pb] - a.I.Km[pa * n + pb];
                        } else {
                            double x = B.blk[(int64_t)pa * n + pb];
                            Hval = (B.sH ^ s_sg[0][ra] ^ s_sg[1][rb]) ? -x : x;
                            D = B.D0 + s_G[0][ra] + s_G[1][rb] + a.I.Jm[pa * n + pb];
                        }
                        if (has_tile) banned = (s_ban[loc >> 5] >> (loc & 31)) & 1u;
                    }
                    const bool live = active && !banned;
                    double ek[NS];
                    double tsel = 0.0;
                    double vsum = 0.0;
#pragma unroll
                    for (int k = 0; k < NS; ++k) {
                        double A = cI[k] * Hval + (has_tile && active ? s_tile[k * SLAB + loc] : 0.0);
                        double delta = E0[k] - D;
                        double r = 1.0 / delta;
                        double e = (A * A) * r;
                        ek[k] = e;
                        if (live) {
                            esum[k] += e;
                            ssum[k] += e * r;
                            double ad = fabs(delta);
                            mind = ad < mind ? ad : mind;
                            tsel += e * a.inv_maxc2[k];
                            if (BWD) {
                                double w = 2.0 * gup[k] * A * r;
                                dcI[k] += w * Hval;
                                vsum += gup[k] * e * r;
                                s_tile[k * SLAB + loc] = w;    // w_k for the sparse-J pass
                            }
                        }
                    }
                    if (BWD && active) {
                        s_vt[loc] = live ? vsum : 0.0;
                        if (!live) {
#pragma unroll
                            for (int k = 0; k < NS; ++k) s_tile[k * SLAB + loc] = 0.0;
                        }
                        if (B.type == BT_SINGLE && live) {
                            double gsum = 0.0;
#pragma unroll
                            for (int k = 0; k < NS; ++k) gsum += s_tile[k * SLAB + loc] * cI[k];
                            // d<I|H|alpha>/dh_{h p} = phase
                            s_dhrow[pa] += 0.5 * (s_sg[0][ra] ? -gsum : gsum);
                        }
                    }
                    if (live) {
                        cnt++;
                        if (want_fp) {
                            uint64_t al[2 * NINT];
                            alpha_bits(pa, sa, pb, sb, al);
                            fpsum += det_fold<NINT>(al);
                        }
                    }
                    if (want_sel) {
                        uint64_t key = 0;
                        bool cand = false;
                        if (live && fabs(tsel) >= __longlong_as_double(s_tau_key) * (1.0 - 1e-12)) {
                            double t = 0.0;
#pragma unroll
                            for (int k = 0; k < NS; ++k) t += ek[k] / a.maxc2[k];
                            key = (uint64_t)__double_as_longlong(fabs(t));
                            cand = key >= s_tau_key;
                        }
                        uint64_t mask = __ballot(cand);
                        if (mask) {
                            unsigned long long base = 0;
                            int tot = __popcll(mask);
                            if (lane == ctz64(mask)) base = atomicAdd(a.cand_count, (unsigned long long)tot);
                            base = __shfl(base, ctz64(mask));
                            if (cand) {
                                unsigned long long slotc = base + __popcll(mask & ((1ull << lane) - 1ull));
                                atomicAdd(&a.hist[key_bin(key)], 1u);
                                if ((int64_t)slotc < a.cand_cap) {
                                    Cand cd;
                                    cd.key = key;
                                    int up = B.type == BT_OS ? (sa == 0 ? pa : pb) : pa;
                                    int dn = B.type == BT_OS ? (sa == 0 ? pb : pa) : pb;
                                    cd.code = pack_code(B.type, B.s1, B.h1, B.h2 < 0 ? 0 : B.h2, up, dn < 0 ? 0 : dn);
                                    cd.g = (uint32_t)g;
                                    cd.pad = 0;
#pragma unroll
                                    for (int k = 0; k < QPD_MAX_STATES; ++k) cd.e[k] = k < NS ? ek[k] : 0.0;
                                    a.cand[slotc] = cd;
                                } else {
                                    atomicOr(a.overflow, 1ull);
                                }
                            }
                            if (lane == ctz64(mask)) s_appended = 1;
                        }
                    }
                }

                if (BWD) {
                    wg_barrier();
                    // ------------------------------------ dh diagonal: particles
                    // sum of v over the slab's cells per particle orbital; one
                    // thread per row / column, so no two threads share an address
                    if (B.type == BT_SINGLE) {
                        for (int loc = tid; loc < sn; loc += QPD_WG) {
                            s_dhd[rvirt[lo + loc]] += s_vt[loc];
                            vtot += s_vt[loc];
                        }
                        wg_barrier();
                    } else if (B.type == BT_OS) {
                        int r0 = (int)(lo / B.nc), r1 = (int)((hi - 1) / B.nc);
                        for (int r = r0 + tid; r <= r1; r += QPD_WG) {
                            double sr = 0.0;
                            for (int col = 0; col < B.nc; ++col) {
                                int64_t c = (int64_t)r * B.nc + col;
                                if (c >= lo && c < hi) sr += s_vt[c - lo];
                            }
                            s_dhd[rvirt[r]] += sr;
                            vtot += sr;
                        }
                        wg_barrier();
                        for (int col = tid; col < B.nc; col += QPD_WG) {
                            double sc = 0.0;
                            for (int r = r0; r <= r1; ++r) {
                                int64_t c = (int64_t)r * B.nc + col;
                                if (c >= lo && c < hi) sc += s_vt[c - lo];
                            }
                            s_dhd[cvirt[col]] += sc;
                        }
                        wg_barrier();
                    } else {
                        int j0, j1, k0, k1;
                        tri_decode(lo, j0, k0);
                        tri_decode(hi - 1, j1, k1);
                        // rows i2 in [k0, k1]: cells (i1 < i2)
                        for (int i2 = k0 + tid; i2 <= k1; i2 += QPD_WG) {
                            double sr = 0.0;
                            for (int i1 = 0; i1 < i2; ++i1) {
                                int64_t c = (int64_t)i2 * (i2 - 1) / 2 + i1;
                                if (c >= lo && c < hi) sr += s_vt[c - lo];
                            }
                            s_dhd[rvirt[i2]] += sr;
                            vtot += sr;
                        }
                        wg_barrier();
                        for (int i1 = tid; i1 < B.nr; i1 += QPD_WG) {
                            double sc = 0.0;
                            for (int i2 = (i1 + 1 > k0 ? i1 + 1 : k0); i2 <= k1; ++i2) {
                                int64_t c = (int64_t)i2 * (i2 - 1) / 2 + i1;
                                if (c >= lo && c < hi) sc += s_vt[c - lo];
                            }
                            s_dhd[rvirt[i1]] += sc;
                        }
                        wg_barrier();
                    }
                    // holes: n_p(I - H) = n_p(I) - [p in H]; subtract the slab total
                    {
                        double vs = 0.0;
                        for (int loc = tid; loc < sn; loc += QPD_WG) vs += s_vt[loc];
                        for (int off = 32; off > 0; off >>= 1) vs += __shfl_xor(vs, off);
                        if (lane == 0) s_red[wave][0] = vs;
                        wg_barrier();
                        if (tid == 0) {
                            double t = 0.0;
                            for (int q = 0; q < NWAVE; ++q) t += s_red[q][0];
                            s_dhd[B.h1] -= t;
                            if (B.type != BT_SINGLE) s_dhd[B.h2] -= t;
                        }
                        wg_barrier();
                    }
                    // ------------------------------- sparse J: dc_J and dh
                    if (any_fine) {
                        fine_round(cbeg);
                        wg_barrier();
                        for (;;) {
                            const int nf = s_nfine;
                            for (int fi = 0; fi < nf; ++fi) {
                                const FineEnt f = s_fine[fi];
                                if (f.earlier) continue;
                                uint64_t Jb[2 * NINT];
#pragma unroll
                                for (int w = 0; w < 2 * NINT; ++w) Jb[w] = a.dets[(int64_t)f.j * 2 * NINT + w];
                                double acc[NS];
#pragma unroll
                                for (int k = 0; k < NS; ++k) acc[k] = 0.0;
                                for_touched(f, lo, hi, [&](int64_t c) {
                                    int loc = (int)(c - lo);
                                    if ((s_ban[loc >> 5] >> (loc & 31)) & 1u) return;
                                    int pa, sa, pb, sb, ra, rb;
                                    particles(c, pa, sa, pb, sb, ra, rb);
                                    uint64_t al[2 * NINT];
                                    alpha_bits(pa, sa, pb, sb, al);
                                    int deg, sgl[4];
                                    double v = sc_offdiag<NINT>(a.I, al, Jb, &deg, sgl);
                                    if (deg == 0) return;
                                    double gsum = 0.0;
#pragma unroll
                                    for (int k = 0; k < NS; ++k) {
                                        double w = s_tile[k * SLAB + loc];
                                        acc[k] += w * v;
                                        gsum += w * s_fc[fi][k];
                                    }
                                    if (deg == 1 && a.dh) {
                                        double gg = 0.5 * gsum * sgl[3];
                                        atomicAdd(&a.dh[(int64_t)sgl[0] * n + sgl[1]], gg);
                                        atomicAdd(&a.dh[(int64_t)sgl[1] * n + sgl[0]], gg);
                                    }
                                });
#pragma unroll
                                for (int k = 0; k < NS; ++k) {
                                    double v = acc[k];
                                    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
                                    if (lane == 0 && v != 0.0 && a.dc) atomicAdd(&a.dc[(int64_t)k * a.n_det + f.j], v);
                                }
                            }
                            if (s_fpos >= cend) break;
                            wg_barrier();
                            fine_round(s_fpos);
                            wg_barrier();
                        }
                    }
                    wg_barrier();
                } else if (has_tile) {
                    wg_barrier();
                }
            }  // slab

            if (BWD && B.type == BT_SINGLE) {
                wg_barrier();
                if (a.dh)
                    for (int x = tid; x < n; x += QPD_WG) {
                        double v = s_dhrow[x];
                        if (v != 0.0) {
                            atomicAdd(&a.dh[(int64_t)B.h1 * n + x], v);
                            atomicAdd(&a.dh[(int64_t)x * n + B.h1], v);
                        }
                    }
            }
            // raise the global selection threshold from the candidate histogram
            if (want_sel) {
                wg_barrier();
                if (s_appended && wave == 0) {
                    uint32_t loc[QP_HIST_BINS / 64];
                    uint64_t tot = 0;
#pragma unroll
                    for (int q = 0; q < QP_HIST_BINS / 64; ++q) {
                        loc[q] = __atomic_load_n(&a.hist[lane * (QP_HIST_BINS / 64) + q], __ATOMIC_RELAXED);
                        tot += loc[q];
                    }
                    // sum over lanes above this one
                    uint64_t above = 0;
                    for (int q = 1; q < 64; ++q) {
                        uint64_t v = __shfl(tot, (lane + q) & 63);
                        if (lane + q < 64) above += v;
                    }
                    int best = -1;
                    uint64_t cum = above;
                    for (int q = QP_HIST_BINS / 64 - 1; q >= 0; --q) {
                        cum += loc[q];
                        if (cum >= (uint64_t)a.n_select) { best = lane * (QP_HIST_BINS / 64) + q; break; }
                    }
                    for (int off = 32; off > 0; off >>= 1) {
                        int o = __shfl_xor(best, off);
                        best = o > best ? o : best;
                    }
                    if (lane == 0 && best > 0) atomicMax(a.tau_bin, best);
                }
                if (tid == 0) s_appended = 0;
            }
            wg_barrier();
        }  // batch

        // ------------------------------------------------ item reduction
        {
            double vals[2 * NS + 1];
#pragma unroll
            for (int k = 0; k < NS; ++k) { vals[k] = esum[k]; vals[NS + k] = BWD ? dcI[k] : ssum[k]; }
            vals[2 * NS] = mind;
            double sS[NS];
#pragma unroll
            for (int k = 0; k < NS; ++k) sS[k] = ssum[k];
#pragma unroll
            for (int q = 0; q < 2 * NS; ++q)
                for (int off = 32; off > 0; off >>= 1) vals[q] += __shfl_xor(vals[q], off);
            for (int off = 32; off > 0; off >>= 1) {
                double o = __shfl_xor(vals[2 * NS], off);
                vals[2 * NS] = o < vals[2 * NS] ? o : vals[2 * NS];
            }
            uint64_t cc = cnt, ff = fpsum, cn = conn;
            for (int off = 32; off > 0; off >>= 1) {
                cc += __shfl_xor(cc, off);
                ff += __shfl_xor(ff, off);
                cn += __shfl_xor(cn, off);
            }
            double vt = vtot;
            for (int off = 32; off > 0; off >>= 1) vt += __shfl_xor(vt, off);
            if (BWD) {
#pragma unroll
                for (int k = 0; k < NS; ++k)
                    for (int off = 32; off > 0; off >>= 1) sS[k] += __shfl_xor(sS[k], off);
            }
            if (lane == 0) {
#pragma unroll
                for (int q = 0; q < 2 * NS + 1; ++q) s_red[wave][q] = vals[q];
                s_red[wave][2 * NS + 1] = vt;
                s_redu[wave][0] = cc; s_redu[wave][1] = ff; s_redu[wave][2] = cn;
            }
            wg_barrier();
            if (tid == 0) {
                double out[2 * NS + 2];
#pragma unroll
                for (int q = 0; q < 2 * NS + 2; ++q) out[q] = s_red[0][q];
                uint64_t oc = s_redu[0][0], of = s_redu[0][1], on = s_redu[0][2];
                for (int w = 1; w < NWAVE; ++w) {
#pragma unroll
                    for (int q = 0; q < 2 * NS; ++q) out[q] += s_red[w][q];
                    out[2 * NS] = s_red[w][2 * NS] < out[2 * NS] ? s_red[w][2 * NS] : out[2 * NS];
                    out[2 * NS + 1] += s_red[w][2 * NS + 1];
                    oc += s_redu[w][0]; of += s_redu[w][1]; on += s_redu[w][2];
                }
#pragma unroll
                for (int k = 0; k < NS; ++k) {
                    a.eps_item[slot * NS + k] = out[k];
                    if (BWD) a.dc_item[slot * NS + k] = out[NS + k];
                    else a.S_item[slot * NS + k] = out[NS + k];
                }
                a.cnt_item[slot] = (uint32_t)oc;
                if (a.fp_item) a.fp_item[slot] = of;
                if (on) atomicAdd(a.conn_total, (unsigned long long)on);
                unsigned long long mb = (unsigned long long)__double_as_longlong(out[2 * NS]);
                atomicMin(a.min_delta_bits, mb);
                s_vtot = out[2 * NS + 1];
            }
            if (BWD) {
                // S per item for the E0 gradient (reduce the saved ssum)
                wg_barrier();
                if (lane == 0) {
#pragma unroll
                    for (int k = 0; k < NS; ++k) s_red[wave][k] = sS[k];
                }
                wg_barrier();
                if (tid == 0) {
#pragma unroll
                    for (int k = 0; k < NS; ++k) {
                        double t = 0.0;
                        for (int w = 0; w < NWAVE; ++w) t += s_red[w][k];
                        a.S_item[slot * NS + k] = t;
                    }
                }
                wg_barrier();
            }
        }
        if (BWD) {
            // n_p(I) part of the diagonal gradient, then flush the item's
            // per-orbital accumulator
            wg_barrier();
            if (a.dh)
                for (int x = tid; x < n; x += QPD_WG) {
                    int np = (int)((s_I[x >> 6] >> (x & 63)) & 1ull) + (int)((s_I[NINT + (x >> 6)] >> (x & 63)) & 1ull);
                    double v = s_dhd[x] + np * s_vtot;
                    if (v != 0.0) atomicAdd(&a.dh[(int64_t)x * n + x], v);
                }
        }
        wg_barrier();
    }
}

template <int NINT, int NS, bool BWD>
void launch_sweep(const SweepArgs &a, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((sweep_kernel<NINT, NS, BWD>), dim3(grid), dim3(QPD_WG), 0, st, a);
}

#define QP_INST(NI, NS)                                                        \
    template void launch_sweep<NI, NS, false>(const SweepArgs &, int, hipStream_t); \
    template void launch_sweep<NI, NS, true>(const SweepArgs &, int, hipStream_t);
QP_INST(1, 1) QP_INST(1, 2) QP_INST(1, 3) QP_INST(1, 4)
QP_INST(2, 1) QP_INST(2, 2) QP_INST(2, 3) QP_INST(2, 4)
QP_INST(3, 1) QP_INST(3, 2) QP_INST(3, 3) QP_INST(3, 4)
QP_INST(4, 1) QP_INST(4, 2) QP_INST(4, 3) QP_INST(4, 4)
