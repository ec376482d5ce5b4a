// qp_dev.h -- internal device-side definitions of the gfx950 EN-PT2 sweep.
//
// Data layouts the context builds from the caller's packed integrals
// (sec. "Storage of the two-electron integrals"; Algorithm 1 gives the packed
// order).  They trade HBM capacity for gather-free, coalesced reads in the
// sweep: every (generator, hole-set) batch reads one contiguous block.
//
//   X [tri(a,b)][c][d] = (ac|bd),  a <= b            n(n+1)/2 x n x n
//       opposite-spin double I -> alpha with holes (a,b), particles (c,d)
//       reads X[tri(a,b)] row-major (c,d): one coalesced n x n block.
//   Y [tris(a,b)][tris(c,d)] = (ac|bd) - (ad|bc), a<b, c<d
//       same-spin double with holes a<b, particles c<d: one coalesced
//       antisymmetrised block per hole pair.            (n(n-1)/2)^2
//   Cj[j][p][q] = (pq|jj),  CXj[j][p][q] = (pq|jj) - (pj|jq)     n^3 each
//       Coulomb/exchange slices for Fock elements F^J_pq of any determinant.
//   Jm[p][q] = (pp|qq),  Km[p][q] = (pq|qp),  JK = Jm - Km   n^2 each
//   tri(a,b) = b(b+1)/2 + a (a<=b),  tris(a,b) = b(b-1)/2 + a (a<b)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define QPD_MAX_ORB 256
#define QPD_MAX_NINT 4
#define QPD_MAX_STATES 4
#define QPD_WG 256

struct DevInts {
    int n;
    const double *h;   // [n][n]
    const double *X;
    const double *Y;
    const double *Cj;
    const double *CXj;
    const double *Jm;
    const double *Km;
    const double *JK;  // Jm - Km: same-spin pair interaction
};

__device__ __forceinline__ int64_t qtri(int64_t a, int64_t b) { return b * (b + 1) / 2 + a; }
__device__ __forceinline__ int64_t qtris(int64_t a, int64_t b) { return b * (b - 1) / 2 + a; }

// chemist (pq|rs) through the X layout.  The integral helpers take the
// DevInts by a deduced type, so that a DevInts read through the constant
// address space binds without a copy.
template <class Ints>
__device__ __forceinline__ double eri_x(const Ints &I, int p, int q, int r, int s)
{
    const int64_t n = I.n;
    if (p <= r) return I.X[(qtri(p, r) * n + q) * n + s];
    return I.X[(qtri(r, p) * n + s) * n + q];
}

// ---------------------------------------------------------------------------
// bit strings: uint64 w[2*NINT]: up words then down words
// ---------------------------------------------------------------------------

__device__ __forceinline__ int popc64(uint64_t x) { return __popcll(x); }
__device__ __forceinline__ int ctz64(uint64_t x) { return __ffsll((unsigned long long)x) - 1; }

// mask of bits strictly between lo and hi (lo < hi) inside word w
__device__ __forceinline__ uint64_t between_mask(int w, int lo, int hi)
{
    int a = lo + 1 - 64 * w;   // first bit (inclusive)
    int b = hi - 1 - 64 * w;   // last bit (inclusive)
    if (a < 0) a = 0;
    if (b > 63) b = 63;
    if (a > b) return 0ull;
    uint64_t up = (b == 63) ? ~0ull : ((1ull << (b + 1)) - 1ull);
    return up & (~0ull << a);
}

// Private arrays are indexed only by compile-time constants here (loops are
// unrolled and runtime choices are selects): a runtime index would place the
// array in scratch memory.

// word q of spin s of a bit string
template <int NINT>
__device__ __forceinline__ uint64_t spin_word(const uint64_t *d, int s, int q)
{
    uint64_t r = 0;
#pragma unroll
    for (int w = 0; w < NINT; ++w)
        if (w == q) r = s ? d[NINT + w] : d[w];
    return r;
}

// occupation of spin-orbital (s, p)
template <int NINT>
__device__ __forceinline__ int occ_bit(const uint64_t *d, int s, int p)
{
    return (int)((spin_word<NINT>(d, s, p >> 6) >> (p & 63)) & 1ull);
}

// parity of the number of set bits of spin s of d strictly between x and y
template <int NINT>
__device__ __forceinline__ int between_parity(const uint64_t *d, int s, int x, int y)
{
    const int lo = x < y ? x : y, hi = x < y ? y : x;
    int c = 0;
#pragma unroll
    for (int w = 0; w < NINT; ++w) c += popc64((s ? d[NINT + w] : d[w]) & between_mask(w, lo, hi));
    return c & 1;
}

// word w of alpha = I - holes + particles; each hole or particle is given as
// (spin, orbital); hc = spin << 8 | orbital, -1 when absent, pb < 0 when absent
template <int NINT>
__device__ __forceinline__ uint64_t alpha_word(const uint64_t *Ib, int w, int hc0, int hc1, int pa, int sa, int pb,
                                               int sb)
{
    uint64_t x = Ib[w];
    const int base = 64 * (w % NINT), sp = w / NINT;
    auto tog = [&](int s_, int p_) {
        if (s_ == sp && p_ - base >= 0 && p_ - base < 64) x ^= 1ull << (p_ - base);
    };
    tog(hc0 >> 8, hc0 & 255);
    if (hc1 >= 0) tog(hc1 >> 8, hc1 & 255);
    tog(sa, pa);
    if (pb >= 0) tog(sb, pb);
    return x;
}

// splitmix64 output function (Steele, Lea & Flood 2014)
__device__ __forceinline__ uint64_t qp_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

template <int NINT>
__device__ __forceinline__ uint64_t det_fold(const uint64_t *d)
{
    uint64_t hsh = 0;
#pragma unroll
    for (int i = 0; i < 2 * NINT; ++i) hsh = qp_mix64(hsh ^ d[i]);
    return hsh;
}

// F^J_{pq} for spin s: h_pq + sum_{j in J} (pq|jj) - sum_{j in J_s} (pj|jq)
template <int NINT, class Ints>
__device__ double fock_offdiag(const Ints &I, const uint64_t *J, int s, int p, int q)
{
    const int64_t n = I.n;
    double v = I.h[p * n + q];
    const int64_t pq = (int64_t)p * n + q;
#pragma unroll
    for (int ss = 0; ss < 2; ++ss) {
        // an electron of the excited spin adds Coulomb minus exchange, one
        // of the other spin Coulomb alone: one integral read per electron
        const double *A = ss == s ? I.CXj : I.Cj;
#pragma unroll
        for (int w = 0; w < NINT; ++w) {
            uint64_t x = J[ss * NINT + w];
            // four electrons per step, their reads issued together; a step
            // past the last electron rereads the first one and adds nothing
            while (x) {
                const int j0 = ctz64(x);
                x &= x - 1;
                const bool m1 = x != 0;
                const int j1 = m1 ? ctz64(x) : j0;
                x &= x - 1;
                const bool m2 = x != 0;
                const int j2 = m2 ? ctz64(x) : j0;
                x &= x - 1;
                const bool m3 = x != 0;
                const int j3 = m3 ? ctz64(x) : j0;
                x &= x - 1;
                const int64_t b = (int64_t)64 * w * n * n + pq;
                const double a0 = A[b + (int64_t)j0 * n * n], a1 = A[b + (int64_t)j1 * n * n];
                const double a2 = A[b + (int64_t)j2 * n * n], a3 = A[b + (int64_t)j3 * n * n];
                v += a0;
                if (m1) v += a1;
                if (m2) v += a2;
                if (m3) v += a3;
            }
        }
    }
    return v;
}

// merge the two lowest set bits of m (bit positions offset by base) into the
// ascending pair (a, b), -1 marking an empty place; value selects only
__device__ __forceinline__ void low2_merge(uint64_t m, int base, int &a, int &b)
{
    const int x1 = m ? base + ctz64(m) : -1;
    const uint64_t m2 = m & (m - 1);
    const int x2 = m2 ? base + ctz64(m2) : -1;
    const bool na = a < 0;
    const int nb = na ? x2 : (b < 0 ? x1 : b);
    a = na ? x1 : a;
    b = nb;
}

// Generic Slater-Condon element <bra|H|ket> for 1 <= degree <= 2 (returns 0
// otherwise).  Phase: product of single-excitation phases, the second one on
// the intermediate determinant (same spin) or per spin (opposite spins).
// When sgl is non-null and the pair is a single excitation, writes
// {hole, particle, spin, sign} (hole in ket, particle in bra).
template <int NINT, class Ints>
__device__ double sc_offdiag(const Ints &I, const uint64_t *bra, const uint64_t *ket,
                             int *deg_out, int *sgl)
{
    int c0 = 0, c1 = 0;
#pragma unroll
    for (int w = 0; w < NINT; ++w) {
        c0 += popc64(bra[w] ^ ket[w]);
        c1 += popc64(bra[NINT + w] ^ ket[NINT + w]);
    }
    const int d0 = c0 >> 1, d1 = c1 >> 1, deg = d0 + d1;
    if (deg_out) *deg_out = deg;
    if (deg == 0 || deg > 2) return 0.0;
    // the (at most two) holes in ket and particles in bra of each spin, ascending
    int h0a = -1, h0b = -1, p0a = -1, p0b = -1, h1a = -1, h1b = -1, p1a = -1, p1b = -1;
#pragma unroll
    for (int w = 0; w < NINT; ++w) {
        const uint64_t x0 = bra[w] ^ ket[w], x1 = bra[NINT + w] ^ ket[NINT + w];
        low2_merge(x0 & ket[w], 64 * w, h0a, h0b);
        low2_merge(x0 & bra[w], 64 * w, p0a, p0b);
        low2_merge(x1 & ket[NINT + w], 64 * w, h1a, h1b);
        low2_merge(x1 & bra[NINT + w], 64 * w, p1a, p1b);
    }
    if (deg == 1) {
        const int s = d0 == 1 ? 0 : 1;
        const int h = s ? h1a : h0a, p = s ? p1a : p0a;
        const int sg = between_parity<NINT>(ket, s, h, p);
        const double v = fock_offdiag<NINT>(I, ket, s, h, p);
        if (sgl) { sgl[0] = h; sgl[1] = p; sgl[2] = s; sgl[3] = sg ? -1 : 1; }
        return sg ? -v : v;
    }
    if (sgl) sgl[0] = -1;
    if (d0 == 1) {
        // opposite spins
        const int sg = between_parity<NINT>(ket, 0, h0a, p0a) ^ between_parity<NINT>(ket, 1, h1a, p1a);
        const double v = eri_x(I, h0a, p0a, h1a, p1a);
        return sg ? -v : v;
    }
    const int s = d0 == 2 ? 0 : 1;
    const int h1 = s ? h1a : h0a, h2 = s ? h1b : h0b, p1 = s ? p1a : p0a, p2 = s ? p1b : p0b;
    // second excitation acts on ket with h1 -> p1 applied: h1 leaves and p1
    // enters the range strictly between h2 and p2
    const int lo = h2 < p2 ? h2 : p2, hi = h2 < p2 ? p2 : h2;
    const int sg = between_parity<NINT>(ket, s, h1, p1) ^ between_parity<NINT>(ket, s, h2, p2) ^
                   (int)(lo < h1 && h1 < hi) ^ (int)(lo < p1 && p1 < hi);
    // (h1 p1|h2 p2) - (h1 p2|h2 p1) with h1 < h2 and p1 < p2: one read of the
    // antisymmetrised layout (the same difference, formed when it was built)
    const int64_t P2 = (int64_t)I.n * (I.n - 1) / 2;
    const double v = I.Y[qtris(h1, h2) * P2 + qtris(p1, p2)];
    return sg ? -v : v;
}

// ---------------------------------------------------------------------------
// shared structures between host launchers and kernels
// ---------------------------------------------------------------------------

// coarse-filter entry for one (generator I, internal J) pair, degree <= 4
struct CoarseEnt {
    int32_t j;       // determinant index
    int32_t flags;   // bit 0: J precedes I in generator order; bits 8..15: degree
    uint16_t D[4];   // I \ J  (spin << 8 | orbital), 0xFFFF padded
    uint16_t E[4];   // J \ I
};

// selection candidate
struct Cand {
    uint64_t key;    // IEEE bits of |sum_k e_k / max c_k^2|
    uint64_t code;   // type | h1 | h2 | p1 | p2 (see pack_code)
    uint32_t g;      // generator rank
    uint32_t pad;
    double e[QPD_MAX_STATES];
};

#define QP_HIST_BINS 2048
#define QP_HIST_BASE 14768   // (biased exponent of 2^-100) << 4

__device__ __forceinline__ int key_bin(uint64_t key)
{
    int64_t b = (int64_t)(key >> 48) - QP_HIST_BASE;
    return b < 0 ? 0 : (b >= QP_HIST_BINS ? QP_HIST_BINS - 1 : (int)b);
}
__device__ __forceinline__ uint64_t bin_edge(int b)
{
    return b <= 0 ? 0ull : ((uint64_t)(b + QP_HIST_BASE) << 48);
}

// batch types
#define BT_SINGLE 0
#define BT_SS 1
#define BT_OS 2

// code: bits 0..7 h1, 8..15 h2, 16..23 p1, 24..31 p2, 32..33 type, 34 spin
// (spin of a single or same-spin batch).  For OS: h1,p1 up; h2,p2 down.
__host__ __device__ __forceinline__ uint64_t pack_code(int type, int spin, int h1, int h2, int p1, int p2)
{
    return (uint64_t)(h1 & 255) | ((uint64_t)(h2 & 255) << 8) | ((uint64_t)(p1 & 255) << 16) |
           ((uint64_t)(p2 & 255) << 24) | ((uint64_t)type << 32) | ((uint64_t)spin << 34);
}

struct SweepArgs {
    DevInts I;
    int n, nup, ndn, ns, nel;
    int64_t n_det;
    const uint64_t *dets;     // [n_det][2][nint]
    const double *coefs;      // [ns][n_det]
    const double *E0;         // [ns]
    const int32_t *perm;      // rank -> det
    const double *F;          // [rank][2][n]
    const double *HII;        // [rank]
    const int64_t *coff;      // [n_det+1], by rank
    const CoarseEnt *cent;
    int64_t n_items;          // dense kernel: n_gen * q_per_gen; general kernel: listed batches
    int q_per_gen;            // work items per generator
    // the generators of the call: ranks 0..n_det-1 (gen_list null, n_gen = n_det)
    // or the ranks gen_list[0..n_gen-1]
    const int32_t *gen_list;
    int64_t n_gen;
    // dense kernel: buffer capacities; batches it hands over are marked in
    // def_bits (nbw words per generator rank, bit b = batch b)
    int rscap, cscap;
    uint32_t *def_bits;
    int nbw;
    // general kernel: its items are the marked batches, listed in (rank, batch) order
    int def_mode;
    const uint32_t *def_g, *def_b;
    int def_parts;            // items per listed batch (row parts)
    int flags;                // bit0 fingerprint, bit1 backward
    // per-item partials (deterministic reduction later)
    double *eps_item;         // [n_items][ns]
    double *S_item;           // [n_items][ns]
    uint32_t *cnt_item;       // [n_items]
    uint64_t *fp_item;        // [n_items]
    uint32_t *conn_item;      // [n_items]
    unsigned long long *min_delta_bits;
    // selection
    int64_t n_select;
    double maxc2[QPD_MAX_STATES];
    double inv_maxc2[QPD_MAX_STATES];
    Cand *cand;
    unsigned long long *cand_count;
    int64_t cand_cap;
    unsigned int *hist;       // [QP_HIST_BINS]
    int *tau_bin;
    unsigned long long *overflow;
    // backward
    const double *gup;        // [ns]
    double *dc_item;          // [n_items][ns]  generator's own dc share
    double *dc;               // [ns][n_det]    other J (atomics)
    double *dh;               // [n][n]         atomics
    // split sweep: the clean-cell kernel (qp_lean.hip) takes every cell of a
    // hole-pair batch that no other determinant touches; the dense kernel then
    // leaves those cells out (split = 1).  The clean-cell kernel's items are the
    // (hole pair, generator) batches in hole-pair order: kl_off[K] .. kl_off[K+1]
    // holds the call positions of the generators whose determinant has both
    // holes of pair K occupied, ascending.  Pair keys: K = a n + b for the
    // opposite-spin pair (a up, b down); K = n^2 + s n(n-1)/2 + tris(a, b) for
    // the same-spin pair a < b of spin s.
    int split;
    int n_pairs;              // hole pairs per generator: nel (nel - 1) / 2
    const int64_t *kl_off;    // [n_keys + 1]
    const int32_t *kl_pos;    // [n_gen * n_pairs]
    int n_keys;
    double *lean_eps;         // [n_gen][n_pairs][ns]  per-batch partial sums
    double *lean_S;           // [n_gen][n_pairs][ns]
    unsigned long long *lean_cnt;  // [n_gen] clean cells counted (atomics)
    unsigned long long *lean_fp;   // [n_gen] fingerprint sums (atomics)
    unsigned long long *lean_conn; // [n_gen] connections of flagged cells (atomics)
    double *lean_dc;          // [n_gen][n_pairs][ns]  adjoint: the generator's dc share per batch
    uint32_t *split_keep;     // [n_det][nbw]  split sweeps: pair batches the dense kernel keeps (bit nel + pair)
    unsigned long long *fine_total;   // fine-filter entries over the batches evaluated (atomics)
    unsigned long long *item_ctr;     // clean-cell launches: per group of waves, items claimed so far
                                      // (ITEM_CTR_STRIDE apart; zero at launch; the same for every system)
};

// counters of one clean-cell launch: one per group of waves (8: one per XCD),
// each on a 128-byte line of its own
constexpr int ITEM_CTR_GROUPS = 8;
constexpr int ITEM_CTR_STRIDE = 16;

// Split sweep: the cells of the hole-pair batch (holes hc0, hc1 as spin << 8 |
// orbital) of generator rank g that other determinants touch.  Of the
// generator's coarse list, the entries J with m = |(I - H) \ J| <= 2 touch
// the batch: m = 2 entries the cells whose particles are all in J \ I (their
// rows are flagged: opposite spins the row-spin particle, same spin the
// larger one), m = 1 entries every cell that has one of J's particles (its
// row and its column are flagged; same spin, both on each particle).  An m = 0
// entry touches every cell: then the function returns false and the batch is
// not split.  rowF and colF are 256-bit masks over virtual indices (row spin,
// column spin), zeroed by the caller; sVidx maps spin * n + orbital to the
// orbital's virtual index (0xFFFF when occupied).  One wave; the result is the
// same on every lane.
template <class Sys>
__device__ bool split_flags(const Sys &a, int64_t g, int n, int nup, int ndn, bool os, int rs, int hc0, int hc1,
                            const uint16_t *sVidx, uint32_t *rowF, uint32_t *colF, int lane)
{
    const int64_t cbeg = a.coff[g], cend = a.coff[g + 1];
    const int nv0 = n - nup, nv1 = n - ndn;
    bool m0 = false;
    for (int64_t base = cbeg; base < cend; base += 64) {
        const int64_t e = base + lane;
        int m = 3;
        CoarseEnt ce;
        if (e < cend) {
            ce = a.cent[e];
            int dc = 0, inmask = 0;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int d = ce.D[t];
                if (d == 0xFFFF) continue;
                dc++;
                inmask |= (d == hc0 ? 1 : 0) | (d == hc1 ? 2 : 0);
            }
            m = dc - __popc(inmask);
        }
        if (m > 2) continue;
        if (m == 0) { m0 = true; continue; }
        int ner = 0, nec = 0, er[4] = {0, 0, 0, 0}, ec[4] = {0, 0, 0, 0};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int ecode = ce.E[t];
            if (ecode == 0xFFFF) continue;
            const int es = ecode >> 8, ep = ecode & 255;
            if (ep >= n) continue;
            const int vi = sVidx[es * n + ep];
            if (vi >= (es == 0 ? nv0 : nv1)) continue;
            if (es == rs) {
#pragma unroll
                for (int q = 0; q < 4; ++q) if (q == ner) er[q] = vi;
                ner++;
            } else if (os) {
#pragma unroll
                for (int q = 0; q < 4; ++q) if (q == nec) ec[q] = vi;
                nec++;
            }
        }
        if (m == 2) {
            if (os) {
                if (nec > 0)
#pragma unroll
                    for (int q = 0; q < 4; ++q) if (q < ner) atomicOr(&rowF[er[q] >> 5], 1u << (er[q] & 31));
            } else {
#pragma unroll
                for (int q1 = 1; q1 < 4; ++q1)
#pragma unroll
                    for (int q0 = 0; q0 < 4; ++q0)
                        if (q0 < q1 && q1 < ner) {
                            const int r = er[q0] > er[q1] ? er[q0] : er[q1];
                            atomicOr(&rowF[r >> 5], 1u << (r & 31));
                        }
            }
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (q < ner) {
                    atomicOr(&rowF[er[q] >> 5], 1u << (er[q] & 31));
                    if (!os) atomicOr(&colF[er[q] >> 5], 1u << (er[q] & 31));
                }
                if (os && q < nec) atomicOr(&colF[ec[q] >> 5], 1u << (ec[q] & 31));
            }
        }
    }
    return __ballot(m0) == 0ull;
}

// The sweep kernels read each system's SweepArgs from a table in device
// memory through the constant address space: the table does not change during
// a launch, so the compiler may reload a field where it is used instead of
// holding it in a register, and it takes the pointers read from the table to
// be global memory (global, not flat, memory instructions).
typedef const __attribute__((address_space(4))) SweepArgs ConstSys;

template <int NINT, int NS, bool BWD>
void launch_sweep(const SweepArgs *sys, const int64_t *item_end, int n_sys, size_t lds, int grid, hipStream_t st);
template <int NINT, int NS, bool BWD>
int sweep_occupancy(size_t lds);
size_t sweep_lds_bytes(int n, int ns, bool bwd);
template <int NINT, int NS, bool BWD>
void launch_fast(const SweepArgs *sys, const int64_t *item_end, int n_sys, bool fp, size_t lds, int grid,
                 hipStream_t st);
template <int NINT, int NS, bool BWD>
int fast_occupancy(size_t lds, bool fp);
size_t fast_lds_bytes(int n, int nvm, int ns, bool bwd, int rscap, int cscap);
template <int NINT, int NS, bool BWD>
void launch_lean(const SweepArgs *sys, const int64_t *item_end, int n_sys, bool fp, size_t lds, int grid,
                 hipStream_t st);
template <int NINT, int NS, bool BWD>
int lean_occupancy(size_t lds, bool fp);
size_t lean_lds_bytes(int n, int nvm, bool bwd);
template <int NINT, int NS, bool BWD>
void launch_corr(const SweepArgs *sys, const int64_t *item_end, int n_sys, bool fp, size_t lds, int grid,
                 hipStream_t st);
template <int NINT, int NS, bool BWD>
int corr_occupancy(size_t lds, bool fp);
size_t corr_lds_bytes(int n, int ns, bool bwd);
// capacities of the dense kernel's per-batch correction buffers; the clean-cell
// kernel applies the same limits to decide which batches it takes
#define QPF_FCAP 32
#define QPF_L2CAP 64
#define QPF_PCAP 2
