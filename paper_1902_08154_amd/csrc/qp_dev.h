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
//   Cj[j][p][q] = (pq|jj),  Xj[j][p][q] = (pj|jq)     n^3 each
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
    const double *Xj;
    const double *Jm;
    const double *Km;
    const double *JK;  // Jm - Km: same-spin pair interaction
};

__device__ __forceinline__ int64_t qtri(int64_t a, int64_t b) { return b * (b + 1) / 2 + a; }
__device__ __forceinline__ int64_t qtris(int64_t a, int64_t b) { return b * (b - 1) / 2 + a; }

// chemist (pq|rs) through the X layout
__device__ __forceinline__ double eri_x(const DevInts &I, int p, int q, int r, int s)
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

// parity of the number of set bits of one spin string strictly between x and y
template <int NINT>
__device__ __forceinline__ int between_parity(const uint64_t *s, int x, int y)
{
    int lo = x < y ? x : y, hi = x < y ? y : x;
    int c = 0;
#pragma unroll
    for (int w = 0; w < NINT; ++w) c += popc64(s[w] & between_mask(w, lo, hi));
    return c & 1;
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
template <int NINT>
__device__ double fock_offdiag(const DevInts &I, const uint64_t *J, int s, int p, int q)
{
    const int64_t n = I.n;
    double v = I.h[p * n + q];
    const int64_t pq = (int64_t)p * n + q;
#pragma unroll
    for (int ss = 0; ss < 2; ++ss) {
#pragma unroll
        for (int w = 0; w < NINT; ++w) {
            uint64_t x = J[ss * NINT + w];
            while (x) {
                int j = 64 * w + ctz64(x);
                x &= x - 1;
                v += I.Cj[(int64_t)j * n * n + pq];
                if (ss == s) v -= I.Xj[(int64_t)j * n * n + pq];
            }
        }
    }
    return v;
}

// Generic Slater-Condon element <bra|H|ket> for 1 <= degree <= 2 (returns 0
// otherwise).  Phase: product of single-excitation phases, the second one on
// the intermediate determinant (same spin) or per spin (opposite spins).
// When sgl is non-null and the pair is a single excitation, writes
// {hole, particle, spin, sign} (hole in ket, particle in bra).
template <int NINT>
__device__ double sc_offdiag(const DevInts &I, const uint64_t *bra, const uint64_t *ket,
                             int *deg_out, int *sgl)
{
    int dsp[2];
    int deg = 0;
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        int c = 0;
#pragma unroll
        for (int w = 0; w < NINT; ++w) c += popc64(bra[s * NINT + w] ^ ket[s * NINT + w]);
        dsp[s] = c >> 1;
        deg += c >> 1;
    }
    if (deg_out) *deg_out = deg;
    if (deg == 0 || deg > 2) return 0.0;
    // holes (in ket) and particles (in bra), per spin, ascending
    int hl[2][2], pt[2][2], nh[2] = {0, 0}, np[2] = {0, 0};
#pragma unroll
    for (int s = 0; s < 2; ++s) {
#pragma unroll
        for (int w = 0; w < NINT; ++w) {
            uint64_t x = bra[s * NINT + w] ^ ket[s * NINT + w];
            uint64_t hh = x & ket[s * NINT + w], pp = x & bra[s * NINT + w];
            while (hh) { if (nh[s] < 2) hl[s][nh[s]] = 64 * w + ctz64(hh); nh[s]++; hh &= hh - 1; }
            while (pp) { if (np[s] < 2) pt[s][np[s]] = 64 * w + ctz64(pp); np[s]++; pp &= pp - 1; }
        }
    }
    if (deg == 1) {
        int s = dsp[0] == 1 ? 0 : 1;
        int h = hl[s][0], p = pt[s][0];
        int sg = between_parity<NINT>(ket + s * NINT, h, p);
        double v = fock_offdiag<NINT>(I, ket, s, h, p);
        if (sgl) { sgl[0] = h; sgl[1] = p; sgl[2] = s; sgl[3] = sg ? -1 : 1; }
        return sg ? -v : v;
    }
    if (sgl) sgl[0] = -1;
    if (dsp[0] == 1) {
        // opposite spins
        int sg = between_parity<NINT>(ket, hl[0][0], pt[0][0]) ^
                 between_parity<NINT>(ket + NINT, hl[1][0], pt[1][0]);
        double v = eri_x(I, hl[0][0], pt[0][0], hl[1][0], pt[1][0]);
        return sg ? -v : v;
    }
    int s = dsp[0] == 2 ? 0 : 1;
    int h1 = hl[s][0], h2 = hl[s][1], p1 = pt[s][0], p2 = pt[s][1];
    uint64_t mid[QPD_MAX_NINT];
#pragma unroll
    for (int w = 0; w < NINT; ++w) mid[w] = ket[s * NINT + w];
    int sg = between_parity<NINT>(mid, h1, p1);
    mid[h1 >> 6] ^= 1ull << (h1 & 63);
    mid[p1 >> 6] ^= 1ull << (p1 & 63);
    sg ^= between_parity<NINT>(mid, h2, p2);
    double v = eri_x(I, h1, p1, h2, p2) - eri_x(I, h1, p2, h2, p1);
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
    int64_t n_items;
    int q_per_gen;            // work items per generator
    unsigned int *item_counter;
    // fast kernel: buffer capacities and the deferred-batch list
    int rscap, cscap;
    int def_mode;             // general kernel: items are the deferred batches
    uint32_t *def_g, *def_b;  // deferred (generator rank, batch)
    int *def_next;            // per-generator linked list of deferred batches
    int *def_head;            // [n_det], -1 terminated
    unsigned long long *def_count;
    int64_t def_cap;
    int flags;                // bit0 fingerprint, bit1 backward
    // per-item partials (deterministic reduction later)
    double *eps_item;         // [n_items][ns]
    double *S_item;           // [n_items][ns]
    uint32_t *cnt_item;       // [n_items]
    uint64_t *fp_item;        // [n_items]
    uint64_t *conn_total;     // atomic
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
};

template <int NINT, int NS, bool BWD>
void launch_sweep(const SweepArgs &a, int grid, hipStream_t st);
template <int NINT, int NS, bool BWD>
int sweep_occupancy(int n);
template <int NINT, int NS, bool BWD>
void launch_fast(const SweepArgs &a, int grid, hipStream_t st);
template <int NINT, int NS, bool BWD>
int fast_occupancy(int n, int rscap, int cscap);
