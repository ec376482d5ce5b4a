// qp_core.hip -- integral layouts, generator ordering, per-generator
// preparation, coarse filter, deterministic reductions, final selection,
// variational energy, and the C ABI (include/qp_pt2.h).
#include "qp_dev.h"
#include "../../include/qp_pt2.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

// ===========================================================================
// integral layouts (from the packed array, offset tri(tri(p,q), tri(r,s)))
// ===========================================================================

__device__ __forceinline__ double packed_eri(const double *eri, int64_t p, int64_t q, int64_t r, int64_t s)
{
    int64_t a = p > q ? p * (p + 1) / 2 + q : q * (q + 1) / 2 + p;
    int64_t b = r > s ? r * (r + 1) / 2 + s : s * (s + 1) / 2 + r;
    int64_t o = a > b ? a * (a + 1) / 2 + b : b * (b + 1) / 2 + a;
    return eri[o];
}

// X[tri(a,b)][c][d] = (ac|bd), a <= b
__global__ void build_X(const double *eri, int n, double *X)
{
    const int64_t n2 = (int64_t)n * n;
    const int64_t total = (int64_t)n * (n + 1) / 2 * n2;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t t = i / n2, cd = i - t * n2;
        int b = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
        while ((int64_t)b * (b + 1) / 2 > t) --b;
        while ((int64_t)(b + 1) * (b + 2) / 2 <= t) ++b;
        int a = (int)(t - (int64_t)b * (b + 1) / 2);
        int c = (int)(cd / n), d = (int)(cd - (int64_t)c * n);
        X[i] = packed_eri(eri, a, c, b, d);
    }
}

// Y[tris(a,b)][tris(c,d)] = (ac|bd) - (ad|bc), a < b, c < d
__global__ void build_Y(const double *eri, int n, double *Y)
{
    const int64_t P2 = (int64_t)n * (n - 1) / 2;
    const int64_t total = P2 * P2;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t t = i / P2, u = i - t * P2;
        int b = (int)((1.0 + sqrt(8.0 * (double)t + 1.0)) * 0.5);
        while ((int64_t)b * (b - 1) / 2 > t) --b;
        while ((int64_t)(b + 1) * b / 2 <= t) ++b;
        int a = (int)(t - (int64_t)b * (b - 1) / 2);
        int d = (int)((1.0 + sqrt(8.0 * (double)u + 1.0)) * 0.5);
        while ((int64_t)d * (d - 1) / 2 > u) --d;
        while ((int64_t)(d + 1) * d / 2 <= u) ++d;
        int c = (int)(u - (int64_t)d * (d - 1) / 2);
        Y[i] = packed_eri(eri, a, c, b, d) - packed_eri(eri, a, d, b, c);
    }
}

// Cj[j][p][q] = (pq|jj), CXj[j][p][q] = (pq|jj) - (pj|jq), Jm[p][q] = (pp|qq), Km[p][q] = (pq|qp)
__global__ void build_small(const double *eri, const double *h, int n, double *Cj, double *CXj,
                            double *Jm, double *Km, double *JK, double *hc)
{
    const int64_t n3 = (int64_t)n * n * n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n3;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t j = i / ((int64_t)n * n), pq = i - j * n * n;
        int64_t p = pq / n, q = pq - p * n;
        Cj[i] = packed_eri(eri, p, q, j, j);
        CXj[i] = Cj[i] - packed_eri(eri, p, j, j, q);
        if (j == 0) {
            Jm[pq] = packed_eri(eri, p, p, q, q);
            Km[pq] = packed_eri(eri, p, q, q, p);
            JK[pq] = Jm[pq] - Km[pq];
            hc[pq] = h[pq];
        }
    }
}

// ===========================================================================
// small helpers
// ===========================================================================

template <int NINT>
__device__ __forceinline__ int det_cmp_dev(const uint64_t *a, const uint64_t *b)
{
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int w = NINT - 1; w >= 0; --w) {
            uint64_t x = a[s * NINT + w], y = b[s * NINT + w];
            if (x != y) return x < y ? -1 : 1;
        }
    return 0;
}

// key_bin on the host (the same bins as the kernels' histogram)
inline int key_bin_host(uint64_t key)
{
    const int64_t b = (int64_t)(key >> 48) - QP_HIST_BASE;
    return b < 0 ? 0 : (b >= QP_HIST_BINS ? QP_HIST_BINS - 1 : (int)b);
}

struct Scalars {
    unsigned int pad0;
    int tau_bin;
    unsigned long long cand_count;
    unsigned long long overflow;
    unsigned long long min_delta_bits;
    unsigned long long coarse_total;
    unsigned long long comp_count;
    long long pad1;
    unsigned long long fine_total;    // fine-filter entries of the batches evaluated
    unsigned long long clean_total;   // alpha of the clean-cell kernel
    int bad_bits;     // a bit set at >= n_orb
    int bad_elec;     // electron counts differ from det 0
    int dup;          // duplicate determinant
    int bad_gen;      // a listed generator index outside [0, n_det)
};

// the per-sweep fields of the scalars, as a fresh preparation leaves them; the
// fields that describe the inputs (coarse-list size, input checks) are kept
__global__ void reset_sweep_scalars(Scalars *sc, int tau_bin0)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc->tau_bin = tau_bin0;
        sc->cand_count = 0ull;
        sc->overflow = 0ull;
        sc->min_delta_bits = 0x7ff0000000000000ull;
        sc->comp_count = 0ull;
        sc->fine_total = 0ull;
        sc->clean_total = 0ull;
        sc->bad_gen = 0;
    }
}

__global__ void fill_ones(double *x, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = 1.0;
}

// generator weight w_J = sum_k c_Jk^2 ; inverse max c^2 per state
__global__ void gen_weights(const double *coefs, int64_t n_det, int ns, double *w, int64_t P, int32_t *idx)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
        if (i < n_det) {
            double s = 0.0;
            for (int k = 0; k < ns; ++k) { double c = coefs[k * n_det + i]; s += c * c; }
            w[i] = s;
            idx[i] = (int32_t)i;
        } else {
            idx[i] = -1;
        }
    }
}

__global__ void max_c2(const double *coefs, int64_t n_det, int ns, double *out /* [ns] */)
{
    __shared__ double red[256];
    for (int k = 0; k < ns; ++k) {
        double m = 0.0;
        for (int64_t i = threadIdx.x; i < n_det; i += blockDim.x) {
            double c = coefs[k * n_det + i];
            m = fmax(m, c * c);
        }
        red[threadIdx.x] = m;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
            __syncthreads();
        }
        if (threadIdx.x == 0) out[k] = red[0];
        __syncthreads();
    }
}

// ---------------------------------------------------------------- bitonic sort
template <int NINT>
struct GenCmp {
    const double *w;
    const uint64_t *dets;
    __device__ bool before(int a, int b) const
    {
        if (a < 0) return false;
        if (b < 0) return true;
        if (w[a] != w[b]) return w[a] > w[b];
        return det_cmp_dev<NINT>(dets + (int64_t)a * 2 * NINT, dets + (int64_t)b * 2 * NINT) < 0;
    }
};

template <int NINT>
struct SelCmp {
    const uint64_t *key;
    const uint64_t *bits;
    __device__ bool before(int a, int b) const
    {
        if (a < 0) return false;
        if (b < 0) return true;
        if (key[a] != key[b]) return key[a] > key[b];
        return det_cmp_dev<NINT>(bits + (int64_t)a * 2 * NINT, bits + (int64_t)b * 2 * NINT) < 0;
    }
};

template <class Cmp>
__global__ void bitonic_step(int32_t *idx, int64_t P, int64_t j, int64_t k, Cmp cmp)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= P) return;
    int64_t l = i ^ j;
    if (l > i) {
        int32_t x = idx[i], y = idx[l];
        bool up = (i & k) == 0;
        bool sw = up ? cmp.before(y, x) : cmp.before(x, y);
        if (sw) { idx[i] = y; idx[l] = x; }
    }
}

// in-LDS stages for j < 1024 (block of 512 threads handles 1024 elements)
template <class Cmp>
__global__ void bitonic_local(int32_t *idx, int64_t P, int64_t k, int64_t jstart, Cmp cmp)
{
    __shared__ int32_t s[1024];
    int64_t base = (int64_t)blockIdx.x * 1024;
    for (int t = threadIdx.x; t < 1024; t += blockDim.x) s[t] = base + t < P ? idx[base + t] : -1;
    __syncthreads();
    for (int64_t j = jstart; j > 0; j >>= 1) {
        for (int t = threadIdx.x; t < 1024; t += blockDim.x) {
            int l = t ^ (int)j;
            if (l > t) {
                int64_t gi = base + t;
                int32_t x = s[t], y = s[l];
                bool up = (gi & k) == 0;
                bool sw = up ? cmp.before(y, x) : cmp.before(x, y);
                if (sw) { s[t] = y; s[l] = x; }
            }
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < 1024; t += blockDim.x) if (base + t < P) idx[base + t] = s[t];
}

template <class Cmp>
static void bitonic_sort(int32_t *idx, int64_t P, Cmp cmp, hipStream_t st)
{
    // P is a power of two >= 1
    const int tb = 256;
    const int64_t blocks = (P + tb - 1) / tb;
    for (int64_t k = 2; k <= P; k <<= 1) {
        int64_t j = k >> 1;
        for (; j >= 1024; j >>= 1)
            hipLaunchKernelGGL(bitonic_step<Cmp>, dim3((unsigned)blocks), dim3(tb), 0, st, idx, P, j, k, cmp);
        if (j > 0) {
            int64_t nb = (P + 1023) / 1024;
            hipLaunchKernelGGL(bitonic_local<Cmp>, dim3((unsigned)nb), dim3(512), 0, st, idx, P, k, j, cmp);
        }
    }
}

// ---------------------------------------------------------------- rank
__global__ void make_rank(const int32_t *perm, int64_t n_det, int32_t *rank)
{
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n_det; g += (int64_t)gridDim.x * blockDim.x)
        rank[perm[g]] = (int32_t)g;
}

// ranks of a list of generators given by determinant index
__global__ void map_gen_ranks(const int32_t *gens, int64_t n_gen, const int32_t *rank, int64_t n_det,
                              int32_t *out, Scalars *sc)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_gen; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t d = gens[i];
        if (d < 0 || d >= n_det) {
            sc->bad_gen = 1;
            out[i] = 0;
        } else {
            out[i] = rank[d];
        }
    }
}

// ---------------------------------------------------------------- per-generator prep
// F[g][s][x] = h_xx + sum_{j in I} (xx|jj) - sum_{j in I_s} (xj|jx); H_II;
// validation of electron counts and stray bits.
template <int NINT>
__global__ void prep_generators(const uint64_t *dets, const int32_t *perm, int64_t n_det, int n,
                                const double *h, const double *Jm, const double *Km, double *F, double *HII,
                                Scalars *sc)
{
    __shared__ uint8_t occ[2][QPD_MAX_ORB];
    __shared__ int no[2];
    __shared__ double red[128];
    const int64_t g = blockIdx.x;
    if (g >= n_det) return;
    const int det = perm[g];
    const uint64_t *I = dets + (int64_t)det * 2 * NINT;
    const uint64_t *I0 = dets;
    if (threadIdx.x < 2) {
        int s = threadIdx.x, c = 0, c0 = 0;
        bool bad = false;
        for (int w = 0; w < NINT; ++w) {
            uint64_t x = I[s * NINT + w];
            c += popc64(x);
            c0 += popc64(I0[s * NINT + w]);
            int lo = n - 64 * w;   // bits >= lo in this word are invalid
            if (lo <= 0) bad |= x != 0;
            else if (lo < 64) bad |= (x >> lo) != 0;
        }
        no[s] = c;
        if (c != c0) atomicOr(&sc->bad_elec, 1);
        if (bad) atomicOr(&sc->bad_bits, 1);
    }
    __syncthreads();
    for (int x = threadIdx.x; x < 2 * n; x += blockDim.x) {
        int s = x / n, p = x - s * n;
        const uint64_t *w = I + s * NINT;
        if ((w[p >> 6] >> (p & 63)) & 1ull) {
            int c = 0;
            for (int q = 0; q < NINT; ++q) {
                if (64 * q + 63 < p) c += popc64(w[q]);
                else if (64 * q <= p) c += popc64(w[q] & ((1ull << (p - 64 * q)) - 1ull));
            }
            occ[s][c] = (uint8_t)p;
        }
    }
    __syncthreads();
    double hpart = 0.0;
    for (int x = threadIdx.x; x < 2 * n; x += blockDim.x) {
        int s = x / n, p = x - s * n;
        double f = h[(int64_t)p * n + p];
        for (int t = 0; t < 2; ++t)
            for (int q = 0; q < no[t]; ++q) {
                int j = occ[t][q];
                f += Jm[(int64_t)p * n + j];
                if (t == s) f -= Km[(int64_t)p * n + j];
            }
        F[(g * 2 + s) * n + p] = f;
        const uint64_t *w = I + s * NINT;
        if ((w[p >> 6] >> (p & 63)) & 1ull) hpart += 0.5 * (h[(int64_t)p * n + p] + f);
    }
    red[threadIdx.x] = hpart;
    __syncthreads();
    for (int s = 64; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) HII[g] = red[0];
}

// ---------------------------------------------------------------- coarse filter
// grid (ceil(n_det/256), nchunk); thread = generator rank; J chunk staged in LDS
template <int NINT, bool FILL>
__global__ void coarse_kernel(const uint64_t *dets, const int32_t *perm, const int32_t *rank, int64_t n_det,
                              int64_t chunk, int nchunk, int32_t *counts, const int64_t *offs,
                              CoarseEnt *out, Scalars *sc)
{
    __shared__ uint64_t sJ[256][2 * NINT];
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int ch = blockIdx.y;
    const bool valid = g < n_det;
    uint64_t I[2 * NINT];
    int det = -1;
    if (valid) {
        det = perm[g];
#pragma unroll
        for (int w = 0; w < 2 * NINT; ++w) I[w] = dets[(int64_t)det * 2 * NINT + w];
    }
    const int64_t j0 = ch * chunk, j1 = (j0 + chunk < n_det) ? j0 + chunk : n_det;
    int c = 0;
    int64_t o = 0;
    if (FILL && valid) o = offs[g * nchunk + ch];
    for (int64_t t0 = j0; t0 < j1; t0 += 256) {
        __syncthreads();
        int64_t jj = t0 + threadIdx.x;
        if (jj < j1)
#pragma unroll
            for (int w = 0; w < 2 * NINT; ++w) sJ[threadIdx.x][w] = dets[jj * 2 * NINT + w];
        __syncthreads();
        if (!valid) continue;
        int lim = (int)((j1 - t0) < 256 ? (j1 - t0) : 256);
        for (int q = 0; q < lim; ++q) {
            int d = 0;
#pragma unroll
            for (int w = 0; w < 2 * NINT; ++w) d += popc64(I[w] ^ sJ[q][w]);
            d >>= 1;
            if (d > 4) continue;
            int64_t j = t0 + q;
            if (j == det) continue;
            if (d == 0) { if (!FILL) atomicOr(&sc->dup, 1); continue; }
            if (FILL) {
                CoarseEnt e;
                e.j = (int32_t)j;
                e.flags = (rank[j] < g ? 1 : 0) | (d << 8);
                int nd = 0, ne = 0;
#pragma unroll
                for (int q2 = 0; q2 < 4; ++q2) { e.D[q2] = 0xFFFF; e.E[q2] = 0xFFFF; }
#pragma unroll
                for (int s = 0; s < 2; ++s)
#pragma unroll
                    for (int w = 0; w < NINT; ++w) {
                        uint64_t x = I[s * NINT + w], y = sJ[q][s * NINT + w];
                        uint64_t dd = x & ~y, ee = y & ~x;
                        while (dd) { if (nd < 4) e.D[nd] = (uint16_t)((s << 8) | (64 * w + ctz64(dd))); nd++; dd &= dd - 1; }
                        while (ee) { if (ne < 4) e.E[ne] = (uint16_t)((s << 8) | (64 * w + ctz64(ee))); ne++; ee &= ee - 1; }
                    }
                out[o + c] = e;
            }
            c++;
        }
    }
    if (!FILL && valid) counts[g * nchunk + ch] = c;
}

// ---------------------------------------------------------------- exclusive scan (int32 -> int64)
__global__ void scan_block(const int32_t *in, int64_t n, int64_t *out, int64_t *bsum)
{
    __shared__ int64_t s[1024];
    int64_t base = (int64_t)blockIdx.x * 1024;
    for (int t = threadIdx.x; t < 1024; t += blockDim.x) s[t] = base + t < n ? in[base + t] : 0;
    __syncthreads();
    // Hillis-Steele inclusive scan
    for (int off = 1; off < 1024; off <<= 1) {
        int64_t v[4];
        int cntv = 0;
        for (int t = threadIdx.x; t < 1024; t += blockDim.x) v[cntv++] = t >= off ? s[t - off] : 0;
        __syncthreads();
        cntv = 0;
        for (int t = threadIdx.x; t < 1024; t += blockDim.x) s[t] += v[cntv++];
        __syncthreads();
    }
    for (int t = threadIdx.x; t < 1024; t += blockDim.x)
        if (base + t < n) out[base + t] = (t == 0 ? 0 : s[t - 1]);
    if (threadIdx.x == 0) bsum[blockIdx.x] = s[1023];
}

__global__ void scan_bsum(int64_t *bsum, int64_t nb, int64_t *total)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        int64_t run = 0;
        for (int64_t i = 0; i < nb; ++i) { int64_t v = bsum[i]; bsum[i] = run; run += v; }
        *total = run;
    }
}

__global__ void scan_add(int64_t *out, int64_t n, const int64_t *bsum)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] += bsum[i / 1024];
}

__global__ void make_coff(const int64_t *offs, int64_t n_det, int nchunk, const int64_t *total, int64_t *coff,
                          Scalars *sc)
{
    int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g < n_det) coff[g] = offs[g * nchunk];
    if (g == n_det) { coff[g] = *total; sc->coarse_total = (unsigned long long)*total; }
}

// ---------------------------------------------------------------- batch marks and fine counts
// One thread per generator of the call, over its coarse list.  An entry J
// lacking dc of the generator's electrons lacks m = dc - |holes of J among
// the batch's| electrons outside a batch's hole set.  The fine filter of a
// batch keeps the entries with m <= 2, so their number over every batch
// follows from dc alone: dc <= 2 reaches every batch; dc = 3 the 3 single
// batches of its holes and the pairs holding one of them; dc = 4 the 6 pairs
// inside its holes.  An entry with m = 0 (dc = 1: every pair holding its
// hole; dc = 2: the pair of its holes) touches every cell of a batch, which
// then stays with the dense kernel: split sweeps mark those pair batches,
// bit nel + pair of the generator rank's words (the dense kernel's batch
// numbering).
template <int NINT>
__global__ void split_mark(const uint64_t *dets, const int32_t *perm, const int32_t *gen_rank, int64_t n_gen,
                           int nup, int ndn, const int64_t *coff, const CoarseEnt *cent, int nbw, uint32_t *keep,
                           unsigned long long *fine_total)
{
    const int64_t pos = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int nel = nup + ndn;
    const int64_t np = (int64_t)nel * (nel - 1) / 2;
    const int64_t np3 = (int64_t)(nel - 3) * (nel - 4) / 2;   // pairs free of 3 given holes
    unsigned long long fine = 0;
    if (pos < n_gen) {
        const int64_t g = gen_rank ? (int64_t)gen_rank[pos] : pos;
        const uint64_t *I = dets + (int64_t)perm[g] * 2 * NINT;
        // hole index over the occupied orbitals, up spin first
        auto hidx = [&](int code) {
            const int s = code >> 8, p = code & 255;
            int c = s ? nup : 0;
            for (int w = 0; w < NINT; ++w) {
                const uint64_t x = I[s * NINT + w];
                if (64 * w + 64 <= p) c += __popcll(x);
                else if (64 * w <= p) c += __popcll(x & ((1ull << (p - 64 * w)) - 1ull));
            }
            return c;
        };
        auto mark = [&](int a, int b) {   // the pair of hole indices a < b
            const int bb = nel + b * (b - 1) / 2 + a;
            uint32_t *w = keep + g * nbw + (bb >> 5);
            *w |= 1u << (bb & 31);
        };
        for (int64_t e = coff[g]; e < coff[g + 1]; ++e) {
            const CoarseEnt ce = cent[e];
            int dc = 0;
            for (int t = 0; t < 4; ++t) dc += ce.D[t] != 0xFFFF ? 1 : 0;
            if (dc <= 2) fine += (unsigned long long)(nel + np);
            else if (dc == 3) fine += (unsigned long long)(3 + np - np3);
            else fine += 6ull;
            if (keep && dc == 1) {
                const int i = hidx(ce.D[0]);
                for (int j = 0; j < nel; ++j)
                    if (j != i) mark(i < j ? i : j, i < j ? j : i);
            } else if (keep && dc == 2) {
                const int i = hidx(ce.D[0]), j = hidx(ce.D[1]);
                mark(i < j ? i : j, i < j ? j : i);
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) fine += __shfl_xor(fine, o);
    if ((threadIdx.x & 63) == 0 && fine) atomicAdd(fine_total, fine);
}

// ---------------------------------------------------------------- hole-pair lists
// The clean-cell kernel's items in hole-pair-major order.  Occupation bitsets
// over the call's generators: bits[(s n + p) nw + w], bit i of word w set when
// the determinant of generator position 64 w + i has orbital p of spin s.
template <int NINT>
__global__ void pair_bits(const uint64_t *dets, const int32_t *perm, const int32_t *gen_list, int64_t n_gen, int n,
                          int64_t nw, uint64_t *bits)
{
    const int lane = threadIdx.x & 63;
    const int64_t w = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
    if (w >= nw) return;
    const int64_t i = w * 64 + lane;
    uint64_t d[2 * NINT];
#pragma unroll
    for (int q = 0; q < 2 * NINT; ++q) d[q] = 0;
    if (i < n_gen) {
        const int64_t gr = gen_list ? (int64_t)gen_list[i] : i;
        const int det = perm[gr];
#pragma unroll
        for (int q = 0; q < 2 * NINT; ++q) d[q] = dets[(int64_t)det * 2 * NINT + q];
    }
    for (int s = 0; s < 2; ++s)
        for (int p = 0; p < n; ++p) {
            const uint64_t m = __ballot(occ_bit<NINT>(d, s, p) != 0);
            if (lane == 0) bits[((int64_t)s * n + p) * nw + w] = m;
        }
}

// the two bitsets of pair key K (see SweepArgs): opposite spins K = a n + b,
// same spin K = n^2 + s n(n-1)/2 + tris(a, b)
__device__ __forceinline__ void pair_sets(int K, int n, int64_t nw, const uint64_t *bits, const uint64_t *&x,
                                          const uint64_t *&y)
{
    if (K < n * n) {
        const int a = K / n, b = K - a * n;
        x = bits + (int64_t)a * nw;
        y = bits + ((int64_t)n + b) * nw;
    } else {
        const int P2 = n * (n - 1) / 2;
        const int t = K - n * n, s = t >= P2 ? 1 : 0, u = t - s * P2;
        int b = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)u)) * 0.5f);
        while (b * (b - 1) / 2 > u) --b;
        while ((b + 1) * b / 2 <= u) ++b;
        const int a = u - b * (b - 1) / 2;
        x = bits + ((int64_t)s * n + a) * nw;
        y = bits + ((int64_t)s * n + b) * nw;
    }
}

// generators per pair key (one wave per key)
__global__ void pair_count(const uint64_t *bits, int n, int64_t nw, int n_keys, int32_t *counts)
{
    const int lane = threadIdx.x & 63;
    const int K = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (K >= n_keys) return;
    const uint64_t *x, *y;
    pair_sets(K, n, nw, bits, x, y);
    int c = 0;
    for (int64_t w = lane; w < nw; w += 64) c += __popcll(x[w] & y[w]);
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if (lane == 0) counts[K] = c;
}

// the generator positions of each key, ascending, at the scanned offsets; a
// write past `cap` (inconsistent electron counts under QP_FLAG_NOCHECK) is dropped
__global__ void pair_fill(const uint64_t *bits, int n, int64_t nw, int n_keys, const int64_t *off, int64_t cap,
                          int32_t *pos)
{
    const int lane = threadIdx.x & 63;
    const int K = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (K >= n_keys) return;
    const uint64_t *x, *y;
    pair_sets(K, n, nw, bits, x, y);
    int64_t o = off[K];
    for (int64_t w0 = 0; w0 < nw; w0 += 64) {
        const int64_t w = w0 + lane;
        uint64_t m = w < nw ? (x[w] & y[w]) : 0ull;
        int c = __popcll(m);
        // exclusive scan of the lanes' counts
        int incl = c;
        for (int d = 1; d < 64; d <<= 1) {
            const int v = __shfl_up(incl, d);
            if (lane >= d) incl += v;
        }
        int64_t at = o + (incl - c);
        while (m) {
            const int b = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            if (at < cap) pos[at] = (int32_t)(w * 64 + b);
            ++at;
        }
        o += __shfl(incl, 63);
    }
}

// per generator: the clean-cell kernel's batch slots, in batch order, after
// the dense kernel's items and the handed-over batches
__global__ void reduce_lean(const double *lean_eps, const double *lean_S, const unsigned long long *lean_cnt,
                            const unsigned long long *lean_fp, const unsigned long long *lean_conn,
                            const double *lean_dc, int64_t n_gen, int n_pairs, int ns, const int32_t *perm,
                            const int32_t *gen_rank, int64_t n_det, double *eps_g, double *S_g, uint64_t *cnt_g,
                            uint64_t *fp_g, uint64_t *conn_g, double *eps_gen, double *dc,
                            unsigned long long *clean_total)
{
    const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    {
        // the clean-cell kernel's alpha, summed over each wave first
        unsigned long long v = i0 < n_gen ? lean_cnt[i0] : 0ull;
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if ((threadIdx.x & 63) == 0 && v) atomicAdd(clean_total, v);
    }
    if (i0 >= n_gen) return;
    for (int k = 0; k < ns; ++k) {
        double e = eps_g[i0 * ns + k], sv = S_g[i0 * ns + k], d = 0.0;
        for (int b = 0; b < n_pairs; ++b) {
            e += lean_eps[(i0 * n_pairs + b) * ns + k];
            sv += lean_S[(i0 * n_pairs + b) * ns + k];
            if (lean_dc) d += lean_dc[(i0 * n_pairs + b) * ns + k];
        }
        eps_g[i0 * ns + k] = e;
        S_g[i0 * ns + k] = sv;
        // adjoint: the generator's own dE/dc from its split batches (the
        // general reduction has already added the rest)
        if (lean_dc && dc) dc[(int64_t)k * n_det + perm[gen_rank ? (int64_t)gen_rank[i0] : i0]] += d;
        if (eps_gen) {
            if (gen_rank) eps_gen[k * n_gen + i0] = e;
            else eps_gen[k * n_det + perm[i0]] = e;
        }
    }
    cnt_g[i0] += lean_cnt[i0];
    fp_g[i0] += lean_fp[i0];
    conn_g[i0] += lean_conn[i0];
}

// ---------------------------------------------------------------- reductions
// per generator: sum its items in order; eps_gen in the caller's index
// Deferred partials of one generator, in increasing batch order (its list is
// built by atomic pushes, so it is re-ordered here for a fixed summation order).
// Batches the dense kernel handed to the general kernel, listed in (rank,
// batch) order: generator g owns entries [off[g], off[g] + cnt[g]).
struct DefParts {
    const int64_t *off;
    const int32_t *cnt;
    int parts;                // slots per listed batch
    const double *eps, *S, *dc;
    const uint32_t *alpha, *conn;
    const uint64_t *fp;
};

// deferred batches per generator rank: popcount of its bitmap words
__global__ void def_count(const uint32_t *bits, int64_t n_det, int nbw, int32_t *cnt)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= n_det) return;
    int c = 0;
    for (int w = 0; w < nbw; ++w) c += __popc(bits[g * nbw + w]);
    cnt[g] = c;
}

// list them at the scanned offsets, batches in increasing order
__global__ void def_fill(const uint32_t *bits, int64_t n_det, int nbw, const int64_t *off, uint32_t *dg,
                         uint32_t *db)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= n_det) return;
    int64_t o = off[g];
    for (int w = 0; w < nbw; ++w) {
        uint32_t x = bits[g * nbw + w];
        while (x) {
            dg[o] = (uint32_t)g;
            db[o] = (uint32_t)(32 * w + __ffs(x) - 1);
            ++o;
            x &= x - 1;
        }
    }
}

// no batches at all (no electrons): every partial is zero
__global__ void reduce_empty(int64_t n_gen, int ns, const int32_t *perm, const int32_t *gen_rank, int64_t n_det,
                             double *eps_g, double *S_g, uint64_t *cnt_g, uint64_t *fp_g, uint64_t *conn_g,
                             uint64_t *defa_g, double *eps_gen)
{
    const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i0 >= n_gen) return;
    for (int k = 0; k < ns; ++k) {
        eps_g[i0 * ns + k] = 0.0;
        S_g[i0 * ns + k] = 0.0;
        if (eps_gen) {
            if (gen_rank) eps_gen[k * n_gen + i0] = 0.0;
            else eps_gen[k * n_det + perm[i0]] = 0.0;
        }
    }
    cnt_g[i0] = 0; fp_g[i0] = 0; conn_g[i0] = 0; defa_g[i0] = 0;
}

// per generator, in a fixed order: its dense-kernel items, then its deferred
// batches in batch order.  Generator i of the call is rank gen_rank[i] (or
// rank i when gen_rank is null); per-generator outputs go to position i, and
// eps_gen to [k][det] for a full sweep or [k][i] for a list.
__global__ void reduce_items(const double *eps_item, const double *S_item, const uint32_t *cnt_item,
                             const uint64_t *fp_item, const uint32_t *conn_item, const double *dc_item,
                             int64_t n_gen, int nq, int ns, const int32_t *perm, const int32_t *gen_rank,
                             int64_t n_det, double *eps_g, double *S_g, uint64_t *cnt_g, uint64_t *fp_g,
                             uint64_t *conn_g, uint64_t *defa_g, double *eps_gen, double *dc, DefParts dp)
{
    const int64_t i0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i0 >= n_gen) return;
    const int64_t g = gen_rank ? (int64_t)gen_rank[i0] : i0;
    const int det = perm[g];
    double e[QPD_MAX_STATES] = {0, 0, 0, 0}, s[QPD_MAX_STATES] = {0, 0, 0, 0}, d[QPD_MAX_STATES] = {0, 0, 0, 0};
    uint64_t c = 0, f = 0, cn = 0, cd = 0;
    for (int i = 0; i < nq; ++i) {
        const int64_t sl = i0 * nq + i;
        for (int k = 0; k < ns; ++k) {
            e[k] += eps_item[sl * ns + k];
            s[k] += S_item[sl * ns + k];
            if (dc_item) d[k] += dc_item[sl * ns + k];
        }
        c += cnt_item[sl];
        cn += conn_item[sl];
        if (fp_item) f += fp_item[sl];
    }
    const int64_t x0 = dp.off[g] * dp.parts, x1 = x0 + (int64_t)dp.cnt[g] * dp.parts;
    for (int64_t x = x0; x < x1; ++x) {
        for (int k = 0; k < ns; ++k) {
            e[k] += dp.eps[x * ns + k];
            s[k] += dp.S[x * ns + k];
            if (dc_item && dp.dc) d[k] += dp.dc[x * ns + k];
        }
        cd += dp.alpha[x];
        cn += dp.conn[x];
        if (fp_item && dp.fp) f += dp.fp[x];
    }
    c += cd;
    for (int k = 0; k < ns; ++k) {
        eps_g[i0 * ns + k] = e[k];
        S_g[i0 * ns + k] = s[k];
        if (eps_gen) {
            if (gen_rank) eps_gen[k * n_gen + i0] = e[k];
            else eps_gen[k * n_det + det] = e[k];
        }
        if (dc_item && dc) dc[k * n_det + det] += d[k];
    }
    conn_g[i0] = cn;
    defa_g[i0] = cd;
    cnt_g[i0] = c;
    fp_g[i0] = f;
}

// single block, fixed summation order
__global__ void reduce_total(const double *eps_g, const double *S_g, const uint64_t *cnt_g, const uint64_t *fp_g,
                             const uint64_t *conn_g, const uint64_t *defa_g, int64_t n_det, int ns, double *e_pt2,
                             qp_pt2_stats *stats, const Scalars *sc, int64_t n_cells, const double *gup,
                             double *grad_E0, const double *E0)
{
    __shared__ double se[256][QPD_MAX_STATES], ss[256][QPD_MAX_STATES];
    __shared__ uint64_t sc_[256], sf[256], sn[256], sd[256];
    const int t = threadIdx.x;
    double e[QPD_MAX_STATES] = {0, 0, 0, 0}, s[QPD_MAX_STATES] = {0, 0, 0, 0};
    uint64_t c = 0, f = 0, cn = 0, cd = 0;
    for (int64_t g = t; g < n_det; g += 256) {
        for (int k = 0; k < ns; ++k) { e[k] += eps_g[g * ns + k]; s[k] += S_g[g * ns + k]; }
        c += cnt_g[g];
        f += fp_g[g];
        cn += conn_g[g];
        cd += defa_g[g];
    }
    for (int k = 0; k < QPD_MAX_STATES; ++k) { se[t][k] = e[k]; ss[t][k] = s[k]; }
    sc_[t] = c; sf[t] = f; sn[t] = cn; sd[t] = cd;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (t < st) {
            for (int k = 0; k < QPD_MAX_STATES; ++k) { se[t][k] += se[t + st][k]; ss[t][k] += ss[t + st][k]; }
            sc_[t] += sc_[t + st];
            sf[t] += sf[t + st];
            sn[t] += sn[t + st];
            sd[t] += sd[t + st];
        }
        __syncthreads();
    }
    if (t == 0) {
        for (int k = 0; k < ns; ++k) {
            if (e_pt2) e_pt2[k] = se[0][k];
            if (grad_E0) grad_E0[k] = -gup[k] * ss[0][k];
        }
        if (stats) {
            stats->n_alpha = sc_[0];
            stats->n_cells = (uint64_t)n_cells;
            stats->fingerprint = sf[0];
            stats->n_coarse = sc->coarse_total;
            stats->n_candidates = sc->cand_count;
            stats->overflow = sc->overflow;
            stats->n_connections = sn[0];
            stats->n_alpha_general = sd[0];
            stats->n_fine = sc->fine_total;
            stats->n_alpha_clean = sc->clean_total;
            for (int k = 0; k < QPD_MAX_STATES; ++k) stats->S[k] = k < ns ? ss[0][k] : 0.0;
            stats->min_abs_delta = __longlong_as_double((long long)sc->min_delta_bits);
            // rPT2 (eq. Z): Z = 1 / (1 - dSigma/dE) with dSigma/dE = -S at E0
            for (int k = 0; k < QPD_MAX_STATES; ++k) {
                const double z = k < ns ? 1.0 / (1.0 + ss[0][k]) : 0.0;
                stats->Z[k] = z;
                stats->e_rpt2[k] = k < ns ? E0[k] + z * se[0][k] : 0.0;
            }
        }
    }
}

// ---------------------------------------------------------------- selection
__global__ void sel_compact(const Cand *cand, const Scalars *sc, int64_t cap, int32_t *comp, Scalars *scw)
{
    int64_t m = (int64_t)sc->cand_count;
    if (m > cap) m = cap;
    const uint64_t edge = bin_edge(sc->tau_bin);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        if (cand[i].key >= edge) {
            unsigned long long p = atomicAdd(&scw->comp_count, 1ull);
            comp[p] = (int32_t)i;
        }
}

template <int NINT>
__global__ void sel_materialise(const Cand *cand, const int32_t *comp, int64_t M, const uint64_t *dets,
                                const int32_t *perm, uint64_t *keys, uint64_t *bits, int64_t P, int32_t *idx)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < P; i += (int64_t)gridDim.x * blockDim.x) {
        if (i >= M) { idx[i] = -1; continue; }
        const Cand cd = cand[comp[i]];
        idx[i] = (int32_t)i;
        keys[i] = cd.key;
        const uint64_t *I = dets + (int64_t)perm[cd.g] * 2 * NINT;
        uint64_t al[2 * NINT];
#pragma unroll
        for (int w = 0; w < 2 * NINT; ++w) al[w] = I[w];
        int h1 = cd.code & 255, h2 = (cd.code >> 8) & 255, p1 = (cd.code >> 16) & 255, p2 = (cd.code >> 24) & 255;
        int type = (cd.code >> 32) & 3, spin = (cd.code >> 34) & 1;
        auto flip = [&](int s, int p) { al[s * NINT + (p >> 6)] ^= 1ull << (p & 63); };
        if (type == BT_SINGLE) { flip(spin, h1); flip(spin, p1); }
        else if (type == BT_SS) { flip(spin, h1); flip(spin, h2); flip(spin, p1); flip(spin, p2); }
        else { flip(0, h1); flip(1, h2); flip(0, p1); flip(1, p2); }
#pragma unroll
        for (int w = 0; w < 2 * NINT; ++w) bits[i * 2 * NINT + w] = al[w];
    }
}

template <int NINT>
__global__ void sel_output(const Cand *cand, const int32_t *comp, const int32_t *sorted, int64_t m, int ns,
                           const uint64_t *bits, const uint64_t *keys, uint64_t *sel_dets, double *sel_e,
                           uint64_t *sel_key, int64_t *n_sel)
{
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x) {
        int32_t i = sorted[r];
        const Cand cd = cand[comp[i]];
#pragma unroll
        for (int w = 0; w < 2 * NINT; ++w) sel_dets[r * 2 * NINT + w] = bits[(int64_t)i * 2 * NINT + w];
        for (int k = 0; k < ns; ++k) sel_e[r * ns + k] = cd.e[k];
        if (sel_key) sel_key[r] = keys[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *n_sel = m;
}

// ---------------------------------------------------------------- variational energy
template <int NINT>
__global__ void energy_rows(const DevInts I, const uint64_t *dets, const double *coefs, const int32_t *perm,
                            const double *HII, const int64_t *coff, const CoarseEnt *cent, int64_t n_det, int ns,
                            double *row /* [n_det][ns] */, double *c2 /* [n_det][ns] */)
{
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n_det; g += (int64_t)gridDim.x * blockDim.x) {
        const int det = perm[g];
        const uint64_t *Ib = dets + (int64_t)det * 2 * NINT;
        double acc[QPD_MAX_STATES];
        for (int k = 0; k < ns; ++k) {
            double c = coefs[k * n_det + det];
            acc[k] = HII[g] * c;
            c2[g * ns + k] = c * c;
        }
        for (int64_t e = coff[g]; e < coff[g + 1]; ++e) {
            const CoarseEnt ce = cent[e];
            if ((ce.flags >> 8) > 2) continue;
            int deg;
            double v = sc_offdiag<NINT>(I, Ib, dets + (int64_t)ce.j * 2 * NINT, &deg, nullptr);
            for (int k = 0; k < ns; ++k) acc[k] += v * coefs[k * n_det + ce.j];
        }
        for (int k = 0; k < ns; ++k) row[g * ns + k] = acc[k] * coefs[k * n_det + det];
    }
}

// ---------------------------------------------------------------- sigma
// W = H U or W = S^2 U over the determinant space of Psi (the sigma vectors
// of a Davidson iteration, sec. "Davidson diagonalization"), one thread per
// determinant, from its coarse list (every J != I with degree <= 4).
//
// number of occupied spin-orbitals before (s, p) in the canonical order: all
// up spin-orbitals, then all down ones, by increasing orbital
template <int NINT>
__device__ __forceinline__ int n_before(const uint64_t *d, int s, int p)
{
    int c = 0;
    if (s == 1)
        for (int w = 0; w < NINT; ++w) c += popc64(d[w]);
    const uint64_t *ds = d + s * NINT;
    for (int w = 0; w < NINT; ++w) {
        if (64 * w + 63 < p) c += popc64(ds[w]);
        else if (64 * w <= p) c += popc64(ds[w] & ((1ull << (p - 64 * w)) - 1ull));
    }
    return c;
}

// <J|S_- S_+|I> for J = I with the spins of orbitals p (down in I) and q (up
// in I) exchanged: the operator string a+(q,dn) a(q,up) a+(p,up) a(p,dn)
// applied to I, one operator at a time
template <int NINT>
__device__ __forceinline__ double spin_exchange(const uint64_t *Ib, int p, int q)
{
    uint64_t d[2 * NINT];
#pragma unroll
    for (int w = 0; w < 2 * NINT; ++w) d[w] = Ib[w];
    int sgn = 0;
    auto op = [&](int s, int o) {
        sgn += n_before<NINT>(d, s, o);
        d[s * NINT + (o >> 6)] ^= 1ull << (o & 63);
    };
    op(1, p);   // a(p, down)
    op(0, p);   // a+(p, up)
    op(0, q);   // a(q, up)
    op(1, q);   // a+(q, down)
    return (sgn & 1) ? -1.0 : 1.0;
}

template <int NINT, bool S2>
__global__ void sigma_rows(const DevInts I, const uint64_t *dets, const int32_t *perm, const double *HII,
                           const int64_t *coff, const CoarseEnt *cent, int64_t n_det, int n_vec, double sz,
                           const double *U, double *W)
{
    for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n_det; g += (int64_t)gridDim.x * blockDim.x) {
        const int det = perm[g];
        uint64_t Ib[2 * NINT];
#pragma unroll
        for (int w = 0; w < 2 * NINT; ++w) Ib[w] = dets[(int64_t)det * 2 * NINT + w];
        double diag;
        if (S2) {
            // S^2 = S_- S_+ + S_z (S_z + 1): S_- S_+ counts the down electrons
            // whose orbital has no up electron
            int nb = 0;
#pragma unroll
            for (int w = 0; w < NINT; ++w) nb += popc64(Ib[NINT + w] & ~Ib[w]);
            diag = sz * (sz + 1.0) + nb;
        } else {
            diag = HII[g];
        }
        for (int v0 = 0; v0 < n_vec; v0 += 4) {
            double acc[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[t] = v0 + t < n_vec ? diag * U[(int64_t)(v0 + t) * n_det + det] : 0.0;
            for (int64_t e = coff[g]; e < coff[g + 1]; ++e) {
                const CoarseEnt ce = cent[e];
                const int deg = ce.flags >> 8;
                double v;
                if (S2) {
                    // a spin exchange: I \ J = {q up, p down}, J \ I = {p up, q down}
                    if (deg != 2) continue;
                    int du = -1, dd = -1, eu = -1, ed = -1;
                    for (int t = 0; t < 2; ++t) {
                        const int x = ce.D[t], y = ce.E[t];
                        if (x >> 8) dd = x & 255; else du = x & 255;
                        if (y >> 8) ed = y & 255; else eu = y & 255;
                    }
                    if (du < 0 || dd < 0 || eu != dd || ed != du || du == dd) continue;
                    v = spin_exchange<NINT>(Ib, dd, du);
                } else {
                    if (deg > 2) continue;
                    int dg;
                    v = sc_offdiag<NINT>(I, Ib, dets + (int64_t)ce.j * 2 * NINT, &dg, nullptr);
                }
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (v0 + t < n_vec) acc[t] += v * U[(int64_t)(v0 + t) * n_det + ce.j];
            }
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (v0 + t < n_vec) W[(int64_t)(v0 + t) * n_det + det] = acc[t];
        }
    }
}

__global__ void energy_total(const double *row, const double *c2, int64_t n_det, int ns, double *E0)
{
    __shared__ double sn[256][QPD_MAX_STATES], sd[256][QPD_MAX_STATES];
    const int t = threadIdx.x;
    double a[QPD_MAX_STATES] = {0, 0, 0, 0}, b[QPD_MAX_STATES] = {0, 0, 0, 0};
    for (int64_t g = t; g < n_det; g += 256)
        for (int k = 0; k < ns; ++k) { a[k] += row[g * ns + k]; b[k] += c2[g * ns + k]; }
    for (int k = 0; k < QPD_MAX_STATES; ++k) { sn[t][k] = a[k]; sd[t][k] = b[k]; }
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (t < st)
            for (int k = 0; k < QPD_MAX_STATES; ++k) { sn[t][k] += sn[t + st][k]; sd[t][k] += sd[t + st][k]; }
        __syncthreads();
    }
    if (t == 0)
        for (int k = 0; k < ns; ++k) E0[k] = sn[0][k] / sd[0][k];
}

// ------------------------------------------------ Davidson vector algebra
// Vectors are rows of length N in device memory; a block of them is
// contiguous ([count][N]).  The subspace algebra of the Davidson method
// (Rayleigh matrix, Ritz vectors, residuals, Gram-Schmidt) is made of these
// few operations, so that only m x m matrices and norms cross to the host.

// part[c][a * nb + b] = sum over chunk c of A_a . B_b
__global__ void dav_dots_part(const double *A, int na, const double *B, int nb, int64_t N, int64_t chunk,
                              double *part)
{
    __shared__ double red[256];
    const int pair = blockIdx.x;
    const int a = pair / nb, b = pair - a * nb;
    const int64_t i0 = (int64_t)blockIdx.y * chunk;
    const int64_t i1 = i0 + chunk < N ? i0 + chunk : N;
    const double *x = A + (int64_t)a * N, *y = B + (int64_t)b * N;
    double s = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) s = fma(x[i], y[i], s);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(int64_t)blockIdx.y * na * nb + pair] = red[0];
}

// out[p] = sum over chunks, in chunk order (the result does not depend on timing)
__global__ void dav_dots_sum(const double *part, int npair, int nchunk, double *out)
{
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < npair; p += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int c = 0; c < nchunk; ++c) s += part[(int64_t)c * npair + p];
        out[p] = s;
    }
}

// Y_k = (acc ? Y_k : 0) + alpha sum_j coef[j][k] A_j, k < kk
__global__ void dav_gemv(const double *A, int m, int64_t N, const double *coef, int kk, double alpha, int acc,
                         double *Y)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        for (int k = 0; k < kk; ++k) {
            double v = 0.0;
            for (int j = 0; j < m; ++j) v = fma(coef[j * kk + k], A[(int64_t)j * N + i], v);
            Y[(int64_t)k * N + i] = acc ? fma(alpha, v, Y[(int64_t)k * N + i]) : alpha * v;
        }
}

// residuals R_k = (H X)_k - theta_k X_k
__global__ void dav_resid(const double *HX, const double *X, const double *theta, int kk, int64_t N, double *R)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        for (int k = 0; k < kk; ++k)
            R[(int64_t)k * N + i] = HX[(int64_t)k * N + i] - theta[k] * X[(int64_t)k * N + i];
}

// diagonal preconditioner: T = R / (theta - H_ii), the denominator kept away from 0
__global__ void dav_precond(const double *R, const double *diag, double theta, int64_t N, double *T)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        double d = theta - diag[i];
        if (fabs(d) < 1e-8) d = d < 0 ? -1e-8 : 1e-8;
        T[i] = R[i] / d;
    }
}

__global__ void dav_scale(double *x, int64_t N, double s)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        x[i] *= s;
}

// the diagonal of H by determinant index, from the values by generator rank
__global__ void dav_diag(const double *HII, const int32_t *perm, int64_t N, double *diag)
{
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < N; r += (int64_t)gridDim.x * blockDim.x)
        diag[perm[r]] = HII[r];
}

// ===========================================================================
// host side
// ===========================================================================

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

enum BufId {
    B_W, B_IDX, B_RANK, B_F, B_HII, B_COUNTS, B_OFFS, B_BSUM, B_COFF, B_CENT, B_EPSI, B_SI, B_CNTI, B_FPI,
    B_DCI, B_EPSG, B_SG, B_CNTG, B_FPG, B_SC, B_HIST, B_CAND, B_COMP, B_SKEY, B_SBITS, B_SIDX, B_MAXC2,
    B_ROW, B_C2, B_TOTAL, B_DEFG, B_DEFB, B_DEFE, B_DEFS, B_DEFC, B_DEFN, B_DEFF, B_DEFD, B_CONNI, B_CONNG,
    B_DEFAG, B_DEFBITS, B_DEFCG, B_DEFOFF, B_DEFBS, B_GENR,
    // semi-stochastic sweep: a round's selection
    B_RSDET, B_RSE, B_RSKEY, B_RSN,
    // split sweep: hole-pair lists and the clean-cell kernel's slots
    B_LBITS, B_LKCNT, B_LKOFF, B_LKBS, B_LPOS, B_LEPS, B_LS, B_LCNT, B_LFP, B_LCONN, B_LDC, B_LKEEP,
    // integral layouts of a system of a batched call
    B_LH, B_LX, B_LY, B_LCJ, B_LXJ, B_LJM, B_LKM, B_LJK,
    // Davidson
    B_ONES, B_DU, B_DW, B_DX, B_DR, B_DHX, B_DDIAG, B_DCOEF, B_DPART, B_DDOT,
    B_COUNT
};

// what a slot's integral layouts were last built from (batched calls)
struct LayoutKey {
    const double *h = nullptr, *eri = nullptr;
    int n = 0;
};

struct Prepared {
    int nint, nup, ndn, nel;
    int64_t n_det;
    int32_t *perm, *rank;
    double *F, *HII;
    int64_t *coff;
    CoarseEnt *cent;
    Scalars *sc;
    double *maxc2;
    double hmax[QPD_MAX_STATES];
    int64_t coarse_total;
};

struct qp_ctx {
    int device = 0;
    void *noalloc = nullptr;   // this device's no-allocation scratch (qp_generator_order_noalloc)
    void *probe_sink = nullptr;   // 8 bytes that qp_alu_probe's kernel never writes in practice
    std::string err;
    int n = 0;
    double *h = nullptr, *X = nullptr, *Y = nullptr, *Cj = nullptr, *CXj = nullptr, *Jm = nullptr, *Km = nullptr,
           *JK = nullptr;
    // device scratch, one set per system slot: slot s serves system s of a
    // batched call; single-system calls use slot 0
    std::vector<std::vector<DevBuf>> slots;
    std::vector<LayoutKey> layout_keys;
    DevBuf args[4];                // per-launch system descriptors (dense, general, clean-cell, split-correction)
    DevBuf defn;                   // per-system count of handed-over batches
    int num_cu = 256;
    size_t lds_per_cu = 163840;
    uint64_t ints_gen = 0;         // bumped by every qp_set_integrals
    // the sigma-build's prepared determinant space, kept in a slot of its own
    // for QP_SIGMA_REUSE: valid while dets, n_det, the integrals and the stream
    // match (the preparation's last kernels run after its host sync, so only
    // later work on the same stream is ordered after them)
    bool sig_valid = false;
    hipStream_t sig_stream = nullptr;
    const uint64_t *sig_dets = nullptr;
    int64_t sig_n_det = 0;
    uint64_t sig_gen = 0;
    Prepared sig_P;
    Scalars *host_sc = nullptr;    // pinned, one per system
    int host_sc_n = 0;
    uint64_t *host_det0 = nullptr; // pinned
    double *host_maxc2 = nullptr;  // pinned
    unsigned char *host_stage = nullptr;  // pinned staging of system descriptors
    size_t host_stage_bytes = 0;
    bool timing = false;
    bool timed = false;
    int split_mode = QP_SPLIT_AUTO;   // which sweeps split clean cells off (qp_set_split)
    // call start, dense sweep start, general kernel start, sweep end, call end
    // [5]: between the dense kernel and the clean-cell kernel
    hipEvent_t ev[8] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
};

namespace {

int fail(qp_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    return code;
}

#define HIPCHK(ctx, call)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) return fail(ctx, QP_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

void *grow(DevBuf &b, size_t bytes)
{
    if (bytes == 0) bytes = 8;
    if (b.bytes >= bytes) return b.p;
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
    size_t want = bytes + bytes / 4;
    if (hipMalloc(&b.p, want) != hipSuccess) {
        (void)hipGetLastError();
        if (hipMalloc(&b.p, bytes) != hipSuccess) { (void)hipGetLastError(); b.p = nullptr; return nullptr; }
        want = bytes;
    }
    b.bytes = want;
    return b.p;
}

void *scratch(qp_ctx *c, int slot, int id, size_t bytes)
{
    if ((int)c->slots.size() <= slot) c->slots.resize(slot + 1);
    std::vector<DevBuf> &v = c->slots[slot];
    if (v.empty()) v.resize(B_COUNT);
    return grow(v[id], bytes);
}

// pinned host staging for the per-launch system descriptors and the per-system
// scalars read back by the host
int host_space(qp_ctx *c, size_t stage_bytes, int n_sys)
{
    if (c->host_stage_bytes < stage_bytes || c->host_sc_n < n_sys) {
        // earlier calls' transfers may still read the old buffers
        HIPCHK(c, hipDeviceSynchronize());
    }
    if (c->host_stage_bytes < stage_bytes) {
        if (c->host_stage) (void)hipHostFree(c->host_stage);
        c->host_stage = nullptr;
        c->host_stage_bytes = 0;
        if (hipHostMalloc((void **)&c->host_stage, stage_bytes, hipHostMallocDefault) != hipSuccess)
            return fail(c, QP_E_OOM, "pinned host allocation failed");
        c->host_stage_bytes = stage_bytes;
    }
    if (c->host_sc_n < n_sys) {
        if (c->host_sc) (void)hipHostFree(c->host_sc);
        c->host_sc = nullptr;
        c->host_sc_n = 0;
        if (hipHostMalloc((void **)&c->host_sc, sizeof(Scalars) * n_sys, hipHostMallocDefault) != hipSuccess)
            return fail(c, QP_E_OOM, "pinned host allocation failed");
        c->host_sc_n = n_sys;
    }
    return QP_OK;
}

int64_t pow2_at_least(int64_t x)
{
    int64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

int grid_for(int64_t n, int tb = 256, int64_t cap = 65536)
{
    int64_t g = (n + tb - 1) / tb;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

// integral layouts of one system into I's (already allocated) arrays
void launch_layouts(const double *h, const double *eri, int n_orb, const DevInts &I, hipStream_t st)
{
    const int64_t n = n_orb;
    const int64_t nX = n * (n + 1) / 2 * n * n;
    const int64_t P2 = n * (n - 1) / 2;
    const int64_t n3 = n * n * n;
    hipLaunchKernelGGL(build_X, dim3(grid_for(nX, 256, 1 << 16)), dim3(256), 0, st, eri, n_orb, (double *)I.X);
    if (P2 > 0)
        hipLaunchKernelGGL(build_Y, dim3(grid_for(P2 * P2, 256, 1 << 16)), dim3(256), 0, st, eri, n_orb, (double *)I.Y);
    hipLaunchKernelGGL(build_small, dim3(grid_for(n3, 256, 1 << 16)), dim3(256), 0, st, eri, h, n_orb, (double *)I.Cj,
                       (double *)I.CXj, (double *)I.Jm, (double *)I.Km, (double *)I.JK, (double *)I.h);
}

struct LayoutSizes {
    size_t nX, nY, n3, n2;
};

LayoutSizes layout_sizes(int n_orb)
{
    const size_t n = n_orb;
    const size_t P2 = n * (n - 1) / 2;
    return {n * (n + 1) / 2 * n * n, std::max<size_t>(1, P2 * P2), n * n * n, n * n};
}

// Everything before the sweep: order, prep, coarse lists.  One host sync.

template <int NINT>
int prepare_t(qp_ctx *c, int slot, const DevInts &I, const uint64_t *dets, const double *coefs, int64_t n_det,
              int ns, int flags, hipStream_t st, Prepared &P)
{
    const int n = I.n;
    P.nint = NINT;
    P.n_det = n_det;
    const int64_t Pw = pow2_at_least(n_det);
    double *w = (double *)scratch(c, slot, B_W, sizeof(double) * n_det);
    int32_t *idx = (int32_t *)scratch(c, slot, B_IDX, sizeof(int32_t) * Pw);
    int32_t *rank = (int32_t *)scratch(c, slot, B_RANK, sizeof(int32_t) * n_det);
    double *F = (double *)scratch(c, slot, B_F, sizeof(double) * n_det * 2 * n);
    double *HII = (double *)scratch(c, slot, B_HII, sizeof(double) * n_det);
    Scalars *sc = (Scalars *)scratch(c, slot, B_SC, sizeof(Scalars));
    double *maxc2 = (double *)scratch(c, slot, B_MAXC2, sizeof(double) * QPD_MAX_STATES);
    if (!w || !idx || !rank || !F || !HII || !sc || !maxc2) return fail(c, QP_E_OOM, "device allocation failed");
    HIPCHK(c, hipMemsetAsync(sc, 0, sizeof(Scalars), st));
    {
        unsigned long long inf = 0x7ff0000000000000ull;
        HIPCHK(c, hipMemcpyAsync(&sc->min_delta_bits, &inf, sizeof(inf), hipMemcpyHostToDevice, st));
    }
    hipLaunchKernelGGL(gen_weights, dim3(grid_for(Pw)), dim3(256), 0, st, coefs, n_det, ns, w, Pw, idx);
    hipLaunchKernelGGL(max_c2, dim3(1), dim3(256), 0, st, coefs, n_det, ns, maxc2);
    bitonic_sort(idx, Pw, GenCmp<NINT>{w, dets}, st);
    hipLaunchKernelGGL(make_rank, dim3(grid_for(n_det)), dim3(256), 0, st, idx, n_det, rank);
    hipLaunchKernelGGL(prep_generators<NINT>, dim3((unsigned)n_det), dim3(128), 0, st, dets, idx, n_det, n, I.h,
                       I.Jm, I.Km, F, HII, sc);
    // coarse counts
    const int64_t gblocks = (n_det + 255) / 256;
    int nchunk = (int)std::max<int64_t>(1, std::min<int64_t>((2048 + gblocks - 1) / gblocks, (n_det + 255) / 256));
    const int64_t chunk = (n_det + nchunk - 1) / nchunk;
    const int64_t ncount = n_det * nchunk;
    int32_t *counts = (int32_t *)scratch(c, slot, B_COUNTS, sizeof(int32_t) * ncount);
    int64_t *offs = (int64_t *)scratch(c, slot, B_OFFS, sizeof(int64_t) * ncount);
    const int64_t nsb = (ncount + 1023) / 1024;
    int64_t *bsum = (int64_t *)scratch(c, slot, B_BSUM, sizeof(int64_t) * nsb);
    int64_t *total = (int64_t *)scratch(c, slot, B_TOTAL, sizeof(int64_t));
    int64_t *coff = (int64_t *)scratch(c, slot, B_COFF, sizeof(int64_t) * (n_det + 1));
    if (!counts || !offs || !bsum || !total || !coff) return fail(c, QP_E_OOM, "device allocation failed");
    hipLaunchKernelGGL((coarse_kernel<NINT, false>), dim3((unsigned)gblocks, nchunk), dim3(256), 0, st, dets, idx, rank,
                       n_det, chunk, nchunk, counts, (const int64_t *)nullptr, (CoarseEnt *)nullptr, sc);
    hipLaunchKernelGGL(scan_block, dim3((unsigned)nsb), dim3(256), 0, st, counts, ncount, offs, bsum);
    hipLaunchKernelGGL(scan_bsum, dim3(1), dim3(1), 0, st, bsum, nsb, total);
    hipLaunchKernelGGL(scan_add, dim3(grid_for(ncount, 256, 1 << 30)), dim3(256), 0, st, offs, ncount, bsum);
    hipLaunchKernelGGL(make_coff, dim3(grid_for(n_det + 1)), dim3(256), 0, st, offs, n_det, nchunk, total, coff, sc);
    HIPCHK(c, hipMemcpyAsync(c->host_det0, dets, sizeof(uint64_t) * 2 * NINT, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipMemcpyAsync(c->host_sc, sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipMemcpyAsync(c->host_maxc2, maxc2, sizeof(double) * QPD_MAX_STATES, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    HIPCHK(c, hipGetLastError());
    const Scalars hs = *c->host_sc;
    if (!(flags & QP_FLAG_NOCHECK)) {
        if (hs.bad_bits) return fail(c, QP_E_NORB, "a determinant has a bit set at or above n_orb");
        if (hs.bad_elec) return fail(c, QP_E_ELEC, "per-spin electron counts differ between determinants");
        if (hs.dup) return fail(c, QP_E_DUP, "duplicate determinant");
    }
    int nup = 0, ndn = 0;
    for (int wq = 0; wq < NINT; ++wq) {
        nup += __builtin_popcountll(c->host_det0[wq]);
        ndn += __builtin_popcountll(c->host_det0[NINT + wq]);
    }
    P.nup = nup; P.ndn = ndn; P.nel = nup + ndn;
    for (int k = 0; k < QPD_MAX_STATES; ++k) P.hmax[k] = c->host_maxc2[k];
    const int64_t ctot = (int64_t)hs.coarse_total;
    CoarseEnt *cent = (CoarseEnt *)scratch(c, slot, B_CENT, sizeof(CoarseEnt) * (ctot > 0 ? ctot : 1));
    if (!cent) return fail(c, QP_E_OOM, "device allocation failed (coarse lists)");
    hipLaunchKernelGGL((coarse_kernel<NINT, true>), dim3((unsigned)gblocks, nchunk), dim3(256), 0, st, dets, idx, rank,
                       n_det, chunk, nchunk, counts, (const int64_t *)offs, cent, sc);
    P.perm = idx; P.rank = rank; P.F = F; P.HII = HII; P.coff = coff; P.cent = cent; P.sc = sc; P.maxc2 = maxc2;
    P.coarse_total = ctot;
    return QP_OK;
}

int prepare(qp_ctx *c, int slot, const DevInts &I, const uint64_t *dets, const double *coefs, int64_t n_det, int ns,
            int flags, hipStream_t st, Prepared &P)
{
    switch ((I.n - 1) / 64 + 1) {
    case 1: return prepare_t<1>(c, slot, I, dets, coefs, n_det, ns, flags, st, P);
    case 2: return prepare_t<2>(c, slot, I, dets, coefs, n_det, ns, flags, st, P);
    case 3: return prepare_t<3>(c, slot, I, dets, coefs, n_det, ns, flags, st, P);
    default: return prepare_t<4>(c, slot, I, dets, coefs, n_det, ns, flags, st, P);
    }
}

int64_t cells_per_generator(int n, int nup, int ndn)
{
    int64_t vu = n - nup, vd = n - ndn;
    return (int64_t)nup * vu + (int64_t)ndn * vd + (int64_t)nup * (nup - 1) / 2 * (vu * (vu - 1) / 2) +
           (int64_t)ndn * (ndn - 1) / 2 * (vd * (vd - 1) / 2) + (int64_t)nup * vu * ndn * vd;
}

int check_system(qp_ctx *c, int n_orb, const uint64_t *dets, const double *coefs, int64_t n_det, int ns,
                 const double *E0)
{
    if (n_det < 0) return fail(c, QP_E_ARG, "n_det < 0");
    if (ns < 1 || ns > QP_MAX_STATES) return fail(c, QP_E_STATES, "n_states must be in [1,4]");
    if (n_orb <= 0) return fail(c, QP_E_NOINT, "integrals not set");
    if (n_det > 0 && (!dets || !coefs || !E0)) return fail(c, QP_E_ARG, "null input pointer");
    if (n_det > (int64_t)INT32_MAX / 2) return fail(c, QP_E_ARG, "n_det too large");
    return QP_OK;
}

int common_checks(qp_ctx *c, const uint64_t *dets, const double *coefs, int64_t n_det, int ns, const double *E0)
{
    if (!c) return QP_E_ARG;
    c->err.clear();
    int rc = check_system(c, c->n, dets, coefs, n_det, ns, E0);
    if (rc != QP_OK) return rc;
    HIPCHK(c, hipSetDevice(c->device));
    return QP_OK;
}

DevInts dev_ints(const qp_ctx *c)
{
    DevInts I;
    I.n = c->n; I.h = c->h; I.X = c->X; I.Y = c->Y; I.Cj = c->Cj; I.CXj = c->CXj; I.Jm = c->Jm; I.Km = c->Km;
    I.JK = c->JK;
    return I;
}

// ------------------------------------------------- launch-shape dispatchers
template <int NINT>
int sweep_occ_t(int ns, bool bwd, size_t lds)
{
    switch (ns) {
    case 1: return bwd ? sweep_occupancy<NINT, 1, true>(lds) : sweep_occupancy<NINT, 1, false>(lds);
    case 2: return bwd ? sweep_occupancy<NINT, 2, true>(lds) : sweep_occupancy<NINT, 2, false>(lds);
    case 3: return bwd ? sweep_occupancy<NINT, 3, true>(lds) : sweep_occupancy<NINT, 3, false>(lds);
    default: return bwd ? sweep_occupancy<NINT, 4, true>(lds) : sweep_occupancy<NINT, 4, false>(lds);
    }
}

template <int NINT>
int fast_occ_t(int ns, bool bwd, size_t lds, bool fp)
{
    switch (ns) {
    case 1: return bwd ? fast_occupancy<NINT, 1, true>(lds, fp) : fast_occupancy<NINT, 1, false>(lds, fp);
    case 2: return bwd ? fast_occupancy<NINT, 2, true>(lds, fp) : fast_occupancy<NINT, 2, false>(lds, fp);
    case 3: return bwd ? fast_occupancy<NINT, 3, true>(lds, fp) : fast_occupancy<NINT, 3, false>(lds, fp);
    default: return bwd ? fast_occupancy<NINT, 4, true>(lds, fp) : fast_occupancy<NINT, 4, false>(lds, fp);
    }
}

// persistent grid: every resident one-wavefront workgroup the CUs can hold
// the three sweep kernels: the dense kernel, the general kernel on handed-over
// batches, and the clean-cell kernel of a split sweep
enum Kind { K_DENSE = 0, K_GENERAL = 1, K_LEAN = 2, K_CORR = 3 };

template <int NINT, bool BWD>
int corr_occ_t(int ns, size_t lds, bool fp)
{
    switch (ns) {
    case 1: return corr_occupancy<NINT, 1, BWD>(lds, fp);
    case 2: return corr_occupancy<NINT, 2, BWD>(lds, fp);
    case 3: return corr_occupancy<NINT, 3, BWD>(lds, fp);
    default: return corr_occupancy<NINT, 4, BWD>(lds, fp);
    }
}

template <int NINT, bool BWD>
int lean_occ_t(int ns, size_t lds, bool fp)
{
    switch (ns) {
    case 1: return lean_occupancy<NINT, 1, BWD>(lds, fp);
    case 2: return lean_occupancy<NINT, 2, BWD>(lds, fp);
    case 3: return lean_occupancy<NINT, 3, BWD>(lds, fp);
    default: return lean_occupancy<NINT, 4, BWD>(lds, fp);
    }
}

template <int NINT>
int kind_occ_t(int kind, int ns, bool bwd, size_t lds, bool fp)
{
    if (kind == K_DENSE) return fast_occ_t<NINT>(ns, bwd, lds, fp);
    if (kind == K_LEAN) return bwd ? lean_occ_t<NINT, true>(ns, lds, fp) : lean_occ_t<NINT, false>(ns, lds, fp);
    if (kind == K_CORR) return bwd ? corr_occ_t<NINT, true>(ns, lds, fp) : corr_occ_t<NINT, false>(ns, lds, fp);
    return sweep_occ_t<NINT>(ns, bwd, lds);
}

int persistent_grid(qp_ctx *c, int kind, int nint, int ns, bool bwd, size_t lds, bool fp)
{
    int per_cu = 8;
    switch (nint) {
    case 1: per_cu = kind_occ_t<1>(kind, ns, bwd, lds, fp); break;
    case 2: per_cu = kind_occ_t<2>(kind, ns, bwd, lds, fp); break;
    case 3: per_cu = kind_occ_t<3>(kind, ns, bwd, lds, fp); break;
    default: per_cu = kind_occ_t<4>(kind, ns, bwd, lds, fp); break;
    }
    // The hardware allocates a workgroup's LDS in granules, which the runtime's
    // occupancy figure does not round to: where the rounded size leaves room
    // for fewer workgroups, a persistent grid sized by the runtime would leave
    // the surplus workgroups waiting for a free slot, and their share of the
    // statically dealt items would run after everyone else's.  The size is
    // rounded to both 512 and 1280 bytes, whichever is larger, to stay on the
    // safe side of the granule.
    if (lds > 0) {
        const size_t r512 = (lds + 511) / 512 * 512, r1280 = (lds + 1279) / 1280 * 1280;
        const int fit = (int)(c->lds_per_cu / (r512 > r1280 ? r512 : r1280));
        if (fit < per_cu) per_cu = fit;
    }
    if (per_cu < 1) per_cu = 1;
    if (per_cu > 32) per_cu = 32;
    return c->num_cu * per_cu;
}

// correction rows (and columns) the dense kernel buffers per batch: 6 up to
// n_orb = 128, 3 above.  Up to 128 orbitals the count drops, to 4 at least,
// while the LDS it takes would leave room for fewer workgroups per CU than
// the kernel's registers allow: batches that overflow the buffers go to the
// general kernel, which costs less than a quarter of the waves (n_orb 128,
// 14+14 electrons, 10^5 determinants: dense kernel 1616 -> 1362 ms, general
// kernel 6 -> 36 ms).  The count depends on the system alone.
int buffer_rows(qp_ctx *c, int n, int nvm, int nint, int ns, bool bwd, bool fp)
{
    if (n > 128) return 3;
    const int regs = persistent_grid(c, K_DENSE, nint, ns, bwd, 0, fp) / c->num_cu;
    int cap = 6;
    while (cap > 4) {
        const size_t lds = fast_lds_bytes(n, nvm, ns, bwd, cap, cap);
        const size_t r512 = (lds + 511) / 512 * 512, r1280 = (lds + 1279) / 1280 * 1280;
        if ((int)(c->lds_per_cu / (r512 > r1280 ? r512 : r1280)) >= regs) break;
        --cap;
    }
    return cap;
}

template <int NINT, int NS>
void launch_ns(int kind, const SweepArgs *sys, const int64_t *end, int n_sys, bool bwd, bool fp, size_t lds,
               int grid, hipStream_t st)
{
    if (kind == K_LEAN) {
        if (bwd) launch_lean<NINT, NS, true>(sys, end, n_sys, fp, lds, grid, st);
        else launch_lean<NINT, NS, false>(sys, end, n_sys, fp, lds, grid, st);
    } else if (kind == K_CORR) {
        if (bwd) launch_corr<NINT, NS, true>(sys, end, n_sys, fp, lds, grid, st);
        else launch_corr<NINT, NS, false>(sys, end, n_sys, fp, lds, grid, st);
    } else if (kind == K_DENSE) {
        if (bwd) launch_fast<NINT, NS, true>(sys, end, n_sys, fp, lds, grid, st);
        else launch_fast<NINT, NS, false>(sys, end, n_sys, fp, lds, grid, st);
    } else {
        if (bwd) launch_sweep<NINT, NS, true>(sys, end, n_sys, lds, grid, st);
        else launch_sweep<NINT, NS, false>(sys, end, n_sys, lds, grid, st);
    }
}

template <int NINT>
void launch_nint(int kind, int ns, const SweepArgs *sys, const int64_t *end, int n_sys, bool bwd, bool fp,
                 size_t lds, int grid, hipStream_t st)
{
    switch (ns) {
    case 1: launch_ns<NINT, 1>(kind, sys, end, n_sys, bwd, fp, lds, grid, st); break;
    case 2: launch_ns<NINT, 2>(kind, sys, end, n_sys, bwd, fp, lds, grid, st); break;
    case 3: launch_ns<NINT, 3>(kind, sys, end, n_sys, bwd, fp, lds, grid, st); break;
    default: launch_ns<NINT, 4>(kind, sys, end, n_sys, bwd, fp, lds, grid, st); break;
    }
}

void launch_kernel(int kind, int nint, int ns, const SweepArgs *sys, const int64_t *end, int n_sys, bool bwd,
                   bool fp, size_t lds, int grid, hipStream_t st)
{
    switch (nint) {
    case 1: launch_nint<1>(kind, ns, sys, end, n_sys, bwd, fp, lds, grid, st); break;
    case 2: launch_nint<2>(kind, ns, sys, end, n_sys, bwd, fp, lds, grid, st); break;
    case 3: launch_nint<3>(kind, ns, sys, end, n_sys, bwd, fp, lds, grid, st); break;
    default: launch_nint<4>(kind, ns, sys, end, n_sys, bwd, fp, lds, grid, st); break;
    }
}

// work items per generator: the forward sweep splits each generator's batches
// over 16 items (batch b goes to item b mod 16) so that the persistent grid
// stays balanced; the adjoint keeps 4, because each item ends with atomic
// updates of the n x n one-electron gradient.  Items are dealt round-robin,
// without a shared counter.
constexpr int Q_FORWARD = 16;
// handed-over batches: up to 8 row parts each, aiming at 8192 general-kernel items
constexpr int64_t DEF_PARTS_MAX = 8;
constexpr int64_t DEF_PARTS_ITEMS = 8192;
constexpr int Q_ADJOINT = 4;
constexpr int64_t MAX_ITEMS = int64_t(1) << 25;

int items_per_generator(int64_t n_det, int nb, bool bwd)
{
    int q = bwd ? Q_ADJOINT : Q_FORWARD;
    if (nb > 0 && q > nb) q = nb;
    while (q > 1 && n_det * q > MAX_ITEMS) q /= 2;
    return std::max(q, 1);
}

// one system of a sweep call
struct SysIn {
    DevInts I;
    const uint64_t *dets;
    const double *coefs;
    int64_t n_det;
    const int32_t *gens;        // generators of the call by determinant index (null: all)
    int64_t n_gen;
    int ns;
    const double *E0;
    int64_t n_select;
    double *e_pt2;
    uint64_t *sel_dets;
    double *sel_e;
    int64_t *n_sel;
    uint64_t *sel_key;          // optional: the selection's criterion keys, in its order
    int sel_floor_bin;          // the selection threshold's starting histogram bin (0: none): alpha
                                // with keys below its lower edge are not candidates
    qp_pt2_stats *stats;
    double *eps_gen;
    const double *gup;
    double *grad_coefs, *grad_E0, *grad_h;
    // order, generator tables and coarse lists already prepared in this
    // system's slot from these same inputs (null: prepare them)
    const Prepared *pre;
};

// per-system state between the phases of a sweep call
struct SysRun {
    int slot = 0;
    int nint = 1;
    int32_t *gen_rank = nullptr;  // ranks of the listed generators (null: all)
    int64_t n_g = 0;              // generators of the call
    bool swept = false;         // has dense-kernel items
    Prepared P;
    int Q = 1;
    int64_t n_items = 0;
    int nbw = 1;
    int64_t nsb = 1;
    SweepArgs a;
    int64_t cand_cap = 0;
    Cand *cand = nullptr;
    uint32_t *def_bits = nullptr;
    int32_t *def_cnt_g = nullptr;
    int64_t *def_off = nullptr, *def_bsum = nullptr;
    double *eps_item = nullptr, *S_item = nullptr, *dc_item = nullptr;
    uint32_t *cnt_item = nullptr, *conn_item = nullptr;
    uint64_t *fp_item = nullptr;
    double *eps_g = nullptr, *S_g = nullptr;
    uint64_t *cnt_g = nullptr, *fp_g = nullptr, *conn_g = nullptr, *defa_g = nullptr;
    int64_t n_def = 0;
    SweepArgs d;
    DefParts dp;
    bool split = false;         // forward split sweep (clean-cell kernel)
    int n_pairs = 0;
};

// the launches of one kernel over several systems: one per (n_int, n_states)
// class, each system's items in system order
struct LaunchPlan {
    int nint, ns;
    size_t lds;
    int grid;
    std::vector<int> sys;       // indices into the call's systems
    std::vector<int64_t> end;   // running item end per listed system
};

std::vector<LaunchPlan> plan_launches(qp_ctx *c, int kind, bool bwd, bool fp, const std::vector<SysIn> &in,
                                      const std::vector<SysRun> &run, const std::vector<int64_t> &items)
{
    std::vector<LaunchPlan> plans;
    for (size_t s = 0; s < in.size(); ++s) {
        if (items[s] <= 0) continue;
        const int nint = run[s].nint, ns = in[s].ns, n = in[s].I.n;
        size_t lds;
        const int nvm = n - std::min(run[s].P.nup, run[s].P.ndn);
        if (kind == K_DENSE) lds = fast_lds_bytes(n, nvm, ns, bwd, run[s].a.rscap, run[s].a.cscap);
        else if (kind == K_LEAN) lds = lean_lds_bytes(n, nvm, bwd);
        else if (kind == K_CORR) lds = corr_lds_bytes(n, ns, bwd);
        else lds = sweep_lds_bytes(n, ns, bwd);
        LaunchPlan *p = nullptr;
        for (auto &q : plans) if (q.nint == nint && q.ns == ns) p = &q;
        if (!p) {
            plans.push_back(LaunchPlan{nint, ns, 0, 0, {}, {}});
            p = &plans.back();
        }
        p->lds = std::max(p->lds, lds);
        p->sys.push_back((int)s);
        p->end.push_back((p->end.empty() ? 0 : p->end.back()) + items[s]);
    }
    for (auto &p : plans) p.grid = persistent_grid(c, kind, p.nint, p.ns, bwd, p.lds, fp);
    return plans;
}

// copy the plans' descriptors to the device in one transfer and launch them
int launch_plans(qp_ctx *c, int kind, bool bwd, bool fp, std::vector<LaunchPlan> &plans,
                 const std::vector<SysRun> &run, hipStream_t st)
{
    if (plans.empty()) return QP_OK;
    size_t nsys = 0;
    for (auto &p : plans) nsys += p.sys.size();
    const size_t args_bytes = sizeof(SweepArgs) * nsys;
    // clean-cell launches: each plan's item counters, zero, staged with the
    // descriptors
    const size_t ctr_at = (args_bytes + sizeof(int64_t) * nsys + 127) / 128 * 128;
    const size_t ctr_bytes = sizeof(unsigned long long) * ITEM_CTR_GROUPS * ITEM_CTR_STRIDE;
    const bool claims = kind == K_LEAN;
    const size_t bytes = claims ? ctr_at + ctr_bytes * plans.size() : args_bytes + sizeof(int64_t) * nsys;
    // the staging area is reused only after a host synchronisation on `st`,
    // which every call performs between its two launch rounds
    const size_t quarter = c->host_stage_bytes / 4 / 16 * 16;
    unsigned char *stage = c->host_stage + kind * quarter;
    if (bytes > quarter) return fail(c, QP_E_ARG, "staging area too small");
    unsigned char *dev = (unsigned char *)grow(c->args[kind], bytes);
    if (!dev) return fail(c, QP_E_OOM, "device allocation failed (system descriptors)");
    SweepArgs *ha = (SweepArgs *)stage;
    int64_t *he = (int64_t *)(stage + args_bytes);
    size_t k = 0;
    for (size_t pi = 0; pi < plans.size(); ++pi) {
        auto &p = plans[pi];
        for (size_t i = 0; i < p.sys.size(); ++i, ++k) {
            ha[k] = kind == K_GENERAL ? run[p.sys[i]].d : run[p.sys[i]].a;
            ha[k].item_ctr = claims ? (unsigned long long *)(dev + ctr_at + ctr_bytes * pi) : nullptr;
            he[k] = p.end[i];
        }
    }
    if (claims) memset(stage + ctr_at, 0, ctr_bytes * plans.size());
    HIPCHK(c, hipMemcpyAsync(dev, stage, bytes, hipMemcpyHostToDevice, st));
    k = 0;
    for (auto &p : plans) {
        const SweepArgs *da = (const SweepArgs *)dev + k;
        const int64_t *de = (const int64_t *)(dev + args_bytes) + k;
        int grid = p.grid;
        if (kind != K_DENSE) grid = (int)std::min<int64_t>(grid, p.end.back());
        launch_kernel(kind, p.nint, p.ns, da, de, (int)p.sys.size(), bwd, fp, p.lds, grid, st);
        HIPCHK(c, hipGetLastError());
        k += p.sys.size();
    }
    return QP_OK;
}

// The sweep over one or more systems (bwd: the adjoint sweep, which also
// yields E_PT2).  Phases, each over all systems: preparation (one host sync
// per system), the dense kernel, the deferred-batch lists (one host sync), the
// general kernel, the deterministic reductions, and the selection (one host
// sync).
int run_sweeps(qp_ctx *c, std::vector<SysIn> &in, int flags, bool bwd, hipStream_t st)
{
    const int n_sys = (int)in.size();
    c->timed = false;
    if (n_sys == 0) return QP_OK;
    {
        // a quarter per kernel kind: descriptors and end offsets, and for the
        // clean-cell kind the item counters of up to 16 launches (4 word
        // counts x 4 state counts)
        const size_t ctr_room = 128 + 16 * sizeof(unsigned long long) * ITEM_CTR_GROUPS * ITEM_CTR_STRIDE;
        int rc = host_space(c, std::max<size_t>(4 << 16, 4 * ((sizeof(SweepArgs) + 8) * (size_t)n_sys + 256 + ctr_room)),
                            n_sys);
        if (rc != QP_OK) return rc;
    }
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[0], st));
    std::vector<SysRun> run(n_sys);
    std::vector<int64_t> items(n_sys, 0), litems(n_sys, 0);
    const bool fp = (flags & QP_FLAG_FINGERPRINT) != 0;

    // ------------------------------------------------------------ phase 1
    for (int s = 0; s < n_sys; ++s) {
        SysIn &x = in[s];
        SysRun &r = run[s];
        r.slot = s;
        const int n = x.I.n;
        const int ns = x.ns;
        r.nint = (n - 1) / 64 + 1;
        if (x.n_det == 0) {
            if (x.e_pt2) HIPCHK(c, hipMemsetAsync(x.e_pt2, 0, sizeof(double) * ns, st));
            if (x.stats) HIPCHK(c, hipMemsetAsync(x.stats, 0, sizeof(qp_pt2_stats), st));
            if (x.n_sel) HIPCHK(c, hipMemsetAsync(x.n_sel, 0, sizeof(int64_t), st));
            if (bwd && x.grad_E0) HIPCHK(c, hipMemsetAsync(x.grad_E0, 0, sizeof(double) * ns, st));
            if (bwd && x.grad_h) HIPCHK(c, hipMemsetAsync(x.grad_h, 0, sizeof(double) * n * n, st));
            continue;
        }
        if (x.pre) {
            r.P = *x.pre;
            hipLaunchKernelGGL(reset_sweep_scalars, dim3(1), dim3(1), 0, st, r.P.sc, x.sel_floor_bin);
        } else {
            int rc = prepare(c, s, x.I, x.dets, x.coefs, x.n_det, ns, flags, st, r.P);
            if (rc != QP_OK) return rc;
            if (x.sel_floor_bin > 0)
                hipLaunchKernelGGL(reset_sweep_scalars, dim3(1), dim3(1), 0, st, r.P.sc, x.sel_floor_bin);
        }
        const int64_t n_det = x.n_det;
        r.n_g = n_det;
        if (x.gens) {
            r.n_g = x.n_gen;
            r.gen_rank = (int32_t *)scratch(c, s, B_GENR, sizeof(int32_t) * std::max<int64_t>(1, x.n_gen));
            if (!r.gen_rank) return fail(c, QP_E_OOM, "device allocation failed (generator list)");
            if (x.n_gen > 0) {
                hipLaunchKernelGGL(map_gen_ranks, dim3(grid_for(x.n_gen)), dim3(256), 0, st, x.gens, x.n_gen,
                                   r.P.rank, n_det, r.gen_rank, r.P.sc);
                // the list is checked unless the caller vouches for it (the
                // semi-stochastic driver builds it from the generator order)
                if (!(flags & QP_FLAG_NOCHECK)) {
                    HIPCHK(c, hipMemcpyAsync(c->host_sc, r.P.sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
                    HIPCHK(c, hipStreamSynchronize(st));
                    if (c->host_sc->bad_gen) return fail(c, QP_E_ARG, "a listed generator is outside [0, n_det)");
                }
            }
        }
        const int64_t n_g = r.n_g;
        const int nel = r.P.nel;
        const int nb = nel + nel * (nel - 1) / 2;
        // the same split as a sweep over every generator, so that a listed
        // generator's results do not depend on the list
        r.Q = items_per_generator(n_det, nb, bwd);
        r.n_items = n_g * r.Q;
        r.swept = r.n_items > 0 && nel > 0;
        const int64_t ni = std::max<int64_t>(1, r.n_items);
        r.eps_item = (double *)scratch(c, s, B_EPSI, sizeof(double) * ni * ns);
        r.S_item = (double *)scratch(c, s, B_SI, sizeof(double) * ni * ns);
        r.cnt_item = (uint32_t *)scratch(c, s, B_CNTI, sizeof(uint32_t) * ni);
        r.fp_item = (uint64_t *)scratch(c, s, B_FPI, sizeof(uint64_t) * ni);
        r.dc_item = bwd ? (double *)scratch(c, s, B_DCI, sizeof(double) * ni * ns) : nullptr;
        r.conn_item = (uint32_t *)scratch(c, s, B_CONNI, sizeof(uint32_t) * ni);
        const int64_t ng1 = std::max<int64_t>(1, n_g);
        r.eps_g = (double *)scratch(c, s, B_EPSG, sizeof(double) * ng1 * ns);
        r.S_g = (double *)scratch(c, s, B_SG, sizeof(double) * ng1 * ns);
        r.cnt_g = (uint64_t *)scratch(c, s, B_CNTG, sizeof(uint64_t) * ng1);
        r.fp_g = (uint64_t *)scratch(c, s, B_FPG, sizeof(uint64_t) * ng1);
        r.conn_g = (uint64_t *)scratch(c, s, B_CONNG, sizeof(uint64_t) * ng1);
        r.defa_g = (uint64_t *)scratch(c, s, B_DEFAG, sizeof(uint64_t) * ng1);
        unsigned int *hist = (unsigned int *)scratch(c, s, B_HIST, sizeof(unsigned int) * QP_HIST_BINS);
        // batches the dense kernel hands to the general kernel: one bit per
        // (generator rank, batch), then a list in (rank, batch) order
        r.nbw = std::max(1, (nb + 31) / 32);
        r.def_bits = (uint32_t *)scratch(c, s, B_DEFBITS, sizeof(uint32_t) * n_det * r.nbw);
        r.def_cnt_g = (int32_t *)scratch(c, s, B_DEFCG, sizeof(int32_t) * n_det);
        r.def_off = (int64_t *)scratch(c, s, B_DEFOFF, sizeof(int64_t) * n_det);
        r.nsb = (n_det + 1023) / 1024;
        r.def_bsum = (int64_t *)scratch(c, s, B_DEFBS, sizeof(int64_t) * std::max<int64_t>(1, r.nsb));
        if (!r.eps_item || !r.S_item || !r.cnt_item || !r.fp_item || (bwd && !r.dc_item) || !r.conn_item ||
            !r.eps_g || !r.S_g || !r.cnt_g || !r.fp_g || !r.conn_g || !r.defa_g || !hist || !r.def_bits ||
            !r.def_cnt_g || !r.def_off || !r.def_bsum)
            return fail(c, QP_E_OOM, "device allocation failed (sweep buffers)");
        HIPCHK(c, hipMemsetAsync(r.def_bits, 0, sizeof(uint32_t) * n_det * r.nbw, st));
        const int nvm = n - std::min(r.P.nup, r.P.ndn);
        const int rscap = buffer_rows(c, n, nvm, r.nint, ns, bwd, fp), cscap = rscap;
        if (x.n_select > 0) {
            const int grid = std::max(persistent_grid(c, K_DENSE, r.nint, ns, bwd,
                                                      fast_lds_bytes(n, nvm, ns, bwd, rscap, cscap), fp),
                                      persistent_grid(c, K_GENERAL, r.nint, ns, bwd, sweep_lds_bytes(n, ns, bwd), fp));
            const int64_t maxcell = std::max<int64_t>((int64_t)(n - r.P.nup) * (n - r.P.ndn),
                                                      (int64_t)(n - r.P.nup) * (n - r.P.nup - 1) / 2);
            r.cand_cap = x.n_select + std::max<int64_t>(1 << 22, 2 * (int64_t)grid * std::min<int64_t>(maxcell, 3072));
            r.cand = (Cand *)scratch(c, s, B_CAND, sizeof(Cand) * r.cand_cap);
            if (!r.cand) return fail(c, QP_E_OOM, "device allocation failed (selection candidates)");
            HIPCHK(c, hipMemsetAsync(hist, 0, sizeof(unsigned int) * QP_HIST_BINS, st));
        }
        if (bwd) {
            if (x.grad_coefs) HIPCHK(c, hipMemsetAsync(x.grad_coefs, 0, sizeof(double) * ns * n_det, st));
            if (x.grad_h) HIPCHK(c, hipMemsetAsync(x.grad_h, 0, sizeof(double) * n * n, st));
        }
        SweepArgs &a = r.a;
        memset(&a, 0, sizeof(a));
        a.I = x.I;
        a.n = n; a.nup = r.P.nup; a.ndn = r.P.ndn; a.ns = ns; a.nel = nel;
        a.n_det = n_det; a.dets = x.dets; a.coefs = x.coefs; a.E0 = x.E0;
        a.perm = r.P.perm; a.F = r.P.F; a.HII = r.P.HII; a.coff = r.P.coff; a.cent = r.P.cent;
        a.n_items = r.n_items;
        a.q_per_gen = r.Q;
        a.gen_list = r.gen_rank;
        a.n_gen = n_g;
        a.flags = (fp ? 1 : 0) | (bwd ? 2 : 0);
        a.eps_item = r.eps_item; a.S_item = r.S_item; a.cnt_item = r.cnt_item; a.fp_item = r.fp_item;
        a.conn_item = r.conn_item;
        a.min_delta_bits = &r.P.sc->min_delta_bits;
        a.fine_total = &r.P.sc->fine_total;
        a.n_select = x.n_select;
        for (int k = 0; k < QPD_MAX_STATES; ++k) {
            a.maxc2[k] = k < ns ? r.P.hmax[k] : 1.0;
            a.inv_maxc2[k] = k < ns ? 1.0 / r.P.hmax[k] : 0.0;
        }
        a.cand = r.cand; a.cand_count = &r.P.sc->cand_count; a.cand_cap = r.cand_cap; a.hist = hist;
        a.tau_bin = &r.P.sc->tau_bin; a.overflow = &r.P.sc->overflow;
        a.gup = x.gup; a.dc_item = r.dc_item; a.dc = x.grad_coefs; a.dh = x.grad_h;
        a.rscap = rscap; a.cscap = cscap;
        a.def_bits = r.def_bits; a.nbw = r.nbw;
        a.def_mode = 0;
        items[s] = r.swept ? r.n_items : 0;
        // split sweep (forward): hole-pair lists for the clean-cell kernel
        // (a fingerprinted adjoint is not split: the adjoint kernels have no
        // fingerprint variant)
        // (auto: batches of at least QP_SPLIT_MIN_VIRT particles per spin, below
        // which the clean-cell kernel's per-batch set-up outweighs its cell
        // loop: n_orb 64, 10+10 electrons, 10^4 determinants forward 17.0 ms
        // unsplit, 28.3 ms split; n_orb 128, 14+14, 10^5: 1.41 s, 1.28 s)
        const int vmin = n - std::max(r.P.nup, r.P.ndn);
        r.split = r.swept && nel >= 2 && !(bwd && fp) &&
                  (c->split_mode == QP_SPLIT_ALWAYS || (c->split_mode == QP_SPLIT_AUTO && vmin >= QP_SPLIT_MIN_VIRT));
        if (r.split) {
            const int np = nel * (nel - 1) / 2;
            const int n_keys = n * n + n * (n - 1);
            const int64_t nw = (n_g + 63) / 64;
            const int64_t tot = n_g * np;
            const int64_t nkb = (n_keys + 1023) / 1024;
            uint64_t *bits = (uint64_t *)scratch(c, s, B_LBITS, sizeof(uint64_t) * 2 * n * nw);
            int32_t *kcnt = (int32_t *)scratch(c, s, B_LKCNT, sizeof(int32_t) * n_keys);
            int64_t *koff = (int64_t *)scratch(c, s, B_LKOFF, sizeof(int64_t) * (n_keys + 1));
            int64_t *kbs = (int64_t *)scratch(c, s, B_LKBS, sizeof(int64_t) * nkb);
            int32_t *kpos = (int32_t *)scratch(c, s, B_LPOS, sizeof(int32_t) * tot);
            double *leps = (double *)scratch(c, s, B_LEPS, sizeof(double) * tot * ns);
            double *lS = (double *)scratch(c, s, B_LS, sizeof(double) * tot * ns);
            unsigned long long *lcnt = (unsigned long long *)scratch(c, s, B_LCNT, sizeof(unsigned long long) * n_g);
            unsigned long long *lfp = (unsigned long long *)scratch(c, s, B_LFP, sizeof(unsigned long long) * n_g);
            unsigned long long *lconn = (unsigned long long *)scratch(c, s, B_LCONN, sizeof(unsigned long long) * n_g);
            double *ldc = bwd ? (double *)scratch(c, s, B_LDC, sizeof(double) * tot * ns) : nullptr;
            uint32_t *lkeep = (uint32_t *)scratch(c, s, B_LKEEP, sizeof(uint32_t) * n_det * r.nbw);
            if (!bits || !kcnt || !koff || !kbs || !kpos || !leps || !lS || !lcnt || !lfp || !lconn || !lkeep || (bwd && !ldc))
                return fail(c, QP_E_OOM, "device allocation failed (clean-cell lists)");
            HIPCHK(c, hipMemsetAsync(lcnt, 0, sizeof(unsigned long long) * n_g, st));
            HIPCHK(c, hipMemsetAsync(lfp, 0, sizeof(unsigned long long) * n_g, st));
            HIPCHK(c, hipMemsetAsync(lconn, 0, sizeof(unsigned long long) * n_g, st));
            switch (r.nint) {
            case 1: hipLaunchKernelGGL(pair_bits<1>, dim3(grid_for(nw, 4, 1 << 30)), dim3(256), 0, st, x.dets, r.P.perm, r.gen_rank, n_g, n, nw, bits); break;
            case 2: hipLaunchKernelGGL(pair_bits<2>, dim3(grid_for(nw, 4, 1 << 30)), dim3(256), 0, st, x.dets, r.P.perm, r.gen_rank, n_g, n, nw, bits); break;
            case 3: hipLaunchKernelGGL(pair_bits<3>, dim3(grid_for(nw, 4, 1 << 30)), dim3(256), 0, st, x.dets, r.P.perm, r.gen_rank, n_g, n, nw, bits); break;
            default: hipLaunchKernelGGL(pair_bits<4>, dim3(grid_for(nw, 4, 1 << 30)), dim3(256), 0, st, x.dets, r.P.perm, r.gen_rank, n_g, n, nw, bits); break;
            }
            hipLaunchKernelGGL(pair_count, dim3((n_keys + 3) / 4), dim3(256), 0, st, bits, n, nw, n_keys, kcnt);
            hipLaunchKernelGGL(scan_block, dim3((unsigned)nkb), dim3(256), 0, st, kcnt, (int64_t)n_keys, koff, kbs);
            hipLaunchKernelGGL(scan_bsum, dim3(1), dim3(1), 0, st, kbs, nkb, koff + n_keys);
            hipLaunchKernelGGL(scan_add, dim3(grid_for(n_keys, 256, 1 << 30)), dim3(256), 0, st, koff, (int64_t)n_keys, kbs);
            hipLaunchKernelGGL(pair_fill, dim3((n_keys + 3) / 4), dim3(256), 0, st, bits, n, nw, n_keys, koff, tot, kpos);
            HIPCHK(c, hipGetLastError());
            a.split = 1;
            a.n_pairs = np;
            a.kl_off = koff;
            a.kl_pos = kpos;
            a.n_keys = n_keys;
            a.lean_eps = leps;
            a.lean_S = lS;
            a.lean_cnt = lcnt;
            a.lean_fp = lfp;
            a.lean_conn = lconn;
            a.lean_dc = ldc;
            a.split_keep = lkeep;
            HIPCHK(c, hipMemsetAsync(lkeep, 0, sizeof(uint32_t) * n_det * r.nbw, st));
            r.n_pairs = np;
            litems[s] = tot;
        }
        // the fine filter's entries over every batch, and (split sweeps) the
        // pair batches the dense kernel keeps
        if (r.swept) {
            const int gb = (int)((n_g + 255) / 256);
            uint32_t *keep = r.split ? a.split_keep : nullptr;
            switch (r.nint) {
            case 1: hipLaunchKernelGGL(split_mark<1>, dim3(gb), dim3(256), 0, st, x.dets, r.P.perm, r.gen_rank, n_g, r.P.nup, r.P.ndn, r.P.coff, r.P.cent, r.nbw, keep, &r.P.sc->fine_total); break;
            case 2: hipLaunchKernelGGL(split_mark<2>, dim3(gb), dim3(256), 0, st, x.dets, r.P.perm, r.gen_rank, n_g, r.P.nup, r.P.ndn, r.P.coff, r.P.cent, r.nbw, keep, &r.P.sc->fine_total); break;
            case 3: hipLaunchKernelGGL(split_mark<3>, dim3(gb), dim3(256), 0, st, x.dets, r.P.perm, r.gen_rank, n_g, r.P.nup, r.P.ndn, r.P.coff, r.P.cent, r.nbw, keep, &r.P.sc->fine_total); break;
            default: hipLaunchKernelGGL(split_mark<4>, dim3(gb), dim3(256), 0, st, x.dets, r.P.perm, r.gen_rank, n_g, r.P.nup, r.P.ndn, r.P.coff, r.P.cent, r.nbw, keep, &r.P.sc->fine_total); break;
            }
            HIPCHK(c, hipGetLastError());
        }
    }

    // ------------------------------------------------- phase 2: dense kernel
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[1], st));
    {
        // forward: the dense kernel first, whose selection candidates raise the
        // threshold before the clean cells of split sweeps; adjoint: the
        // clean-cell kernel first, which marks the batches it takes for the
        // dense kernel (the flagged cells follow it, added to the same slots)
        int rc = QP_OK;
        if (!bwd) {
            std::vector<LaunchPlan> plans = plan_launches(c, K_DENSE, bwd, fp, in, run, items);
            rc = launch_plans(c, K_DENSE, bwd, fp, plans, run, st);
            if (rc != QP_OK) return rc;
        }
        if (c->timing) HIPCHK(c, hipEventRecord(c->ev[5], st));
        std::vector<LaunchPlan> lplans = plan_launches(c, K_LEAN, bwd, fp, in, run, litems);
        rc = launch_plans(c, K_LEAN, bwd, fp, lplans, run, st);
        if (rc != QP_OK) return rc;
        if (c->timing) HIPCHK(c, hipEventRecord(c->ev[7], st));
        std::vector<LaunchPlan> cplans = plan_launches(c, K_CORR, bwd, fp, in, run, litems);
        rc = launch_plans(c, K_CORR, bwd, fp, cplans, run, st);
        if (rc != QP_OK) return rc;
        if (c->timing) HIPCHK(c, hipEventRecord(c->ev[6], st));
        if (bwd) {
            std::vector<LaunchPlan> plans = plan_launches(c, K_DENSE, bwd, fp, in, run, items);
            rc = launch_plans(c, K_DENSE, bwd, fp, plans, run, st);
            if (rc != QP_OK) return rc;
        }
    }
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[2], st));

    // -------------------------------------- phase 3: lists of handed-over batches
    int64_t *def_n = (int64_t *)grow(c->defn, sizeof(int64_t) * n_sys);
    if (!def_n) return fail(c, QP_E_OOM, "device allocation failed (deferred counts)");
    HIPCHK(c, hipMemsetAsync(def_n, 0, sizeof(int64_t) * n_sys, st));
    bool any = false;
    for (int s = 0; s < n_sys; ++s) {
        SysRun &r = run[s];
        if (!r.swept) continue;
        any = true;
        const int64_t n_det = in[s].n_det;
        hipLaunchKernelGGL(def_count, dim3(grid_for(n_det)), dim3(256), 0, st, r.def_bits, n_det, r.nbw, r.def_cnt_g);
        hipLaunchKernelGGL(scan_block, dim3((unsigned)r.nsb), dim3(256), 0, st, r.def_cnt_g, n_det, r.def_off,
                           r.def_bsum);
        hipLaunchKernelGGL(scan_bsum, dim3(1), dim3(1), 0, st, r.def_bsum, r.nsb, def_n + s);
        hipLaunchKernelGGL(scan_add, dim3(grid_for(n_det, 256, 1 << 30)), dim3(256), 0, st, r.def_off, n_det,
                           r.def_bsum);
    }
    std::vector<int64_t> gitems(n_sys, 0);
    if (any) {
        int64_t *hn = (int64_t *)c->host_stage;   // the dense round's staging has been consumed by now
        HIPCHK(c, hipMemcpyAsync(hn, def_n, sizeof(int64_t) * n_sys, hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        HIPCHK(c, hipGetLastError());
        for (int s = 0; s < n_sys; ++s) run[s].n_def = run[s].swept ? hn[s] : 0;
        for (int s = 0; s < n_sys; ++s) {
            SysRun &r = run[s];
            if (!r.swept) continue;
            const int ns = in[s].ns;
            // a listed batch is split into row parts when there are few of them,
            // so that the general kernel's time is not that of its largest batch;
            // the split depends on the system alone
            const int parts = (int)std::min<int64_t>(DEF_PARTS_MAX, std::max<int64_t>(
                1, (DEF_PARTS_ITEMS + std::max<int64_t>(1, r.n_def) - 1) / std::max<int64_t>(1, r.n_def)));
            const int64_t m = std::max<int64_t>(1, r.n_def) * parts;
            uint32_t *def_g = (uint32_t *)scratch(c, s, B_DEFG, sizeof(uint32_t) * m);
            uint32_t *def_b = (uint32_t *)scratch(c, s, B_DEFB, sizeof(uint32_t) * m);
            double *def_eps = (double *)scratch(c, s, B_DEFE, sizeof(double) * m * ns);
            double *def_S = (double *)scratch(c, s, B_DEFS, sizeof(double) * m * ns);
            uint32_t *def_alpha = (uint32_t *)scratch(c, s, B_DEFC, sizeof(uint32_t) * m);
            uint32_t *def_conn = (uint32_t *)scratch(c, s, B_DEFN, sizeof(uint32_t) * m);
            uint64_t *def_fp = (uint64_t *)scratch(c, s, B_DEFF, sizeof(uint64_t) * m);
            double *def_dc = bwd ? (double *)scratch(c, s, B_DEFD, sizeof(double) * m * ns) : nullptr;
            if (!def_g || !def_b || !def_eps || !def_S || !def_alpha || !def_conn || !def_fp || (bwd && !def_dc))
                return fail(c, QP_E_OOM, "device allocation failed (deferred batches)");
            r.dp.eps = def_eps; r.dp.S = def_S; r.dp.alpha = def_alpha; r.dp.conn = def_conn; r.dp.fp = def_fp;
            r.dp.dc = def_dc;
            r.dp.off = r.def_off;
            r.dp.cnt = r.def_cnt_g;
            r.dp.parts = parts;
            if (r.n_def > 0) {
                hipLaunchKernelGGL(def_fill, dim3(grid_for(in[s].n_det)), dim3(256), 0, st, r.def_bits, in[s].n_det,
                                   r.nbw, r.def_off, def_g, def_b);
                // the general kernel on the listed batches: its own slots
                SweepArgs &d = r.d;
                d = r.a;
                d.def_mode = 1;
                d.def_g = def_g; d.def_b = def_b;
                d.def_parts = parts;
                d.n_items = r.n_def * parts;
                d.eps_item = def_eps; d.S_item = def_S; d.cnt_item = def_alpha; d.fp_item = def_fp;
                d.conn_item = def_conn; d.dc_item = def_dc;
                gitems[s] = r.n_def * parts;
            }
        }
    }
    // ------------------------------------------------ phase 4: general kernel
    {
        std::vector<LaunchPlan> plans = plan_launches(c, K_GENERAL, bwd, fp, in, run, gitems);
        int rc = launch_plans(c, K_GENERAL, bwd, fp, plans, run, st);
        if (rc != QP_OK) return rc;
    }
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[3], st));

    // ---------------------------------------------------- phase 5: reductions
    for (int s = 0; s < n_sys; ++s) {
        SysIn &x = in[s];
        SysRun &r = run[s];
        if (x.n_det == 0) continue;
        const int ns = x.ns;
        if (r.swept)
            hipLaunchKernelGGL(reduce_items, dim3(grid_for(r.n_g)), dim3(256), 0, st, r.eps_item, r.S_item,
                               r.cnt_item, fp ? r.fp_item : (const uint64_t *)nullptr, r.conn_item, r.dc_item,
                               r.n_g, r.Q, ns, r.P.perm, (const int32_t *)r.gen_rank, x.n_det, r.eps_g, r.S_g,
                               r.cnt_g, r.fp_g, r.conn_g, r.defa_g, bwd ? nullptr : x.eps_gen,
                               bwd ? x.grad_coefs : nullptr, r.dp);
        if (r.swept && r.split)
            hipLaunchKernelGGL(reduce_lean, dim3(grid_for(r.n_g)), dim3(256), 0, st, r.a.lean_eps, r.a.lean_S,
                               r.a.lean_cnt, r.a.lean_fp, r.a.lean_conn, bwd ? r.a.lean_dc : (const double *)nullptr,
                               r.n_g, r.n_pairs, ns, r.P.perm, (const int32_t *)r.gen_rank, x.n_det, r.eps_g, r.S_g,
                               r.cnt_g, r.fp_g, r.conn_g, bwd ? nullptr : x.eps_gen,
                               bwd ? x.grad_coefs : nullptr, &r.P.sc->clean_total);
        else if (!r.swept && r.n_g > 0)
            hipLaunchKernelGGL(reduce_empty, dim3(grid_for(r.n_g)), dim3(256), 0, st, r.n_g, ns, r.P.perm,
                               (const int32_t *)r.gen_rank, x.n_det, r.eps_g, r.S_g, r.cnt_g, r.fp_g, r.conn_g,
                               r.defa_g, bwd ? nullptr : x.eps_gen);
        const int64_t n_cells = r.n_g * cells_per_generator(x.I.n, r.P.nup, r.P.ndn);
        hipLaunchKernelGGL(reduce_total, dim3(1), dim3(256), 0, st, r.eps_g, r.S_g, r.cnt_g, r.fp_g, r.conn_g,
                           r.defa_g, r.n_g, ns, x.e_pt2, x.stats, r.P.sc, n_cells, x.gup,
                           bwd ? x.grad_E0 : nullptr, x.E0);
        HIPCHK(c, hipGetLastError());
    }

    // ----------------------------------------------------- phase 6: selection
    if (!bwd) {
        bool sel = false;
        for (int s = 0; s < n_sys; ++s) {
            SysRun &r = run[s];
            if (in[s].n_det == 0 || in[s].n_select <= 0) continue;
            sel = true;
            int32_t *comp = (int32_t *)scratch(c, s, B_COMP, sizeof(int32_t) * r.cand_cap);
            if (!comp) return fail(c, QP_E_OOM, "device allocation failed (selection)");
            hipLaunchKernelGGL(sel_compact, dim3(grid_for(r.cand_cap, 256, 8192)), dim3(256), 0, st, r.cand, r.P.sc,
                               r.cand_cap, comp, r.P.sc);
            HIPCHK(c, hipMemcpyAsync(c->host_sc + s, r.P.sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
        }
        if (sel) {
            HIPCHK(c, hipStreamSynchronize(st));
            for (int s = 0; s < n_sys; ++s) {
                SysIn &x = in[s];
                SysRun &r = run[s];
                if (x.n_det == 0 || x.n_select <= 0) continue;
                const Scalars hs = c->host_sc[s];
                if (hs.overflow & 1ull) return fail(c, QP_E_OVERFLOW, "selection candidate buffer overflowed");
                const int64_t M = (int64_t)hs.comp_count;
                const int64_t m = std::min<int64_t>(M, x.n_select);
                const int64_t PP = pow2_at_least(std::max<int64_t>(M, 1));
                const int nint = r.nint;
                int32_t *comp = (int32_t *)scratch(c, s, B_COMP, sizeof(int32_t) * r.cand_cap);
                uint64_t *skey = (uint64_t *)scratch(c, s, B_SKEY, sizeof(uint64_t) * PP);
                uint64_t *sbits = (uint64_t *)scratch(c, s, B_SBITS, sizeof(uint64_t) * PP * 2 * nint);
                int32_t *sidx = (int32_t *)scratch(c, s, B_SIDX, sizeof(int32_t) * PP);
                if (!comp || !skey || !sbits || !sidx) return fail(c, QP_E_OOM, "device allocation failed (selection sort)");
                switch (nint) {
#define SELCASE(NI)                                                                                        \
    case NI:                                                                                               \
        hipLaunchKernelGGL(sel_materialise<NI>, dim3(grid_for(PP)), dim3(256), 0, st, r.cand, comp, M, x.dets, \
                           r.P.perm, skey, sbits, PP, sidx);                                               \
        bitonic_sort(sidx, PP, SelCmp<NI>{skey, sbits}, st);                                              \
        hipLaunchKernelGGL(sel_output<NI>, dim3(grid_for(std::max<int64_t>(m, 1))), dim3(256), 0, st, r.cand, comp, \
                           sidx, m, x.ns, sbits, skey, x.sel_dets, x.sel_e, x.sel_key, x.n_sel);          \
        break;
                    SELCASE(1) SELCASE(2) SELCASE(3) SELCASE(4)
#undef SELCASE
                default: break;
                }
                HIPCHK(c, hipGetLastError());
            }
        }
    }
    if (c->timing) {
        HIPCHK(c, hipEventRecord(c->ev[4], st));
        c->timed = true;
    }
    return QP_OK;
}

// W = H U (or S^2 U) for n_vec vectors [n_vec][n_det], over a prepared Psi
void launch_sigma(const DevInts &I, const Prepared &P, const uint64_t *dets, int64_t n_det, int n_vec, bool s2,
                  const double *U, double *W, hipStream_t st)
{
    const double sz = 0.5 * (P.nup - P.ndn);
    const int grid = grid_for(n_det, 64, 1 << 20);
    switch (P.nint) {
#define SIGCASE(NI)                                                                                        \
    case NI:                                                                                               \
        if (s2) hipLaunchKernelGGL((sigma_rows<NI, true>), dim3(grid), dim3(64), 0, st, I, dets, P.perm, P.HII, \
                                   P.coff, P.cent, n_det, n_vec, sz, U, W);                                \
        else hipLaunchKernelGGL((sigma_rows<NI, false>), dim3(grid), dim3(64), 0, st, I, dets, P.perm, P.HII, \
                                P.coff, P.cent, n_det, n_vec, sz, U, W);                                   \
        break;
        SIGCASE(1) SIGCASE(2) SIGCASE(3) SIGCASE(4)
#undef SIGCASE
    default: break;
    }
}

// eigen-decomposition of a small symmetric matrix a [m][m] (destroyed) by
// cyclic Jacobi rotations; eigenvalues ascending in w, vectors in columns of v
void jacobi_eigen(std::vector<double> &a, int m, std::vector<double> &w, std::vector<double> &v)
{
    v.assign((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) v[(size_t)i * m + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j) {
                const double x = a[(size_t)i * m + j] * a[(size_t)i * m + j];
                tot += x;
                if (i != j) off += x;
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int p = 0; p < m; ++p)
            for (int q = p + 1; q < m; ++q) {
                const double apq = a[(size_t)p * m + q];
                if (apq == 0.0) continue;
                const double app = a[(size_t)p * m + p], aqq = a[(size_t)q * m + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < m; ++k) {
                    const double akp = a[(size_t)k * m + p], akq = a[(size_t)k * m + q];
                    a[(size_t)k * m + p] = cs * akp - sn * akq;
                    a[(size_t)k * m + q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < m; ++k) {
                    const double apk = a[(size_t)p * m + k], aqk = a[(size_t)q * m + k];
                    a[(size_t)p * m + k] = cs * apk - sn * aqk;
                    a[(size_t)q * m + k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < m; ++k) {
                    const double vkp = v[(size_t)k * m + p], vkq = v[(size_t)k * m + q];
                    v[(size_t)k * m + p] = cs * vkp - sn * vkq;
                    v[(size_t)k * m + q] = sn * vkp + cs * vkq;
                }
            }
    }
    std::vector<int> idx(m);
    for (int i = 0; i < m; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int x, int y) { return a[(size_t)x * m + x] < a[(size_t)y * m + y]; });
    std::vector<double> v2((size_t)m * m);
    w.resize(m);
    for (int j = 0; j < m; ++j) {
        w[j] = a[(size_t)idx[j] * m + idx[j]];
        for (int k = 0; k < m; ++k) v2[(size_t)k * m + j] = v[(size_t)k * m + idx[j]];
    }
    v.swap(v2);
}


}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

// ===========================================================================
// ALU issue-rate probe: eight independent chains per lane of one VALU
// instruction each (written in asm so that every op is exactly one
// instruction), enough waves per SIMD to hide the chains' latency
// ===========================================================================

#define PROBE_FMA(a) asm volatile("v_fma_f64 %0, %1, %2, %0" : "+v"(a) : "v"(b), "v"(cc))
#define PROBE_ADD(x) asm volatile("v_add_u32 %0, %1, %0" : "+v"(x) : "v"(y))

template <int KIND>
__global__ __launch_bounds__(256) void alu_probe(int64_t iters, double *sink)
{
    const double b = 1.0 - 0x1p-40, cc = 0x1p-40;
    const uint32_t y = blockIdx.x | 1u;
    double a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5, a6 = a0 + 6,
           a7 = a0 + 7;
    uint32_t x0 = threadIdx.x, x1 = x0 + 1, x2 = x0 + 2, x3 = x0 + 3, x4 = x0 + 4, x5 = x0 + 5, x6 = x0 + 6,
             x7 = x0 + 7;
    for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            if (KIND != 1) {
                PROBE_FMA(a0); PROBE_FMA(a1); PROBE_FMA(a2); PROBE_FMA(a3);
                PROBE_FMA(a4); PROBE_FMA(a5); PROBE_FMA(a6); PROBE_FMA(a7);
            }
            if (KIND != 0) {
                PROBE_ADD(x0); PROBE_ADD(x1); PROBE_ADD(x2); PROBE_ADD(x3);
                PROBE_ADD(x4); PROBE_ADD(x5); PROBE_ADD(x6); PROBE_ADD(x7);
            }
        }
    }
    const double s = a0 + a1 + a2 + a3 + a4 + a5 + a6 + a7;
    const uint32_t t = x0 ^ x1 ^ x2 ^ x3 ^ x4 ^ x5 ^ x6 ^ x7;
    if (s == -1.0 && t == 0x5a5a5a5au) sink[0] = s;   // never true; keeps the chains' results live
}

#undef PROBE_FMA
#undef PROBE_ADD

extern "C" {

// ---------------------------------------------------------------- no-allocation generator order
// The scratch of qp_generator_order_noalloc: the weights sum_k c_Ik^2 of up to
// QP_NOALLOC_MAX_DET determinants, then their index array (padded to a power
// of two for the sort).  Each GPU holds its own copy, at its own address,
// until the process ends; host code reaches it only through the address that
// hipGetSymbolAddress gives for that device (the array's name is a host-side
// stand-in).
static __device__ __align__(256) unsigned char noalloc_scratch[(size_t)QP_NOALLOC_MAX_DET * (8 + 4)];

static std::mutex noalloc_mu;
static void *noalloc_ptr[64] = {};   // per device ordinal

// the array's address on `device`, which must be current; taken once per device
static void *noalloc_setup(int device)
{
    std::lock_guard<std::mutex> lock(noalloc_mu);
    if (device < 0 || device >= 64) return nullptr;
    if (!noalloc_ptr[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch)) != hipSuccess) return nullptr;
        noalloc_ptr[device] = p;
    }
    return noalloc_ptr[device];
}

int qp_create(qp_ctx **ctx, int device)
{
    if (!ctx) return QP_E_ARG;
    *ctx = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return QP_E_HIP;
    qp_ctx *c = new qp_ctx();
    c->device = device;
    if (hipSetDevice(device) != hipSuccess) { delete c; return QP_E_HIP; }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0) {
        c->num_cu = prop.multiProcessorCount;
        if (prop.maxSharedMemoryPerMultiProcessor > 0) c->lds_per_cu = prop.maxSharedMemoryPerMultiProcessor;
    }
    if (hipHostMalloc((void **)&c->host_sc, sizeof(Scalars), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&c->host_det0, sizeof(uint64_t) * 2 * QPD_MAX_NINT, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&c->host_maxc2, sizeof(double) * QPD_MAX_STATES, hipHostMallocDefault) != hipSuccess) {
        qp_destroy(c);
        return QP_E_HIP;
    }
    c->host_sc_n = 1;
    c->noalloc = noalloc_setup(device);
    if (!c->noalloc) {
        qp_destroy(c);
        return QP_E_HIP;
    }
    *ctx = c;
    return QP_OK;
}

void qp_destroy(qp_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    for (auto &v : c->slots)
        for (auto &b : v) if (b.p) (void)hipFree(b.p);
    for (auto &b : c->args) if (b.p) (void)hipFree(b.p);
    if (c->defn.p) (void)hipFree(c->defn.p);
    if (c->probe_sink) (void)hipFree(c->probe_sink);
    for (auto &e : c->ev) if (e) (void)hipEventDestroy(e);
    double *arrs[] = {c->h, c->X, c->Y, c->Cj, c->CXj, c->Jm, c->Km, c->JK};
    for (double *p : arrs) if (p) (void)hipFree(p);
    if (c->host_sc) (void)hipHostFree(c->host_sc);
    if (c->host_det0) (void)hipHostFree(c->host_det0);
    if (c->host_maxc2) (void)hipHostFree(c->host_maxc2);
    if (c->host_stage) (void)hipHostFree(c->host_stage);
    delete c;
}

const char *qp_last_error(const qp_ctx *c)
{
    return c ? c->err.c_str() : "null context";
}

int qp_set_integrals(qp_ctx *c, const double *h, const double *eri_packed, int n_orb, void *stream)
{
    if (!c) return QP_E_ARG;
    c->err.clear();
    if (!h || !eri_packed) return fail(c, QP_E_ARG, "null integral pointer");
    if (n_orb < 1 || n_orb > QP_MAX_ORB) return fail(c, QP_E_NORB, "n_orb must be in [1,256]");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(c, hipStreamSynchronize(st));
    ++c->ints_gen;
    double **arrs[] = {&c->h, &c->X, &c->Y, &c->Cj, &c->CXj, &c->Jm, &c->Km, &c->JK};
    for (double **p : arrs) if (*p) { (void)hipFree(*p); *p = nullptr; }
    c->n = 0;
    const LayoutSizes z = layout_sizes(n_orb);
    if (hipMalloc(&c->X, z.nX * 8) != hipSuccess || hipMalloc(&c->Y, z.nY * 8) != hipSuccess ||
        hipMalloc(&c->Cj, z.n3 * 8) != hipSuccess || hipMalloc(&c->CXj, z.n3 * 8) != hipSuccess ||
        hipMalloc(&c->Jm, z.n2 * 8) != hipSuccess || hipMalloc(&c->Km, z.n2 * 8) != hipSuccess ||
        hipMalloc(&c->JK, z.n2 * 8) != hipSuccess || hipMalloc(&c->h, z.n2 * 8) != hipSuccess) {
        (void)hipGetLastError();
        for (double **p : arrs) if (*p) { (void)hipFree(*p); *p = nullptr; }
        return fail(c, QP_E_OOM, "device allocation failed (integral layouts)");
    }
    DevInts I = dev_ints(c);
    I.n = n_orb;
    launch_layouts(h, eri_packed, n_orb, I, st);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(st));
    c->n = n_orb;
    return QP_OK;
}

int qp_pt2(qp_ctx *c, const uint64_t *dets, const double *coefs, int64_t n_det, int n_states, const double *E0,
           int64_t n_select, int flags, double *e_pt2, uint64_t *sel_dets, double *sel_e, int64_t *n_sel,
           qp_pt2_stats *stats, double *eps_gen, void *stream)
{
    int rc = common_checks(c, dets, coefs, n_det, n_states, E0);
    if (rc != QP_OK) return rc;
    if (!e_pt2) return fail(c, QP_E_ARG, "e_pt2 is required");
    if (n_select < 0) return fail(c, QP_E_ARG, "n_select < 0");
    if (n_select > 0 && (!sel_dets || !sel_e || !n_sel)) return fail(c, QP_E_ARG, "selection outputs required");
    if (n_select > (int64_t)INT32_MAX / 4) return fail(c, QP_E_ARG, "n_select too large");
    std::vector<SysIn> in(1);
    SysIn &x = in[0];
    memset(&x, 0, sizeof(x));
    x.I = dev_ints(c);
    x.dets = dets; x.coefs = coefs; x.n_det = n_det; x.ns = n_states; x.E0 = E0;
    x.n_select = n_select; x.e_pt2 = e_pt2; x.sel_dets = sel_dets; x.sel_e = sel_e; x.n_sel = n_sel;
    x.stats = stats; x.eps_gen = eps_gen;
    return run_sweeps(c, in, flags, false, (hipStream_t)stream);
}

int qp_pt2_backward(qp_ctx *c, const uint64_t *dets, const double *coefs, int64_t n_det, int n_states,
                    const double *E0, const double *grad_e_pt2, int flags, double *grad_coefs, double *grad_E0,
                    double *grad_h, qp_pt2_stats *stats, void *stream)
{
    int rc = common_checks(c, dets, coefs, n_det, n_states, E0);
    if (rc != QP_OK) return rc;
    if (!grad_e_pt2) return fail(c, QP_E_ARG, "grad_e_pt2 is required");
    std::vector<SysIn> in(1);
    SysIn &x = in[0];
    memset(&x, 0, sizeof(x));
    x.I = dev_ints(c);
    x.dets = dets; x.coefs = coefs; x.n_det = n_det; x.ns = n_states; x.E0 = E0;
    x.stats = stats; x.gup = grad_e_pt2;
    x.grad_coefs = grad_coefs; x.grad_E0 = grad_E0; x.grad_h = grad_h;
    return run_sweeps(c, in, flags, true, (hipStream_t)stream);
}

int qp_generator_order(qp_ctx *c, const uint64_t *dets, const double *coefs, int64_t n_det, int n_states,
                       int flags, int32_t *order_out, void *stream)
{
    int rc = common_checks(c, dets, coefs, n_det, n_states, coefs);
    if (rc != QP_OK) return rc;
    if (n_det > 0 && !order_out) return fail(c, QP_E_ARG, "order_out is required");
    if (n_det == 0) return QP_OK;
    hipStream_t st = (hipStream_t)stream;
    Prepared P;
    rc = prepare(c, 0, dev_ints(c), dets, coefs, n_det, n_states, flags, st, P);
    if (rc != QP_OK) return rc;
    HIPCHK(c, hipMemcpyAsync(order_out, P.perm, sizeof(int32_t) * n_det, hipMemcpyDeviceToDevice, st));
    return QP_OK;
}

int qp_generator_order_noalloc(qp_ctx *c, const uint64_t *dets, const double *coefs, int64_t n_det,
                               int n_states, int flags, int32_t *order_out, void *stream)
{
    (void)flags;
    int rc = common_checks(c, dets, coefs, n_det, n_states, coefs);
    if (rc != QP_OK) return rc;
    if (n_det > 0 && !order_out) return fail(c, QP_E_ARG, "order_out is required");
    if (n_det > QP_NOALLOC_MAX_DET) return fail(c, QP_E_ARG, "n_det exceeds QP_NOALLOC_MAX_DET");
    if (n_det == 0) return QP_OK;
    if (!c->noalloc) return fail(c, QP_E_HIP, "no-allocation scratch unavailable");
    hipStream_t st = (hipStream_t)stream;
    const int64_t Pw = pow2_at_least(n_det);   // <= QP_NOALLOC_MAX_DET, a power of two
    double *w = (double *)c->noalloc;
    int32_t *idx = (int32_t *)((unsigned char *)c->noalloc + sizeof(double) * QP_NOALLOC_MAX_DET);
    // the same kernels as the ordering inside every sweep: every entry the sort
    // reads is written first (weights of the determinants, indices with -1
    // padding), so nothing of an earlier call's contents is used
    hipLaunchKernelGGL(gen_weights, dim3(grid_for(Pw)), dim3(256), 0, st, coefs, n_det, n_states, w, Pw, idx);
    switch ((c->n - 1) / 64 + 1) {
    case 1: bitonic_sort(idx, Pw, GenCmp<1>{w, dets}, st); break;
    case 2: bitonic_sort(idx, Pw, GenCmp<2>{w, dets}, st); break;
    case 3: bitonic_sort(idx, Pw, GenCmp<3>{w, dets}, st); break;
    default: bitonic_sort(idx, Pw, GenCmp<4>{w, dets}, st); break;
    }
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(order_out, idx, sizeof(int32_t) * n_det, hipMemcpyDeviceToDevice, st));
    return QP_OK;
}

int qp_pt2_generators(qp_ctx *c, const uint64_t *dets, const double *coefs, int64_t n_det, int n_states,
                      const double *E0, const int32_t *gens, int64_t n_gen, int64_t n_select, int flags,
                      double *eps_out, uint64_t *sel_dets, double *sel_e, int64_t *n_sel, qp_pt2_stats *stats,
                      void *stream)
{
    int rc = common_checks(c, dets, coefs, n_det, n_states, E0);
    if (rc != QP_OK) return rc;
    if (n_gen < 0 || n_gen > n_det) return fail(c, QP_E_ARG, "n_gen must be in [0, n_det]");
    if (n_gen > 0 && (!gens || !eps_out)) return fail(c, QP_E_ARG, "gens and eps_out are required");
    if (n_select < 0) return fail(c, QP_E_ARG, "n_select < 0");
    if (n_select > 0 && (!sel_dets || !sel_e || !n_sel)) return fail(c, QP_E_ARG, "selection outputs required");
    if (n_select > (int64_t)INT32_MAX / 4) return fail(c, QP_E_ARG, "n_select too large");
    std::vector<SysIn> in(1);
    SysIn &x = in[0];
    memset(&x, 0, sizeof(x));
    x.I = dev_ints(c);
    x.dets = dets; x.coefs = coefs; x.n_det = n_det; x.ns = n_states; x.E0 = E0;
    x.gens = gens; x.n_gen = n_gen;
    x.n_select = n_select; x.sel_dets = sel_dets; x.sel_e = sel_e; x.n_sel = n_sel;
    x.stats = stats; x.eps_gen = eps_out;
    return run_sweeps(c, in, flags, false, (hipStream_t)stream);
}

int qp_pt2_stochastic(qp_ctx *c, const uint64_t *dets, const double *coefs, int64_t n_det, int n_states,
                      const double *E0, const double *uniforms, int64_t n_uniforms, double rel_err,
                      int64_t det_chunk, int64_t draws_per_round, int64_t n_select, int flags, double *e_est,
                      double *e_err, int64_t *n_computed, int64_t *n_rounds, uint64_t *sel_dets, double *sel_e,
                      int64_t *n_sel, uint8_t *computed_out, void *stream)
{
    int rc = common_checks(c, dets, coefs, n_det, n_states, E0);
    if (rc != QP_OK) return rc;
    if (!e_est || !e_err || !n_computed || !n_rounds) return fail(c, QP_E_ARG, "outputs are required");
    if (n_uniforms < 0 || (n_uniforms > 0 && !uniforms)) return fail(c, QP_E_ARG, "bad uniform list");
    if (det_chunk < 1 || draws_per_round < 0 || !(rel_err >= 0.0)) return fail(c, QP_E_ARG, "bad schedule");
    if (n_select < 0) return fail(c, QP_E_ARG, "n_select < 0");
    if (n_select > 0 && (!sel_dets || !sel_e || !n_sel)) return fail(c, QP_E_ARG, "selection outputs required");
    if (n_select > (int64_t)INT32_MAX / 4) return fail(c, QP_E_ARG, "n_select too large");
    const int ns = n_states;
    for (int k = 0; k < ns; ++k) { e_est[k] = 0.0; e_err[k] = 0.0; }
    *n_computed = 0;
    *n_rounds = 0;
    hipStream_t st = (hipStream_t)stream;
    if (n_det == 0) {
        if (n_select > 0) {
            HIPCHK(c, hipMemsetAsync(n_sel, 0, sizeof(int64_t), st));
            HIPCHK(c, hipStreamSynchronize(st));
        }
        return QP_OK;
    }
    // on-the-fly selection: every round also selects the top n_select alpha
    // owned by its generators (with the criterion keys the kernels computed);
    // the rounds' generators partition the computed ones, so merging the
    // rounds' lists and keeping the first n_select gives the selection over
    // all computed generators, in the same order as one sweep of them
    const int nint = (c->n + 63) / 64;
    const int64_t dw = 2 * nint;
    std::vector<uint64_t> mkey, mdet, rkey_h, rdet_h, tkey, tdet;
    std::vector<double> me, re_h, te;
    uint64_t *rdet = nullptr, *rkey = nullptr;
    double *re = nullptr;
    int64_t *rn = nullptr;
    if (n_select > 0) {
        rdet = (uint64_t *)scratch(c, 0, B_RSDET, sizeof(uint64_t) * n_select * dw);
        re = (double *)scratch(c, 0, B_RSE, sizeof(double) * n_select * ns);
        rkey = (uint64_t *)scratch(c, 0, B_RSKEY, sizeof(uint64_t) * n_select);
        rn = (int64_t *)scratch(c, 0, B_RSN, sizeof(int64_t));
        if (!rdet || !re || !rkey || !rn) return fail(c, QP_E_OOM, "device allocation failed (stochastic selection)");
        rdet_h.resize((size_t)n_select * dw);
        re_h.resize((size_t)n_select * ns);
        rkey_h.resize((size_t)n_select);
    }
    // a before b in the selection order: larger key, then smaller bit string
    // (each spin's words from the highest)
    auto before = [&](uint64_t ka, const uint64_t *da, uint64_t kb, const uint64_t *db) {
        if (ka != kb) return ka > kb;
        for (int sp = 0; sp < 2; ++sp)
            for (int w = nint - 1; w >= 0; --w) {
                const uint64_t x = da[sp * nint + w], y = db[sp * nint + w];
                if (x != y) return x < y;
            }
        return false;
    };
    // generator order and weights w_r = sum_k c_k(det of rank r)^2
    std::vector<int32_t> perm(n_det);
    std::vector<double> ch((size_t)ns * n_det);
    // prepared once: every round sweeps a list of generators of the same inputs
    Prepared P;
    {
        rc = prepare(c, 0, dev_ints(c), dets, coefs, n_det, ns, flags, st, P);
        if (rc != QP_OK) return rc;
        HIPCHK(c, hipMemcpyAsync(perm.data(), P.perm, sizeof(int32_t) * n_det, hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipMemcpyAsync(ch.data(), coefs, sizeof(double) * ns * n_det, hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
    }
    std::vector<double> w(n_det), cum(n_det), tail(n_det + 1, 0.0);
    double run = 0.0;
    for (int64_t r = 0; r < n_det; ++r) {
        double v = 0.0;
        for (int k = 0; k < ns; ++k) {
            const double x = ch[(size_t)k * n_det + perm[r]];
            v += x * x;
        }
        w[r] = v;
        run += v;
        cum[r] = run;
    }
    for (int64_t r = n_det - 1; r >= 0; --r) tail[r] = tail[r + 1] + w[r];   // weight of ranks >= r
    const double W = run;
    // memoised eps_r,k, the draw log, and the deterministic prefix [0, d)
    std::vector<double> eps((size_t)n_det * ns, 0.0);
    std::vector<char> done(n_det, 0), queued(n_det, 0);   // queued: in this round's list
    std::vector<int64_t> draws;
    int64_t d = 0, next_u = 0, computed = 0, rounds = 0;
    std::vector<double> det_sum(ns, 0.0);
    int32_t *dgen = (int32_t *)scratch(c, 0, B_ROW, sizeof(int32_t) * n_det);
    double *deps = (double *)scratch(c, 0, B_C2, sizeof(double) * n_det * ns);
    int32_t *hgen = nullptr;
    double *heps = nullptr;
    if (!dgen || !deps) return fail(c, QP_E_OOM, "device allocation failed (stochastic driver)");
    if (hipHostMalloc((void **)&hgen, sizeof(int32_t) * n_det, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&heps, sizeof(double) * n_det * ns, hipHostMallocDefault) != hipSuccess) {
        if (hgen) (void)hipHostFree(hgen);
        return fail(c, QP_E_OOM, "pinned host allocation failed (stochastic driver)");
    }
    auto cleanup = [&]() { (void)hipHostFree(hgen); (void)hipHostFree(heps); };
    std::vector<int64_t> todo;
    for (;;) {
        // one round: the deterministic prefix grows by det_chunk generators and
        // draws_per_round generators are drawn with probability w_r / W
        todo.clear();
        const int64_t d_new = std::min<int64_t>(n_det, d + det_chunk);
        for (int64_t r = d; r < d_new; ++r)
            if (!done[r]) { todo.push_back(r); queued[r] = 1; }
        int64_t drawn = 0;
        while (drawn < draws_per_round && next_u < n_uniforms && W > 0.0) {
            const double t = uniforms[next_u++] * W;
            int64_t r = std::upper_bound(cum.begin(), cum.end(), t) - cum.begin();
            if (r >= n_det) r = n_det - 1;
            draws.push_back(r);
            ++drawn;
            if (r >= d_new && !done[r] && !queued[r]) { todo.push_back(r); queued[r] = 1; }
        }
        if (!todo.empty()) {
            for (size_t i = 0; i < todo.size(); ++i) hgen[i] = perm[todo[i]];
            const int64_t m = (int64_t)todo.size();
            HIPCHK(c, hipMemcpyAsync(dgen, hgen, sizeof(int32_t) * m, hipMemcpyHostToDevice, st));
            std::vector<SysIn> in(1);
            SysIn &x = in[0];
            memset(&x, 0, sizeof(x));
            x.I = dev_ints(c);
            x.dets = dets; x.coefs = coefs; x.n_det = n_det; x.ns = ns; x.E0 = E0;
            x.gens = dgen; x.n_gen = m; x.eps_gen = deps;
            x.pre = &P;
            if (n_select > 0) {
                x.n_select = n_select; x.sel_dets = rdet; x.sel_e = re; x.n_sel = rn; x.sel_key = rkey;
                // once n_select alpha are held, an alpha whose key is below the
                // last one's can no longer enter: the round starts its
                // threshold at the lower edge of that key's histogram bin
                if ((int64_t)mkey.size() == n_select) x.sel_floor_bin = key_bin_host(mkey.back());
            }
            rc = run_sweeps(c, in, flags | QP_FLAG_NOCHECK, false, st);
            if (rc != QP_OK) { cleanup(); return rc; }
            HIPCHK(c, hipMemcpyAsync(heps, deps, sizeof(double) * m * ns, hipMemcpyDeviceToHost, st));
            int64_t rcount = 0;
            if (n_select > 0) {
                HIPCHK(c, hipMemcpyAsync(&rcount, rn, sizeof(int64_t), hipMemcpyDeviceToHost, st));
                HIPCHK(c, hipMemcpyAsync(rdet_h.data(), rdet, sizeof(uint64_t) * n_select * dw, hipMemcpyDeviceToHost, st));
                HIPCHK(c, hipMemcpyAsync(re_h.data(), re, sizeof(double) * n_select * ns, hipMemcpyDeviceToHost, st));
                HIPCHK(c, hipMemcpyAsync(rkey_h.data(), rkey, sizeof(uint64_t) * n_select, hipMemcpyDeviceToHost, st));
            }
            HIPCHK(c, hipStreamSynchronize(st));
            for (int64_t i = 0; i < m; ++i) {
                const int64_t r = todo[i];
                for (int k = 0; k < ns; ++k) eps[(size_t)r * ns + k] = heps[(size_t)k * m + i];
                done[r] = 1;
                queued[r] = 0;
            }
            computed += m;
            if (n_select > 0 && rcount > 0) {
                // merge the round's sorted list into the running one, keep n_select
                const int64_t a_n = (int64_t)mkey.size(), tot = std::min<int64_t>(a_n + rcount, n_select);
                tkey.resize(tot);
                tdet.resize((size_t)tot * dw);
                te.resize((size_t)tot * ns);
                int64_t ia = 0, ib = 0;
                for (int64_t o = 0; o < tot; ++o) {
                    const bool take_a = ib >= rcount ||
                                        (ia < a_n && before(mkey[ia], &mdet[(size_t)ia * dw], rkey_h[ib],
                                                            &rdet_h[(size_t)ib * dw]));
                    const uint64_t *kd = take_a ? &mdet[(size_t)ia * dw] : &rdet_h[(size_t)ib * dw];
                    const double *ke = take_a ? &me[(size_t)ia * ns] : &re_h[(size_t)ib * ns];
                    tkey[o] = take_a ? mkey[ia] : rkey_h[ib];
                    std::copy(kd, kd + dw, &tdet[(size_t)o * dw]);
                    std::copy(ke, ke + ns, &te[(size_t)o * ns]);
                    if (take_a) ++ia; else ++ib;
                }
                mkey.swap(tkey);
                mdet.swap(tdet);
                me.swap(te);
            }
        }
        for (int64_t r = d; r < d_new; ++r)
            for (int k = 0; k < ns; ++k) det_sum[k] += eps[(size_t)r * ns + k];
        d = d_new;
        ++rounds;
        // estimate: the prefix exactly, the rest by the draws that fall in it,
        // each weighted by W_S / w_r (W_S the weight of the rest)
        bool converged = true;
        if (d == n_det) {
            for (int k = 0; k < ns; ++k) { e_est[k] = det_sum[k]; e_err[k] = 0.0; }
        } else {
            const double WS = tail[d];
            int64_t mS = 0;
            for (int64_t r : draws) mS += r >= d;
            for (int k = 0; k < ns; ++k) {
                double mean = 0.0, m2 = 0.0;
                int64_t j = 0;
                for (int64_t r : draws) {
                    if (r < d) continue;
                    const double y = WS * eps[(size_t)r * ns + k] / w[r];
                    ++j;
                    const double dlt = y - mean;
                    mean += dlt / (double)j;
                    m2 += dlt * (y - mean);
                }
                e_est[k] = det_sum[k] + (mS > 0 ? mean : 0.0);
                e_err[k] = mS > 1 ? std::sqrt(m2 / (double)(mS - 1) / (double)mS) : HUGE_VAL;
                if (!(mS > 1 && e_err[k] <= rel_err * std::fabs(e_est[k]))) converged = false;
            }
        }
        // stop when every state meets the relative error, when the prefix
        // covers every generator, or when the random numbers run out
        if (d == n_det || converged) break;
        if (draws_per_round > 0 && next_u >= n_uniforms) break;
    }
    cleanup();
    *n_computed = computed;
    *n_rounds = rounds;
    if (n_select > 0) {
        // the merged selection, and the computed flags, to the caller's device
        // arrays; the host vectors live until the copies end
        const int64_t msel = (int64_t)mkey.size();
        if (msel > 0) {
            HIPCHK(c, hipMemcpyAsync(sel_dets, mdet.data(), sizeof(uint64_t) * msel * dw, hipMemcpyHostToDevice, st));
            HIPCHK(c, hipMemcpyAsync(sel_e, me.data(), sizeof(double) * msel * ns, hipMemcpyHostToDevice, st));
        }
        HIPCHK(c, hipMemcpyAsync(n_sel, &msel, sizeof(int64_t), hipMemcpyHostToDevice, st));
        HIPCHK(c, hipStreamSynchronize(st));
    }
    if (computed_out) {
        // 1 for every determinant whose eps was computed, in the caller's order
        std::vector<uint8_t> fl((size_t)n_det, 0);
        for (int64_t r = 0; r < n_det; ++r)
            if (done[r]) fl[(size_t)perm[r]] = 1;
        HIPCHK(c, hipMemcpyAsync(computed_out, fl.data(), (size_t)n_det, hipMemcpyHostToDevice, st));
        HIPCHK(c, hipStreamSynchronize(st));
    }
    return QP_OK;
}

int qp_pt2_batched(qp_ctx *c, int n_sys, const qp_system *sys, int with_backward, int flags, void *stream)
{
    if (!c) return QP_E_ARG;
    c->err.clear();
    if (n_sys < 0 || (n_sys > 0 && !sys)) return fail(c, QP_E_ARG, "bad system list");
    if (n_sys > QP_MAX_SYSTEMS) return fail(c, QP_E_ARG, "too many systems");
    for (int s = 0; s < n_sys; ++s) {
        const qp_system &y = sys[s];
        const std::string who = "system " + std::to_string(s) + ": ";
        if (y.n_orb < 1 || y.n_orb > QP_MAX_ORB) return fail(c, QP_E_NORB, who + "n_orb must be in [1,256]");
        if (!y.h || !y.eri_packed) return fail(c, QP_E_ARG, who + "null integral pointer");
        int rc = check_system(c, y.n_orb, y.dets, y.coefs, y.n_det, y.n_states, y.E0);
        if (rc != QP_OK) { c->err = who + c->err; return rc; }
        if (!y.e_pt2) return fail(c, QP_E_ARG, who + "e_pt2 is required");
        if (y.n_select < 0) return fail(c, QP_E_ARG, who + "n_select < 0");
        if (y.n_select > 0 && with_backward) return fail(c, QP_E_ARG, who + "no selection with the adjoint sweep");
        if (y.n_select > 0 && (!y.sel_dets || !y.sel_e || !y.n_sel))
            return fail(c, QP_E_ARG, who + "selection outputs required");
        if (y.n_select > (int64_t)INT32_MAX / 4) return fail(c, QP_E_ARG, who + "n_select too large");
        if (with_backward && !y.grad_e_pt2) return fail(c, QP_E_ARG, who + "grad_e_pt2 is required");
    }
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    if ((int)c->layout_keys.size() < n_sys) c->layout_keys.resize(n_sys);
    std::vector<SysIn> in(n_sys);
    for (int s = 0; s < n_sys; ++s) {
        const qp_system &y = sys[s];
        SysIn &x = in[s];
        memset(&x, 0, sizeof(x));
        // the system's integral layouts, in its own slot
        const LayoutSizes z = layout_sizes(y.n_orb);
        DevInts I;
        I.n = y.n_orb;
        I.X = (double *)scratch(c, s, B_LX, z.nX * 8);
        I.Y = (double *)scratch(c, s, B_LY, z.nY * 8);
        I.Cj = (double *)scratch(c, s, B_LCJ, z.n3 * 8);
        I.CXj = (double *)scratch(c, s, B_LXJ, z.n3 * 8);
        I.Jm = (double *)scratch(c, s, B_LJM, z.n2 * 8);
        I.Km = (double *)scratch(c, s, B_LKM, z.n2 * 8);
        I.JK = (double *)scratch(c, s, B_LJK, z.n2 * 8);
        I.h = (double *)scratch(c, s, B_LH, z.n2 * 8);
        if (!I.X || !I.Y || !I.Cj || !I.CXj || !I.Jm || !I.Km || !I.JK || !I.h)
            return fail(c, QP_E_OOM, "device allocation failed (integral layouts)");
        LayoutKey &key = c->layout_keys[s];
        const bool same = key.h == y.h && key.eri == y.eri_packed && key.n == y.n_orb;
        if (!((flags & QP_FLAG_REUSE_INTEGRALS) && same)) {
            key = LayoutKey{};
            launch_layouts(y.h, y.eri_packed, y.n_orb, I, st);
            HIPCHK(c, hipGetLastError());
            key.h = y.h; key.eri = y.eri_packed; key.n = y.n_orb;
        }
        x.I = I;
        x.dets = y.dets; x.coefs = y.coefs; x.n_det = y.n_det; x.ns = y.n_states; x.E0 = y.E0;
        x.n_select = y.n_select; x.e_pt2 = y.e_pt2; x.sel_dets = y.sel_dets; x.sel_e = y.sel_e; x.n_sel = y.n_sel;
        x.stats = y.stats; x.eps_gen = with_backward ? nullptr : y.eps_gen;
        if (with_backward) {
            x.gup = y.grad_e_pt2;
            x.grad_coefs = y.grad_coefs; x.grad_E0 = y.grad_E0; x.grad_h = y.grad_h;
        }
    }
    return run_sweeps(c, in, flags & ~QP_FLAG_REUSE_INTEGRALS, with_backward != 0, st);
}

int qp_sigma(qp_ctx *c, const uint64_t *dets, int64_t n_det, int n_vec, const double *U, int flags, double *W,
             void *stream)
{
    if (!c) return QP_E_ARG;
    c->err.clear();
    if (n_det < 0 || n_vec < 0) return fail(c, QP_E_ARG, "negative size");
    if (c->n <= 0) return fail(c, QP_E_NOINT, "integrals not set");
    if (n_det == 0 || n_vec == 0) return QP_OK;
    if (!dets || !U || !W) return fail(c, QP_E_ARG, "null pointer");
    if (n_det > (int64_t)INT32_MAX / 2) return fail(c, QP_E_ARG, "n_det too large");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    const DevInts I = dev_ints(c);
    // the determinant space is prepared in a slot no other call uses, so that
    // QP_SIGMA_REUSE can find it again
    const int slot = QP_MAX_SYSTEMS;
    const bool reuse = (flags & QP_SIGMA_REUSE) && c->sig_valid && c->sig_dets == dets && c->sig_n_det == n_det &&
                       c->sig_gen == c->ints_gen && c->sig_stream == st;
    if (!reuse) {
        c->sig_valid = false;
        // the generator order does not matter here: every weight is 1
        double *ones = (double *)scratch(c, slot, B_ONES, sizeof(double) * n_det);
        if (!ones) return fail(c, QP_E_OOM, "device allocation failed");
        hipLaunchKernelGGL(fill_ones, dim3(grid_for(n_det)), dim3(256), 0, st, ones, n_det);
        int rc = prepare(c, slot, I, dets, ones, n_det, 1, flags & ~(QP_SIGMA_S2 | QP_SIGMA_REUSE), st, c->sig_P);
        if (rc != QP_OK) return rc;
        c->sig_valid = true;
        c->sig_dets = dets;
        c->sig_n_det = n_det;
        c->sig_gen = c->ints_gen;
        c->sig_stream = st;
    }
    launch_sigma(I, c->sig_P, dets, n_det, n_vec, (flags & QP_SIGMA_S2) != 0, U, W, st);
    HIPCHK(c, hipGetLastError());
    return QP_OK;
}

int qp_davidson(qp_ctx *c, const uint64_t *dets, int64_t n_det, int n_states, const double *guess, double tol,
                int max_iter, int flags, double *E_out, double *C_out, double *s2_out, int *n_iter, void *stream)
{
    if (!c) return QP_E_ARG;
    c->err.clear();
    if (n_det < 1) return fail(c, QP_E_ARG, "n_det must be >= 1");
    if (n_states < 1 || n_states > QP_MAX_STATES) return fail(c, QP_E_STATES, "n_states must be in [1,4]");
    if (n_states > n_det) return fail(c, QP_E_ARG, "more states than determinants");
    if (!dets || !E_out || !C_out) return fail(c, QP_E_ARG, "null pointer");
    if (!(tol > 0.0) || max_iter < 1) return fail(c, QP_E_ARG, "bad tolerance or iteration limit");
    if (c->n <= 0) return fail(c, QP_E_NOINT, "integrals not set");
    if (n_det > (int64_t)INT32_MAX / 2) return fail(c, QP_E_ARG, "n_det too large");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    const int ns = n_states;
    const int64_t N = n_det;
    double *ones = (double *)scratch(c, 0, B_ONES, sizeof(double) * N);
    if (!ones) return fail(c, QP_E_OOM, "device allocation failed");
    hipLaunchKernelGGL(fill_ones, dim3(grid_for(N)), dim3(256), 0, st, ones, N);
    const DevInts I = dev_ints(c);
    Prepared P;
    int rc = prepare(c, 0, I, dets, ones, N, 1, flags, st, P);
    if (rc != QP_OK) return rc;
    // Device-resident basis V [max_sub][N] with H V beside it, Ritz vectors X,
    // H X and residuals R [ns][N] (R also holds the new directions); the host
    // keeps the m x m Rayleigh matrix and solves the subspace problem.
    const int max_sub = (int)std::min<int64_t>(N, std::max(8 * ns, 24));
    const int64_t chunk = std::max<int64_t>(4096, (N + 63) / 64);
    const int nchunk = (int)((N + chunk - 1) / chunk);
    double *dU = (double *)scratch(c, 0, B_DU, sizeof(double) * N * max_sub);
    double *dW = (double *)scratch(c, 0, B_DW, sizeof(double) * N * max_sub);
    double *dX = (double *)scratch(c, 0, B_DX, sizeof(double) * N * ns);
    double *dR = (double *)scratch(c, 0, B_DR, sizeof(double) * N * ns);
    double *dHX = (double *)scratch(c, 0, B_DHX, sizeof(double) * N * ns);
    double *ddiag = (double *)scratch(c, 0, B_DDIAG, sizeof(double) * N);
    double *dcoef = (double *)scratch(c, 0, B_DCOEF, sizeof(double) * (max_sub * max_sub + QPD_MAX_STATES));
    double *dpart = (double *)scratch(c, 0, B_DPART, sizeof(double) * nchunk * max_sub * max_sub);
    double *ddot = (double *)scratch(c, 0, B_DDOT, sizeof(double) * 2 * max_sub * max_sub);
    if (!dU || !dW || !dX || !dR || !dHX || !ddiag || !dcoef || !dpart || !ddot)
        return fail(c, QP_E_OOM, "device allocation failed (Davidson)");
    double *dtheta = dcoef + max_sub * max_sub;
    const int gN = grid_for(N);
    hipLaunchKernelGGL(dav_diag, dim3(gN), dim3(256), 0, st, P.HII, P.perm, N, ddiag);
    // out[a * nb + b] = A_a . B_b into device memory, in stream order
    auto dots_dev = [&](const double *A, int na, const double *B, int nb, double *out) {
        const int np = na * nb;
        if (np == 0) return;
        hipLaunchKernelGGL(dav_dots_part, dim3(np, nchunk), dim3(256), 0, st, A, na, B, nb, N, chunk, dpart);
        hipLaunchKernelGGL(dav_dots_sum, dim3(grid_for(np)), dim3(256), 0, st, dpart, np, nchunk, out);
    };
    // the same, brought to the host (one synchronisation)
    auto dots = [&](const double *A, int na, const double *B, int nb, std::vector<double> &out) -> bool {
        const int np = na * nb;
        out.assign(np, 0.0);
        if (np == 0) return true;
        dots_dev(A, na, B, nb, ddot);
        return hipMemcpyAsync(out.data(), ddot, sizeof(double) * np, hipMemcpyDeviceToHost, st) == hipSuccess &&
               hipStreamSynchronize(st) == hipSuccess;
    };
    // Y_k = (acc ? Y_k : 0) + alpha sum_j coef[j][k] A_j
    auto gemv = [&](const double *A, int m, const std::vector<double> &coef, int kk, double alpha, bool acc,
                    double *Y) -> bool {
        if (hipMemcpyAsync(dcoef, coef.data(), sizeof(double) * m * kk, hipMemcpyHostToDevice, st) != hipSuccess)
            return false;
        hipLaunchKernelGGL(dav_gemv, dim3(gN), dim3(256), 0, st, A, m, N, dcoef, kk, alpha, acc ? 1 : 0, Y);
        return true;
    };
    int m = 0;        // basis size
    int g_done = 0;   // basis vectors whose Rayleigh rows are known
    std::vector<double> G((size_t)max_sub * max_sub, 0.0);
    bool ok = true;
    // orthonormalise the rows against the basis and each other (classical
    // Gram-Schmidt, twice), drop the negligible ones, append the rest and
    // their sigma-vectors
    auto add_vectors = [&](const std::vector<const double *> &rows) -> int {
        const int m0 = m;
        std::vector<double> nn;
        for (const double *src : rows) {
            if (m >= max_sub) break;
            double *x = dU + (int64_t)m * N;
            if (hipMemcpyAsync(x, src, sizeof(double) * N, hipMemcpyDeviceToDevice, st) != hipSuccess) return -1;
            // x -= V (V^T x), the coefficients staying on the device
            for (int pass = 0; pass < 2 && m > 0; ++pass) {
                dots_dev(dU, m, x, 1, ddot);
                hipLaunchKernelGGL(dav_gemv, dim3(gN), dim3(256), 0, st, dU, m, N, ddot, 1, -1.0, 1, x);
            }
            if (!dots(x, 1, x, 1, nn)) return -1;
            const double nrm = std::sqrt(std::max(nn[0], 0.0));
            if (nrm < 1e-10) continue;
            hipLaunchKernelGGL(dav_scale, dim3(gN), dim3(256), 0, st, x, N, 1.0 / nrm);
            ++m;
        }
        if (m > m0) launch_sigma(I, P, dets, N, m - m0, false, dU + (int64_t)m0 * N, dW + (int64_t)m0 * N, st);
        return m - m0;
    };
    // start: the guess, else unit vectors on the lowest diagonal elements
    std::vector<const double *> rows;
    if (guess) {
        HIPCHK(c, hipMemcpyAsync(dR, guess, sizeof(double) * ns * N, hipMemcpyDeviceToDevice, st));
    } else {
        std::vector<double> diag(N);
        HIPCHK(c, hipMemcpyAsync(diag.data(), ddiag, sizeof(double) * N, hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        std::vector<int64_t> idx(N);
        for (int64_t i = 0; i < N; ++i) idx[i] = i;
        std::partial_sort(idx.begin(), idx.begin() + ns, idx.end(),
                          [&](int64_t x, int64_t y) { return diag[x] < diag[y] || (diag[x] == diag[y] && x < y); });
        std::vector<double> e((size_t)ns * N, 0.0);
        for (int k = 0; k < ns; ++k) e[(size_t)k * N + idx[k]] = 1.0;
        HIPCHK(c, hipMemcpyAsync(dR, e.data(), sizeof(double) * ns * N, hipMemcpyHostToDevice, st));
        HIPCHK(c, hipStreamSynchronize(st));
    }
    for (int k = 0; k < ns; ++k) rows.push_back(dR + (int64_t)k * N);
    if (add_vectors(rows) < 0) return fail(c, QP_E_HIP, "Davidson vector operation failed");
    if (m < ns) return fail(c, QP_E_ARG, "the guess has fewer than n_states independent vectors");
    std::vector<double> theta, y, D1, D2, rn;
    int it = 0;
    bool converged = false;
    for (; it < max_iter; ++it) {
        // Rayleigh rows of the vectors added since the last iteration
        if (g_done < m) {
            const int k = m - g_done;
            dots_dev(dU, m, dW + (int64_t)g_done * N, k, ddot);
            dots_dev(dU + (int64_t)g_done * N, k, dW, m, ddot + (int64_t)m * k);
            D1.resize((size_t)2 * m * k);
            ok = hipMemcpyAsync(D1.data(), ddot, sizeof(double) * 2 * m * k, hipMemcpyDeviceToHost, st) == hipSuccess &&
                 hipStreamSynchronize(st) == hipSuccess;
            if (!ok) break;
            D2.assign(D1.begin() + (size_t)m * k, D1.end());
            for (int a = 0; a < m; ++a)
                for (int b = 0; b < k; ++b) {
                    const double g = 0.5 * (D1[(size_t)a * k + b] + D2[(size_t)b * m + a]);
                    G[(size_t)a * max_sub + g_done + b] = G[(size_t)(g_done + b) * max_sub + a] = g;
                }
            g_done = m;
        }
        std::vector<double> Gm((size_t)m * m);
        for (int a = 0; a < m; ++a)
            for (int b = 0; b < m; ++b) Gm[(size_t)a * m + b] = G[(size_t)a * max_sub + b];
        jacobi_eigen(Gm, m, theta, y);
        // Ritz vectors X = V y, H X = (H V) y, residuals R = H X - theta X
        std::vector<double> cy((size_t)m * ns);
        for (int j = 0; j < m; ++j)
            for (int k = 0; k < ns; ++k) cy[(size_t)j * ns + k] = y[(size_t)j * m + k];
        ok = gemv(dU, m, cy, ns, 1.0, false, dX) && gemv(dW, m, cy, ns, 1.0, false, dHX) &&
             hipMemcpyAsync(dtheta, theta.data(), sizeof(double) * ns, hipMemcpyHostToDevice, st) == hipSuccess;
        if (!ok) break;
        hipLaunchKernelGGL(dav_resid, dim3(gN), dim3(256), 0, st, dHX, dX, dtheta, ns, N, dR);
        if (!(ok = dots(dR, ns, dR, ns, rn))) break;
        double rmax = 0.0;
        for (int k = 0; k < ns; ++k) rmax = std::max(rmax, std::sqrt(std::max(rn[(size_t)k * ns + k], 0.0)));
        if (rmax < tol) { converged = true; break; }
        // corrections from the diagonal preconditioner, in place of the residuals
        rows.clear();
        for (int k = 0; k < ns; ++k) {
            if (std::sqrt(std::max(rn[(size_t)k * ns + k], 0.0)) < tol) continue;
            hipLaunchKernelGGL(dav_precond, dim3(gN), dim3(256), 0, st, dR + (int64_t)k * N, ddiag, theta[k], N,
                               dR + (int64_t)k * N);
            rows.push_back(dR + (int64_t)k * N);
        }
        if (m + (int)rows.size() > max_sub) {
            // restart from the current Ritz vectors
            ok = hipMemcpyAsync(dU, dX, sizeof(double) * ns * N, hipMemcpyDeviceToDevice, st) == hipSuccess &&
                 hipMemcpyAsync(dW, dHX, sizeof(double) * ns * N, hipMemcpyDeviceToDevice, st) == hipSuccess;
            if (!ok) break;
            m = ns;
            g_done = 0;
        }
        const int added = add_vectors(rows);
        if (added < 0) { ok = false; break; }
        if (added == 0) break;
    }
    if (!ok) return fail(c, QP_E_HIP, "Davidson vector operation failed");
    HIPCHK(c, hipGetLastError());
    if (n_iter) *n_iter = it;
    for (int k = 0; k < ns; ++k) E_out[k] = theta[k];
    std::vector<double> cx((size_t)ns * N);
    HIPCHK(c, hipMemcpyAsync(cx.data(), dX, sizeof(double) * ns * N, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));
    for (int k = 0; k < ns; ++k) {
        // a fixed sign: the largest component positive
        double *xk = cx.data() + (size_t)k * N;
        int64_t im = 0;
        for (int64_t i = 1; i < N; ++i) if (std::fabs(xk[i]) > std::fabs(xk[im])) im = i;
        if (xk[im] < 0) for (int64_t i = 0; i < N; ++i) xk[i] = -xk[i];
    }
    HIPCHK(c, hipMemcpyAsync(C_out, cx.data(), sizeof(double) * ns * N, hipMemcpyHostToDevice, st));
    if (s2_out) {
        launch_sigma(I, P, dets, N, ns, true, C_out, dW, st);
        std::vector<double> sw;
        if (!dots(C_out, ns, dW, ns, sw)) return fail(c, QP_E_HIP, "Davidson vector operation failed");
        for (int k = 0; k < ns; ++k) s2_out[k] = sw[(size_t)k * ns + k];
    }
    HIPCHK(c, hipStreamSynchronize(st));
    if (!converged) return fail(c, QP_E_NOCONV, "Davidson did not converge");
    return QP_OK;
}

int qp_energy(qp_ctx *c, const uint64_t *dets, const double *coefs, int64_t n_det, int n_states, int flags,
              double *E0_out, void *stream)
{
    int rc = common_checks(c, dets, coefs, n_det, n_states, E0_out);
    if (rc != QP_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (n_det == 0) return fail(c, QP_E_ARG, "empty wave function has no energy");
    const int nint = (c->n - 1) / 64 + 1;
    const DevInts I = dev_ints(c);
    Prepared P;
    rc = prepare(c, 0, I, dets, coefs, n_det, n_states, flags, st, P);
    if (rc != QP_OK) return rc;
    double *row = (double *)scratch(c, 0, B_ROW, sizeof(double) * n_det * n_states);
    double *c2 = (double *)scratch(c, 0, B_C2, sizeof(double) * n_det * n_states);
    if (!row || !c2) return fail(c, QP_E_OOM, "device allocation failed (energy)");
    switch (nint) {
#define ECASE(NI)                                                                                          \
    case NI:                                                                                               \
        hipLaunchKernelGGL(energy_rows<NI>, dim3(grid_for(n_det, 64)), dim3(64), 0, st, I, dets, coefs, P.perm, P.HII, \
                           P.coff, P.cent, n_det, n_states, row, c2);                                      \
        break;
        ECASE(1) ECASE(2) ECASE(3) ECASE(4)
#undef ECASE
    default: break;
    }
    hipLaunchKernelGGL(energy_total, dim3(1), dim3(256), 0, st, row, c2, n_det, n_states, E0_out);
    HIPCHK(c, hipGetLastError());
    return QP_OK;
}

int qp_set_timing(qp_ctx *c, int enable)
{
    if (!c) return QP_E_ARG;
    c->err.clear();
    HIPCHK(c, hipSetDevice(c->device));
    if (enable && !c->ev[0])
        for (auto &e : c->ev) HIPCHK(c, hipEventCreate(&e));
    c->timing = enable != 0;
    c->timed = false;
    return QP_OK;
}

int qp_last_timing(qp_ctx *c, double *out_ms)
{
    if (!c || !out_ms) return QP_E_ARG;
    if (!c->timing || !c->timed) return fail(c, QP_E_ARG, "no timed call");
    HIPCHK(c, hipEventSynchronize(c->ev[4]));
    // the dense kernel runs before the clean-cell and split-correction kernels
    // in the forward sweep and after them in the adjoint
    float a = 0.f, a2 = 0.f, b = 0.f, t = 0.f, l = 0.f, l1 = 0.f;
    HIPCHK(c, hipEventElapsedTime(&a, c->ev[1], c->ev[5]));
    HIPCHK(c, hipEventElapsedTime(&a2, c->ev[6], c->ev[2]));
    HIPCHK(c, hipEventElapsedTime(&l, c->ev[5], c->ev[6]));
    HIPCHK(c, hipEventElapsedTime(&l1, c->ev[5], c->ev[7]));
    HIPCHK(c, hipEventElapsedTime(&b, c->ev[2], c->ev[3]));
    HIPCHK(c, hipEventElapsedTime(&t, c->ev[0], c->ev[4]));
    out_ms[0] = a + a2;
    out_ms[1] = b;
    out_ms[2] = t;
    out_ms[3] = l;
    out_ms[4] = l1;
    return QP_OK;
}

int qp_alu_probe(qp_ctx *c, int kind, int64_t iters, void *stream, double *out_lane_ops_per_s)
{
    if (!c || !out_lane_ops_per_s) return QP_E_ARG;
    c->err.clear();
    if (kind < QP_PROBE_F64_FMA || kind > QP_PROBE_MIXED || iters < 1 || iters > (int64_t)1 << 24)
        return fail(c, QP_E_ARG, "probe kind must be QP_PROBE_F64_FMA, QP_PROBE_I32_ADD or QP_PROBE_MIXED, "
                                 "iters in [1, 2^24]");
    HIPCHK(c, hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    const dim3 grid((unsigned)c->num_cu * 8), block(256);   // 8 waves per SIMD
    auto launch = [&]() {
        if (kind == QP_PROBE_F64_FMA)
            hipLaunchKernelGGL(alu_probe<0>, grid, block, 0, st, iters, (double *)c->probe_sink);
        else if (kind == QP_PROBE_I32_ADD)
            hipLaunchKernelGGL(alu_probe<1>, grid, block, 0, st, iters, (double *)c->probe_sink);
        else
            hipLaunchKernelGGL(alu_probe<2>, grid, block, 0, st, iters, (double *)c->probe_sink);
    };
    if (!c->probe_sink && hipMalloc(&c->probe_sink, sizeof(double)) != hipSuccess) {
        c->probe_sink = nullptr;
        return fail(c, QP_E_OOM, "device allocation failed (probe)");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float ms = 0.f;
    if (e == hipSuccess) {
        launch();   // untimed: brings the clocks up
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    if (e == hipSuccess) {
        launch();
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(c, QP_E_HIP, std::string("probe: ") + hipGetErrorString(e));
    const double per_lane = (double)iters * 64.0 * (kind == QP_PROBE_MIXED ? 2.0 : 1.0);
    *out_lane_ops_per_s = per_lane * grid.x * block.x / (1e-3 * (double)ms);
    return QP_OK;
}

int qp_set_split(qp_ctx *c, int mode)
{
    if (!c) return QP_E_ARG;
    c->err.clear();
    if (mode != QP_SPLIT_NEVER && mode != QP_SPLIT_AUTO && mode != QP_SPLIT_ALWAYS)
        return fail(c, QP_E_ARG, "split mode must be QP_SPLIT_NEVER, QP_SPLIT_AUTO or QP_SPLIT_ALWAYS");
    c->split_mode = mode;
    return QP_OK;
}

}  // extern "C"
