// qp_core.hip -- integral layouts, generator ordering, per-generator
// preparation, coarse filter, deterministic reductions, final selection,
// variational energy, and the C ABI (include/qp_pt2.h).
#include "qp_dev.h"
#include "../../include/qp_pt2.h"

#include <algorithm>
#include <cstdio>
#include <cstring>
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

// Cj[j][p][q] = (pq|jj), Xj[j][p][q] = (pj|jq), Jm[p][q] = (pp|qq), Km[p][q] = (pq|qp)
__global__ void build_small(const double *eri, const double *h, int n, double *Cj, double *Xj,
                            double *Jm, double *Km, double *JK, double *hc)
{
    const int64_t n3 = (int64_t)n * n * n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n3;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t j = i / ((int64_t)n * n), pq = i - j * n * n;
        int64_t p = pq / n, q = pq - p * n;
        Cj[i] = packed_eri(eri, p, q, j, j);
        Xj[i] = packed_eri(eri, p, j, j, q);
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

struct Scalars {
    unsigned int pad0;
    int tau_bin;
    unsigned long long cand_count;
    unsigned long long overflow;
    unsigned long long min_delta_bits;
    unsigned long long coarse_total;
    unsigned long long comp_count;
    long long def_count;                // batches deferred to the general kernel
    int bad_bits;     // a bit set at >= n_orb
    int bad_elec;     // electron counts differ from det 0
    int dup;          // duplicate determinant
    int pad;
};

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
            if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
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
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
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

// ---------------------------------------------------------------- reductions
// per generator: sum its items in order; eps_gen in the caller's index
// Deferred partials of one generator, in increasing batch order (its list is
// built by atomic pushes, so it is re-ordered here for a fixed summation order).
// Batches the dense kernel handed to the general kernel, listed in (rank,
// batch) order: generator g owns entries [off[g], off[g] + cnt[g]).
struct DefParts {
    const int64_t *off;
    const int32_t *cnt;
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
__global__ void reduce_empty(int64_t n_det, int ns, const int32_t *perm, double *eps_g, double *S_g, uint64_t *cnt_g,
                             uint64_t *fp_g, uint64_t *conn_g, uint64_t *defa_g, double *eps_gen)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= n_det) return;
    for (int k = 0; k < ns; ++k) {
        eps_g[g * ns + k] = 0.0;
        S_g[g * ns + k] = 0.0;
        if (eps_gen) eps_gen[k * n_det + perm[g]] = 0.0;
    }
    cnt_g[g] = 0; fp_g[g] = 0; conn_g[g] = 0; defa_g[g] = 0;
}

// per generator, in a fixed order: its dense-kernel items, then its deferred
// batches in batch order
__global__ void reduce_items(const double *eps_item, const double *S_item, const uint32_t *cnt_item,
                             const uint64_t *fp_item, const uint32_t *conn_item, const double *dc_item,
                             int64_t n_det, int nq, int ns, const int32_t *perm, double *eps_g, double *S_g,
                             uint64_t *cnt_g, uint64_t *fp_g, uint64_t *conn_g, uint64_t *defa_g, double *eps_gen,
                             double *dc, DefParts dp)
{
    int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= n_det) return;
    const int det = perm[g];
    double e[QPD_MAX_STATES] = {0, 0, 0, 0}, s[QPD_MAX_STATES] = {0, 0, 0, 0}, d[QPD_MAX_STATES] = {0, 0, 0, 0};
    uint64_t c = 0, f = 0, cn = 0, cd = 0;
    for (int i = 0; i < nq; ++i) {
        const int64_t sl = g * nq + i;
        for (int k = 0; k < ns; ++k) {
            e[k] += eps_item[sl * ns + k];
            s[k] += S_item[sl * ns + k];
            if (dc_item) d[k] += dc_item[sl * ns + k];
        }
        c += cnt_item[sl];
        cn += conn_item[sl];
        if (fp_item) f += fp_item[sl];
    }
    const int64_t x0 = dp.off[g], x1 = x0 + dp.cnt[g];
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
        eps_g[g * ns + k] = e[k];
        S_g[g * ns + k] = s[k];
        if (eps_gen) eps_gen[k * n_det + det] = e[k];
        if (dc_item && dc) dc[k * n_det + det] += d[k];
    }
    conn_g[g] = cn;
    defa_g[g] = cd;
    cnt_g[g] = c;
    fp_g[g] = f;
}

// single block, fixed summation order
__global__ void reduce_total(const double *eps_g, const double *S_g, const uint64_t *cnt_g, const uint64_t *fp_g,
                             const uint64_t *conn_g, const uint64_t *defa_g, int64_t n_det, int ns, double *e_pt2,
                             qp_pt2_stats *stats, const Scalars *sc, int64_t n_cells, const double *gup,
                             double *grad_E0)
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
            for (int k = 0; k < QPD_MAX_STATES; ++k) stats->S[k] = k < ns ? ss[0][k] : 0.0;
            stats->min_abs_delta = __longlong_as_double((long long)sc->min_delta_bits);
            for (int k = 0; k < 3; ++k) stats->reserved_d[k] = 0.0;
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
                           const uint64_t *bits, uint64_t *sel_dets, double *sel_e, int64_t *n_sel)
{
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x) {
        int32_t i = sorted[r];
        const Cand cd = cand[comp[i]];
#pragma unroll
        for (int w = 0; w < 2 * NINT; ++w) sel_dets[r * 2 * NINT + w] = bits[(int64_t)i * 2 * NINT + w];
        for (int k = 0; k < ns; ++k) sel_e[r * ns + k] = cd.e[k];
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

// ===========================================================================
// host side
// ===========================================================================

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct qp_ctx {
    int device = 0;
    std::string err;
    int n = 0;
    double *h = nullptr, *X = nullptr, *Y = nullptr, *Cj = nullptr, *Xj = nullptr, *Jm = nullptr, *Km = nullptr,
           *JK = nullptr;
    std::vector<DevBuf> bufs;
    int num_cu = 256;
    Scalars *host_sc = nullptr;   // pinned
    uint64_t *host_det0 = nullptr;
    bool timing = false;
    bool timed = false;
    // call start, dense sweep start, general kernel start, sweep end, call end
    hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
};

namespace {

enum BufId {
    B_W, B_IDX, B_RANK, B_F, B_HII, B_COUNTS, B_OFFS, B_BSUM, B_COFF, B_CENT, B_EPSI, B_SI, B_CNTI, B_FPI,
    B_DCI, B_EPSG, B_SG, B_CNTG, B_FPG, B_SC, B_HIST, B_CAND, B_COMP, B_SKEY, B_SBITS, B_SIDX, B_MAXC2,
    B_ROW, B_C2, B_TOTAL, B_DEFG, B_DEFB, B_DEFN, B_DEFE, B_DEFS, B_DEFC, B_DEFF, B_DEFD, B_CONNI, B_CONNG,
    B_DEFAG, B_DEFBITS, B_DEFCG, B_DEFOFF, B_DEFBS, B_COUNT
};

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

void *scratch(qp_ctx *c, int id, size_t bytes)
{
    if (bytes == 0) bytes = 8;
    DevBuf &b = c->bufs[id];
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

template <int NINT, int NS>
void sweep_dispatch_ns(const SweepArgs &a, int grid, bool bwd, hipStream_t st)
{
    if (bwd) launch_sweep<NINT, NS, true>(a, grid, st);
    else launch_sweep<NINT, NS, false>(a, grid, st);
}

template <int NINT>
void sweep_dispatch(const SweepArgs &a, int grid, bool bwd, hipStream_t st)
{
    switch (a.ns) {
    case 1: sweep_dispatch_ns<NINT, 1>(a, grid, bwd, st); break;
    case 2: sweep_dispatch_ns<NINT, 2>(a, grid, bwd, st); break;
    case 3: sweep_dispatch_ns<NINT, 3>(a, grid, bwd, st); break;
    default: sweep_dispatch_ns<NINT, 4>(a, grid, bwd, st); break;
    }
}

// Everything before the sweep: order, prep, coarse lists.  One host sync.
struct Prepared {
    int nint, nup, ndn, nel;
    int64_t n_det;
    int32_t *perm, *rank;
    double *F, *HII;
    int64_t *coff;
    CoarseEnt *cent;
    Scalars *sc;
    double *maxc2;
    int64_t coarse_total;
};

template <int NINT>
int prepare_t(qp_ctx *c, const uint64_t *dets, const double *coefs, int64_t n_det, int ns, int flags,
              hipStream_t st, Prepared &P)
{
    const int n = c->n;
    P.nint = NINT;
    P.n_det = n_det;
    const int64_t Pw = pow2_at_least(n_det);
    double *w = (double *)scratch(c, B_W, sizeof(double) * n_det);
    int32_t *idx = (int32_t *)scratch(c, B_IDX, sizeof(int32_t) * Pw);
    int32_t *rank = (int32_t *)scratch(c, B_RANK, sizeof(int32_t) * n_det);
    double *F = (double *)scratch(c, B_F, sizeof(double) * n_det * 2 * n);
    double *HII = (double *)scratch(c, B_HII, sizeof(double) * n_det);
    Scalars *sc = (Scalars *)scratch(c, B_SC, sizeof(Scalars));
    double *maxc2 = (double *)scratch(c, B_MAXC2, sizeof(double) * QPD_MAX_STATES);
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
    hipLaunchKernelGGL(prep_generators<NINT>, dim3((unsigned)n_det), dim3(128), 0, st, dets, idx, n_det, n, c->h,
                       c->Jm, c->Km, F, HII, sc);
    // coarse counts
    const int64_t gblocks = (n_det + 255) / 256;
    int nchunk = (int)std::max<int64_t>(1, std::min<int64_t>((2048 + gblocks - 1) / gblocks, (n_det + 255) / 256));
    const int64_t chunk = (n_det + nchunk - 1) / nchunk;
    const int64_t ncount = n_det * nchunk;
    int32_t *counts = (int32_t *)scratch(c, B_COUNTS, sizeof(int32_t) * ncount);
    int64_t *offs = (int64_t *)scratch(c, B_OFFS, sizeof(int64_t) * ncount);
    const int64_t nsb = (ncount + 1023) / 1024;
    int64_t *bsum = (int64_t *)scratch(c, B_BSUM, sizeof(int64_t) * nsb);
    int64_t *total = (int64_t *)scratch(c, B_TOTAL, sizeof(int64_t));
    int64_t *coff = (int64_t *)scratch(c, B_COFF, sizeof(int64_t) * (n_det + 1));
    if (!counts || !offs || !bsum || !total || !coff) return fail(c, QP_E_OOM, "device allocation failed");
    hipLaunchKernelGGL((coarse_kernel<NINT, false>), dim3((unsigned)gblocks, nchunk), dim3(256), 0, st, dets, idx, rank,
                       n_det, chunk, nchunk, counts, (const int64_t *)nullptr, (CoarseEnt *)nullptr, sc);
    hipLaunchKernelGGL(scan_block, dim3((unsigned)nsb), dim3(256), 0, st, counts, ncount, offs, bsum);
    hipLaunchKernelGGL(scan_bsum, dim3(1), dim3(1), 0, st, bsum, nsb, total);
    hipLaunchKernelGGL(scan_add, dim3(grid_for(ncount, 256, 1 << 30)), dim3(256), 0, st, offs, ncount, bsum);
    hipLaunchKernelGGL(make_coff, dim3(grid_for(n_det + 1)), dim3(256), 0, st, offs, n_det, nchunk, total, coff, sc);
    HIPCHK(c, hipMemcpyAsync(c->host_det0, dets, sizeof(uint64_t) * 2 * NINT, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipMemcpyAsync(c->host_sc, sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
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
    const int64_t ctot = (int64_t)hs.coarse_total;
    CoarseEnt *cent = (CoarseEnt *)scratch(c, B_CENT, sizeof(CoarseEnt) * (ctot > 0 ? ctot : 1));
    if (!cent) return fail(c, QP_E_OOM, "device allocation failed (coarse lists)");
    hipLaunchKernelGGL((coarse_kernel<NINT, true>), dim3((unsigned)gblocks, nchunk), dim3(256), 0, st, dets, idx, rank,
                       n_det, chunk, nchunk, counts, (const int64_t *)offs, cent, sc);
    P.perm = idx; P.rank = rank; P.F = F; P.HII = HII; P.coff = coff; P.cent = cent; P.sc = sc; P.maxc2 = maxc2;
    P.coarse_total = ctot;
    return QP_OK;
}

int prepare(qp_ctx *c, int nint, const uint64_t *dets, const double *coefs, int64_t n_det, int ns, int flags,
            hipStream_t st, Prepared &P)
{
    switch (nint) {
    case 1: return prepare_t<1>(c, dets, coefs, n_det, ns, flags, st, P);
    case 2: return prepare_t<2>(c, dets, coefs, n_det, ns, flags, st, P);
    case 3: return prepare_t<3>(c, dets, coefs, n_det, ns, flags, st, P);
    default: return prepare_t<4>(c, dets, coefs, n_det, ns, flags, st, P);
    }
}

int64_t cells_per_generator(int n, int nup, int ndn)
{
    int64_t vu = n - nup, vd = n - ndn;
    return (int64_t)nup * vu + (int64_t)ndn * vd + (int64_t)nup * (nup - 1) / 2 * (vu * (vu - 1) / 2) +
           (int64_t)ndn * (ndn - 1) / 2 * (vd * (vd - 1) / 2) + (int64_t)nup * vu * ndn * vd;
}

int common_checks(qp_ctx *c, const uint64_t *dets, const double *coefs, int64_t n_det, int ns, const double *E0)
{
    if (!c) return QP_E_ARG;
    c->err.clear();
    if (n_det < 0) return fail(c, QP_E_ARG, "n_det < 0");
    if (ns < 1 || ns > QP_MAX_STATES) return fail(c, QP_E_STATES, "n_states must be in [1,4]");
    if (c->n <= 0) return fail(c, QP_E_NOINT, "integrals not set");
    if (n_det > 0 && (!dets || !coefs || !E0)) return fail(c, QP_E_ARG, "null input pointer");
    if (n_det > (int64_t)INT32_MAX / 2) return fail(c, QP_E_ARG, "n_det too large");
    HIPCHK(c, hipSetDevice(c->device));
    return QP_OK;
}

DevInts dev_ints(const qp_ctx *c)
{
    DevInts I;
    I.n = c->n; I.h = c->h; I.X = c->X; I.Y = c->Y; I.Cj = c->Cj; I.Xj = c->Xj; I.Jm = c->Jm; I.Km = c->Km;
    I.JK = c->JK;
    return I;
}

template <int NINT>
int occ_ns(int n, int ns, bool bwd)
{
    switch (ns) {
    case 1: return bwd ? sweep_occupancy<NINT, 1, true>(n) : sweep_occupancy<NINT, 1, false>(n);
    case 2: return bwd ? sweep_occupancy<NINT, 2, true>(n) : sweep_occupancy<NINT, 2, false>(n);
    case 3: return bwd ? sweep_occupancy<NINT, 3, true>(n) : sweep_occupancy<NINT, 3, false>(n);
    default: return bwd ? sweep_occupancy<NINT, 4, true>(n) : sweep_occupancy<NINT, 4, false>(n);
    }
}

// persistent grid: every resident one-wavefront workgroup the CUs can hold
int sweep_grid(qp_ctx *c, int nint, int ns, bool bwd)
{
    int per_cu = 8;
    switch (nint) {
    case 1: per_cu = occ_ns<1>(c->n, ns, bwd); break;
    case 2: per_cu = occ_ns<2>(c->n, ns, bwd); break;
    case 3: per_cu = occ_ns<3>(c->n, ns, bwd); break;
    default: per_cu = occ_ns<4>(c->n, ns, bwd); break;
    }
    if (per_cu < 1) per_cu = 1;
    if (per_cu > 32) per_cu = 32;
    return c->num_cu * per_cu;
}

template <int NINT>
int focc_ns(int n, int nvm, int ns, bool bwd, int rc, int cc)
{
    switch (ns) {
    case 1: return bwd ? fast_occupancy<NINT, 1, true>(n, nvm, rc, cc) : fast_occupancy<NINT, 1, false>(n, nvm, rc, cc);
    case 2: return bwd ? fast_occupancy<NINT, 2, true>(n, nvm, rc, cc) : fast_occupancy<NINT, 2, false>(n, nvm, rc, cc);
    case 3: return bwd ? fast_occupancy<NINT, 3, true>(n, nvm, rc, cc) : fast_occupancy<NINT, 3, false>(n, nvm, rc, cc);
    default: return bwd ? fast_occupancy<NINT, 4, true>(n, nvm, rc, cc) : fast_occupancy<NINT, 4, false>(n, nvm, rc, cc);
    }
}

int fast_grid(qp_ctx *c, int nint, int ns, bool bwd, int nvm, int rc, int cc)
{
    int per_cu = 8;
    switch (nint) {
    case 1: per_cu = focc_ns<1>(c->n, nvm, ns, bwd, rc, cc); break;
    case 2: per_cu = focc_ns<2>(c->n, nvm, ns, bwd, rc, cc); break;
    case 3: per_cu = focc_ns<3>(c->n, nvm, ns, bwd, rc, cc); break;
    default: per_cu = focc_ns<4>(c->n, nvm, ns, bwd, rc, cc); break;
    }
    if (per_cu < 1) per_cu = 1;
    if (per_cu > 32) per_cu = 32;
    return c->num_cu * per_cu;
}

template <int NINT, int NS>
void fast_dispatch_ns(const SweepArgs &a, int grid, bool bwd, hipStream_t st)
{
    if (bwd) launch_fast<NINT, NS, true>(a, grid, st);
    else launch_fast<NINT, NS, false>(a, grid, st);
}

template <int NINT>
void fast_dispatch(const SweepArgs &a, int grid, bool bwd, hipStream_t st)
{
    switch (a.ns) {
    case 1: fast_dispatch_ns<NINT, 1>(a, grid, bwd, st); break;
    case 2: fast_dispatch_ns<NINT, 2>(a, grid, bwd, st); break;
    case 3: fast_dispatch_ns<NINT, 3>(a, grid, bwd, st); break;
    default: fast_dispatch_ns<NINT, 4>(a, grid, bwd, st); break;
    }
}

// work items per generator: the forward sweep splits each generator's batches
// over 16 items (batch b goes to item b mod 16) so that the persistent grid
// stays balanced; the adjoint keeps 4, because each item ends with atomic
// updates of the n x n one-electron gradient.  Items are dealt round-robin,
// without a shared counter.
constexpr int Q_FORWARD = 16;
constexpr int Q_ADJOINT = 4;
constexpr int64_t MAX_ITEMS = int64_t(1) << 25;

int items_per_generator(int64_t n_det, int nb, bool bwd)
{
    int q = bwd ? Q_ADJOINT : Q_FORWARD;
    if (nb > 0 && q > nb) q = nb;
    while (q > 1 && n_det * q > MAX_ITEMS) q /= 2;
    return std::max(q, 1);
}

int run_sweep(qp_ctx *c, const uint64_t *dets, const double *coefs, int64_t n_det, int ns, const double *E0,
              int64_t n_select, int flags, bool bwd, const double *gup, double *e_pt2, uint64_t *sel_dets,
              double *sel_e, int64_t *n_sel, qp_pt2_stats *stats, double *eps_gen, double *grad_coefs,
              double *grad_E0, double *grad_h, hipStream_t st)
{
    const int n = c->n;
    const int nint = (n - 1) / 64 + 1;
    c->timed = false;
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[0], st));
    Prepared P;
    int rc = prepare(c, nint, dets, coefs, n_det, ns, flags, st, P);
    if (rc != QP_OK) return rc;
    const int nel = P.nel;
    const int Q = items_per_generator(n_det, nel + nel * (nel - 1) / 2, bwd);
    const int64_t n_items = n_det * Q;
    double *eps_item = (double *)scratch(c, B_EPSI, sizeof(double) * std::max<int64_t>(1, n_items) * ns);
    double *S_item = (double *)scratch(c, B_SI, sizeof(double) * std::max<int64_t>(1, n_items) * ns);
    uint32_t *cnt_item = (uint32_t *)scratch(c, B_CNTI, sizeof(uint32_t) * std::max<int64_t>(1, n_items));
    uint64_t *fp_item = (uint64_t *)scratch(c, B_FPI, sizeof(uint64_t) * std::max<int64_t>(1, n_items));
    double *dc_item = bwd ? (double *)scratch(c, B_DCI, sizeof(double) * std::max<int64_t>(1, n_items) * ns) : nullptr;
    double *eps_g = (double *)scratch(c, B_EPSG, sizeof(double) * n_det * ns);
    double *S_g = (double *)scratch(c, B_SG, sizeof(double) * n_det * ns);
    uint64_t *cnt_g = (uint64_t *)scratch(c, B_CNTG, sizeof(uint64_t) * n_det);
    uint64_t *fp_g = (uint64_t *)scratch(c, B_FPG, sizeof(uint64_t) * n_det);
    unsigned int *hist = (unsigned int *)scratch(c, B_HIST, sizeof(unsigned int) * QP_HIST_BINS);
    if (!eps_item || !S_item || !cnt_item || !fp_item || (bwd && !dc_item) || !eps_g || !S_g || !cnt_g || !fp_g || !hist)
        return fail(c, QP_E_OOM, "device allocation failed (sweep buffers)");
    const int rscap = n <= 128 ? 6 : 3, cscap = n <= 128 ? 6 : 3;
    const int fgrid = fast_grid(c, nint, ns, bwd, n - std::min(P.nup, P.ndn), rscap, cscap);
    const int ggrid = sweep_grid(c, nint, ns, bwd);
    const int grid = std::max(fgrid, ggrid);
    // batches the dense kernel hands to the general kernel: one bit per
    // (generator rank, batch), then a list in (rank, batch) order
    const int nb = nel + nel * (nel - 1) / 2;
    const int nbw = std::max(1, (nb + 31) / 32);
    uint32_t *conn_item = (uint32_t *)scratch(c, B_CONNI, sizeof(uint32_t) * std::max<int64_t>(1, n_items));
    uint64_t *conn_g = (uint64_t *)scratch(c, B_CONNG, sizeof(uint64_t) * n_det);
    uint64_t *defa_g = (uint64_t *)scratch(c, B_DEFAG, sizeof(uint64_t) * n_det);
    uint32_t *def_bits = (uint32_t *)scratch(c, B_DEFBITS, sizeof(uint32_t) * n_det * nbw);
    int32_t *def_cnt_g = (int32_t *)scratch(c, B_DEFCG, sizeof(int32_t) * n_det);
    int64_t *def_off = (int64_t *)scratch(c, B_DEFOFF, sizeof(int64_t) * n_det);
    const int64_t nsb = (n_det + 1023) / 1024;
    int64_t *def_bsum = (int64_t *)scratch(c, B_DEFBS, sizeof(int64_t) * std::max<int64_t>(1, nsb));
    if (!conn_item || !conn_g || !defa_g || !def_bits || !def_cnt_g || !def_off || !def_bsum)
        return fail(c, QP_E_OOM, "device allocation failed (deferred batches)");
    HIPCHK(c, hipMemsetAsync(def_bits, 0, sizeof(uint32_t) * n_det * nbw, st));
    int64_t cand_cap = 0;
    Cand *cand = nullptr;
    if (n_select > 0) {
        const int64_t maxcell = std::max<int64_t>((int64_t)(n - P.nup) * (n - P.ndn), (int64_t)(n - P.nup) * (n - P.nup - 1) / 2);
        cand_cap = n_select + std::max<int64_t>(1 << 22, 2 * (int64_t)grid * std::min<int64_t>(maxcell, 3072));
        cand = (Cand *)scratch(c, B_CAND, sizeof(Cand) * cand_cap);
        if (!cand) return fail(c, QP_E_OOM, "device allocation failed (selection candidates)");
        HIPCHK(c, hipMemsetAsync(hist, 0, sizeof(unsigned int) * QP_HIST_BINS, st));
    }
    if (bwd) {
        if (grad_coefs) HIPCHK(c, hipMemsetAsync(grad_coefs, 0, sizeof(double) * ns * n_det, st));
        if (grad_h) HIPCHK(c, hipMemsetAsync(grad_h, 0, sizeof(double) * n * n, st));
    }
    double hmax[QPD_MAX_STATES];
    HIPCHK(c, hipMemcpyAsync(hmax, P.maxc2, sizeof(double) * QPD_MAX_STATES, hipMemcpyDeviceToHost, st));
    HIPCHK(c, hipStreamSynchronize(st));

    SweepArgs a;
    memset(&a, 0, sizeof(a));
    a.I = dev_ints(c);
    a.n = n; a.nup = P.nup; a.ndn = P.ndn; a.ns = ns; a.nel = nel;
    a.n_det = n_det; a.dets = dets; a.coefs = coefs; a.E0 = E0;
    a.perm = P.perm; a.F = P.F; a.HII = P.HII; a.coff = P.coff; a.cent = P.cent;
    a.n_items = n_items;
    a.q_per_gen = Q;
    a.flags = ((flags & QP_FLAG_FINGERPRINT) ? 1 : 0) | (bwd ? 2 : 0);
    a.eps_item = eps_item; a.S_item = S_item; a.cnt_item = cnt_item; a.fp_item = fp_item; a.conn_item = conn_item;
    a.min_delta_bits = &P.sc->min_delta_bits;
    a.n_select = n_select;
    for (int k = 0; k < QPD_MAX_STATES; ++k) {
        a.maxc2[k] = k < ns ? hmax[k] : 1.0;
        a.inv_maxc2[k] = k < ns ? 1.0 / hmax[k] : 0.0;
    }
    a.cand = cand; a.cand_count = &P.sc->cand_count; a.cand_cap = cand_cap; a.hist = hist;
    a.tau_bin = &P.sc->tau_bin; a.overflow = &P.sc->overflow;
    a.gup = gup; a.dc_item = dc_item; a.dc = grad_coefs; a.dh = grad_h;
    a.rscap = rscap; a.cscap = cscap;
    a.def_bits = def_bits; a.nbw = nbw;
    a.def_mode = 0;

    int64_t n_def = 0;
    double *def_eps = nullptr, *def_S = nullptr, *def_dc = nullptr;
    uint32_t *def_alpha = nullptr, *def_conn = nullptr;
    uint64_t *def_fp = nullptr;
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev[1], st));
    if (n_items > 0 && nel > 0) {
        switch (nint) {
        case 1: fast_dispatch<1>(a, fgrid, bwd, st); break;
        case 2: fast_dispatch<2>(a, fgrid, bwd, st); break;
        case 3: fast_dispatch<3>(a, fgrid, bwd, st); break;
        default: fast_dispatch<4>(a, fgrid, bwd, st); break;
        }
        if (c->timing) HIPCHK(c, hipEventRecord(c->ev[2], st));
        HIPCHK(c, hipGetLastError());
        hipLaunchKernelGGL(def_count, dim3(grid_for(n_det)), dim3(256), 0, st, def_bits, n_det, nbw, def_cnt_g);
        hipLaunchKernelGGL(scan_block, dim3((unsigned)nsb), dim3(256), 0, st, def_cnt_g, n_det, def_off, def_bsum);
        hipLaunchKernelGGL(scan_bsum, dim3(1), dim3(1), 0, st, def_bsum, nsb, (int64_t *)&P.sc->def_count);
        hipLaunchKernelGGL(scan_add, dim3(grid_for(n_det, 256, 1 << 30)), dim3(256), 0, st, def_off, n_det, def_bsum);
        HIPCHK(c, hipMemcpyAsync(&n_def, &P.sc->def_count, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        HIPCHK(c, hipGetLastError());
        const int64_t m = std::max<int64_t>(1, n_def);
        uint32_t *def_g = (uint32_t *)scratch(c, B_DEFG, sizeof(uint32_t) * m);
        uint32_t *def_b = (uint32_t *)scratch(c, B_DEFB, sizeof(uint32_t) * m);
        def_eps = (double *)scratch(c, B_DEFE, sizeof(double) * m * ns);
        def_S = (double *)scratch(c, B_DEFS, sizeof(double) * m * ns);
        def_alpha = (uint32_t *)scratch(c, B_DEFC, sizeof(uint32_t) * m);
        def_conn = (uint32_t *)scratch(c, B_DEFN, sizeof(uint32_t) * m);
        def_fp = (uint64_t *)scratch(c, B_DEFF, sizeof(uint64_t) * m);
        def_dc = bwd ? (double *)scratch(c, B_DEFD, sizeof(double) * m * ns) : nullptr;
        if (!def_g || !def_b || !def_eps || !def_S || !def_alpha || !def_conn || !def_fp || (bwd && !def_dc))
            return fail(c, QP_E_OOM, "device allocation failed (deferred batches)");
        if (n_def > 0) {
            hipLaunchKernelGGL(def_fill, dim3(grid_for(n_det)), dim3(256), 0, st, def_bits, n_det, nbw, def_off,
                               def_g, def_b);
            // the general kernel on the listed batches: its own slots
            SweepArgs d = a;
            d.def_mode = 1;
            d.def_g = def_g; d.def_b = def_b; d.def_n = (const int64_t *)&P.sc->def_count;
            d.eps_item = def_eps; d.S_item = def_S; d.cnt_item = def_alpha; d.fp_item = def_fp;
            d.conn_item = def_conn; d.dc_item = def_dc;
            const int dgrid = (int)std::min<int64_t>(ggrid, n_def);
            switch (nint) {
            case 1: sweep_dispatch<1>(d, dgrid, bwd, st); break;
            case 2: sweep_dispatch<2>(d, dgrid, bwd, st); break;
            case 3: sweep_dispatch<3>(d, dgrid, bwd, st); break;
            default: sweep_dispatch<4>(d, dgrid, bwd, st); break;
            }
            HIPCHK(c, hipGetLastError());
        }
        if (c->timing) HIPCHK(c, hipEventRecord(c->ev[3], st));
    } else {
        if (c->timing) HIPCHK(c, hipEventRecord(c->ev[2], st));
        if (c->timing) HIPCHK(c, hipEventRecord(c->ev[3], st));
    }
    DefParts dp;
    memset(&dp, 0, sizeof(dp));
    dp.off = def_off; dp.cnt = def_cnt_g; dp.eps = def_eps; dp.S = def_S; dp.dc = def_dc;
    dp.alpha = def_alpha; dp.conn = def_conn; dp.fp = def_fp;
    if (n_items > 0 && nel > 0)
        hipLaunchKernelGGL(reduce_items, dim3(grid_for(n_det)), dim3(256), 0, st, eps_item, S_item, cnt_item,
                           (flags & QP_FLAG_FINGERPRINT) ? fp_item : (const uint64_t *)nullptr, conn_item, dc_item,
                           n_det, Q, ns, P.perm, eps_g, S_g, cnt_g, fp_g, conn_g, defa_g, bwd ? nullptr : eps_gen,
                           bwd ? grad_coefs : nullptr, dp);
    else
        hipLaunchKernelGGL(reduce_empty, dim3(grid_for(n_det)), dim3(256), 0, st, n_det, ns, P.perm, eps_g, S_g,
                           cnt_g, fp_g, conn_g, defa_g, bwd ? nullptr : eps_gen);
    const int64_t n_cells = n_det * cells_per_generator(n, P.nup, P.ndn);
    hipLaunchKernelGGL(reduce_total, dim3(1), dim3(256), 0, st, eps_g, S_g, cnt_g, fp_g, conn_g, defa_g, n_det, ns,
                       bwd ? nullptr : e_pt2, stats, P.sc, n_cells, gup, bwd ? grad_E0 : nullptr);
    HIPCHK(c, hipGetLastError());

    if (!bwd && n_select > 0) {
        int32_t *comp = (int32_t *)scratch(c, B_COMP, sizeof(int32_t) * cand_cap);
        if (!comp) return fail(c, QP_E_OOM, "device allocation failed (selection)");
        hipLaunchKernelGGL(sel_compact, dim3(grid_for(cand_cap, 256, 8192)), dim3(256), 0, st, cand, P.sc, cand_cap,
                           comp, P.sc);
        HIPCHK(c, hipMemcpyAsync(c->host_sc, P.sc, sizeof(Scalars), hipMemcpyDeviceToHost, st));
        HIPCHK(c, hipStreamSynchronize(st));
        const Scalars hs = *c->host_sc;
        if (hs.overflow & 1ull) return fail(c, QP_E_OVERFLOW, "selection candidate buffer overflowed");
        const int64_t M = (int64_t)hs.comp_count;
        const int64_t m = std::min<int64_t>(M, n_select);
        const int64_t PP = pow2_at_least(std::max<int64_t>(M, 1));
        uint64_t *skey = (uint64_t *)scratch(c, B_SKEY, sizeof(uint64_t) * PP);
        uint64_t *sbits = (uint64_t *)scratch(c, B_SBITS, sizeof(uint64_t) * PP * 2 * nint);
        int32_t *sidx = (int32_t *)scratch(c, B_SIDX, sizeof(int32_t) * PP);
        if (!skey || !sbits || !sidx) return fail(c, QP_E_OOM, "device allocation failed (selection sort)");
        switch (nint) {
#define SELCASE(NI)                                                                                        \
    case NI:                                                                                               \
        hipLaunchKernelGGL(sel_materialise<NI>, dim3(grid_for(PP)), dim3(256), 0, st, cand, comp, M, dets, P.perm, \
                           skey, sbits, PP, sidx);                                                         \
        bitonic_sort(sidx, PP, SelCmp<NI>{skey, sbits}, st);                                              \
        hipLaunchKernelGGL(sel_output<NI>, dim3(grid_for(std::max<int64_t>(m, 1))), dim3(256), 0, st, cand, comp, sidx, m, \
                           ns, sbits, sel_dets, sel_e, n_sel);                                             \
        break;
            SELCASE(1) SELCASE(2) SELCASE(3) SELCASE(4)
#undef SELCASE
        default: break;
        }
        HIPCHK(c, hipGetLastError());
    }
    if (c->timing) {
        HIPCHK(c, hipEventRecord(c->ev[4], st));
        c->timed = true;
    }
    return QP_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

int qp_create(qp_ctx **ctx, int device)
{
    if (!ctx) return QP_E_ARG;
    *ctx = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return QP_E_HIP;
    qp_ctx *c = new qp_ctx();
    c->device = device;
    c->bufs.resize(B_COUNT);
    if (hipSetDevice(device) != hipSuccess) { delete c; return QP_E_HIP; }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->num_cu = prop.multiProcessorCount;
    if (hipHostMalloc((void **)&c->host_sc, sizeof(Scalars), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&c->host_det0, sizeof(uint64_t) * 2 * QPD_MAX_NINT, hipHostMallocDefault) != hipSuccess) {
        delete c;
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
    for (auto &b : c->bufs) if (b.p) (void)hipFree(b.p);
    for (auto &e : c->ev) if (e) (void)hipEventDestroy(e);
    double *arrs[] = {c->h, c->X, c->Y, c->Cj, c->Xj, c->Jm, c->Km, c->JK};
    for (double *p : arrs) if (p) (void)hipFree(p);
    if (c->host_sc) (void)hipHostFree(c->host_sc);
    if (c->host_det0) (void)hipHostFree(c->host_det0);
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
    double **arrs[] = {&c->h, &c->X, &c->Y, &c->Cj, &c->Xj, &c->Jm, &c->Km, &c->JK};
    for (double **p : arrs) if (*p) { (void)hipFree(*p); *p = nullptr; }
    c->n = 0;
    const int64_t n = n_orb;
    const size_t nX = (size_t)(n * (n + 1) / 2) * n * n;
    const size_t P2 = (size_t)(n * (n - 1) / 2);
    const size_t nY = std::max<size_t>(1, P2 * P2);
    const size_t n3 = (size_t)n * n * n, n2 = (size_t)n * n;
    if (hipMalloc(&c->X, nX * 8) != hipSuccess || hipMalloc(&c->Y, nY * 8) != hipSuccess ||
        hipMalloc(&c->Cj, n3 * 8) != hipSuccess || hipMalloc(&c->Xj, n3 * 8) != hipSuccess ||
        hipMalloc(&c->Jm, n2 * 8) != hipSuccess || hipMalloc(&c->Km, n2 * 8) != hipSuccess ||
        hipMalloc(&c->JK, n2 * 8) != hipSuccess || hipMalloc(&c->h, n2 * 8) != hipSuccess) {
        (void)hipGetLastError();
        for (double **p : arrs) if (*p) { (void)hipFree(*p); *p = nullptr; }
        return fail(c, QP_E_OOM, "device allocation failed (integral layouts)");
    }
    hipLaunchKernelGGL(build_X, dim3(grid_for((int64_t)nX, 256, 1 << 16)), dim3(256), 0, st, eri_packed, n_orb, c->X);
    if (P2 > 0)
        hipLaunchKernelGGL(build_Y, dim3(grid_for((int64_t)(P2 * P2), 256, 1 << 16)), dim3(256), 0, st, eri_packed, n_orb, c->Y);
    hipLaunchKernelGGL(build_small, dim3(grid_for((int64_t)n3, 256, 1 << 16)), dim3(256), 0, st, eri_packed, h, n_orb,
                       c->Cj, c->Xj, c->Jm, c->Km, c->JK, c->h);
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
    hipStream_t st = (hipStream_t)stream;
    if (n_det == 0) {
        HIPCHK(c, hipMemsetAsync(e_pt2, 0, sizeof(double) * n_states, st));
        if (stats) HIPCHK(c, hipMemsetAsync(stats, 0, sizeof(qp_pt2_stats), st));
        if (n_sel) HIPCHK(c, hipMemsetAsync(n_sel, 0, sizeof(int64_t), st));
        return QP_OK;
    }
    return run_sweep(c, dets, coefs, n_det, n_states, E0, n_select, flags, false, nullptr, e_pt2, sel_dets, sel_e,
                     n_sel, stats, eps_gen, nullptr, nullptr, nullptr, st);
}

int qp_pt2_backward(qp_ctx *c, const uint64_t *dets, const double *coefs, int64_t n_det, int n_states,
                    const double *E0, const double *grad_e_pt2, int flags, double *grad_coefs, double *grad_E0,
                    double *grad_h, qp_pt2_stats *stats, void *stream)
{
    int rc = common_checks(c, dets, coefs, n_det, n_states, E0);
    if (rc != QP_OK) return rc;
    if (!grad_e_pt2) return fail(c, QP_E_ARG, "grad_e_pt2 is required");
    hipStream_t st = (hipStream_t)stream;
    if (n_det == 0) {
        if (grad_E0) HIPCHK(c, hipMemsetAsync(grad_E0, 0, sizeof(double) * n_states, st));
        if (grad_h) HIPCHK(c, hipMemsetAsync(grad_h, 0, sizeof(double) * c->n * c->n, st));
        if (stats) HIPCHK(c, hipMemsetAsync(stats, 0, sizeof(qp_pt2_stats), st));
        return QP_OK;
    }
    return run_sweep(c, dets, coefs, n_det, n_states, E0, 0, flags, true, grad_e_pt2, nullptr, nullptr, nullptr,
                     nullptr, stats, nullptr, grad_coefs, grad_E0, grad_h, st);
}

int qp_energy(qp_ctx *c, const uint64_t *dets, const double *coefs, int64_t n_det, int n_states, int flags,
              double *E0_out, void *stream)
{
    int rc = common_checks(c, dets, coefs, n_det, n_states, E0_out);
    if (rc != QP_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (n_det == 0) return fail(c, QP_E_ARG, "empty wave function has no energy");
    const int nint = (c->n - 1) / 64 + 1;
    Prepared P;
    rc = prepare(c, nint, dets, coefs, n_det, n_states, flags, st, P);
    if (rc != QP_OK) return rc;
    double *row = (double *)scratch(c, B_ROW, sizeof(double) * n_det * n_states);
    double *c2 = (double *)scratch(c, B_C2, sizeof(double) * n_det * n_states);
    if (!row || !c2) return fail(c, QP_E_OOM, "device allocation failed (energy)");
    DevInts I = dev_ints(c);
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
    float a = 0.f, b = 0.f, t = 0.f;
    HIPCHK(c, hipEventElapsedTime(&a, c->ev[1], c->ev[2]));
    HIPCHK(c, hipEventElapsedTime(&b, c->ev[2], c->ev[3]));
    HIPCHK(c, hipEventElapsedTime(&t, c->ev[0], c->ev[4]));
    out_ms[0] = a;
    out_ms[1] = b;
    out_ms[2] = t;
    return QP_OK;
}

}  // extern "C"
