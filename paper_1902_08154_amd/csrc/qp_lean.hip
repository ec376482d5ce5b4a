// qp_lean.hip -- the clean-cell pass of the EN-PT2 / selection sweep (gfx950).
//
// A hole-pair batch of generator I (holes H, |H| = 2) has a cell for every
// particle pair P; its external determinant is alpha = I - H + P (sec. "CIPSI
// selection and PT2 energy", appendix on the selection implementation).  Only a
// few cells of a batch are touched by other internal determinants J (the
// corrections and bans of the dense kernel: whole rows and columns for J that
// lack one hole, single cells for J that lack neither).  Every other cell --
// almost all of them -- has <Psi|H|alpha> = c_I <I|H|alpha>, an integral of the
// batch's block up to a sign, so that
//     e_alpha,k = c_Ik^2 x^2 / (E0_k - H_alpha,alpha)        (eq. e2)
// where x is the block element: the sign drops out, and so does every
// per-determinant bit operation.  This kernel takes exactly those cells; the
// dense kernel (split mode) takes the rest of the batch, and whole batches the
// clean cells cannot be separated from (an integral plane, a ban of the whole
// batch, buffers that overflow).
//
// Work order.  Items are (hole pair, generator) batches in hole-pair-major
// order: all generators whose determinant has the two holes of pair K occupied
// come one after the other, so the waves in flight share one or two integral
// blocks, which then stay in the L2 of every XCD instead of being fetched from
// HBM once per generator.
//
// One workgroup is one wavefront.  Lanes run over columns (particles of one
// spin), the loop over rows; per cell the kernel reads the block element and
// the pair term of H_alpha,alpha (two coalesced loads) and does the energy
// arithmetic in FP64.  A batch's sums are written to its own slot, so the
// per-generator reduction adds them in a fixed order.
#include "qp_dev.h"

namespace qplean {

constexpr int WAVE = 64;
constexpr double DEAD_D = -1e300;   // H_alpha,alpha of a lane with no cell
constexpr int CL_CAP = 256;         // listed selection candidates per wave

// reciprocal: the hardware estimate (measured relative error below 2^-24.4
// over |d| in [1e-8, 1e6]) and one Newton step, which leaves at most about 12
// ulp (the squared estimate error plus the step's own rounding)
__device__ __forceinline__ double rcp1(double d)
{
    const double r0 = __builtin_amdgcn_rcp(d);
    return fma(r0, fma(-d, r0, 1.0), r0);
}

__device__ __forceinline__ double min_abs(double m, double x)
{
    double r;
    asm("v_min_f64 %0, %1, |%2|" : "=v"(r) : "v"(m), "v"(x));
    return r;
}

__device__ __forceinline__ uint32_t rfl(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double rfl(double v)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

template <typename T>
__device__ __forceinline__ T in_vgpr(T x)
{
    asm volatile("" : "+v"(x));
    return x;
}

__device__ __forceinline__ double wsum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

template <typename T>
__device__ __forceinline__ T *carve(unsigned char *base, unsigned &off, int count)
{
    off = (off + 15u) & ~15u;
    T *r = reinterpret_cast<T *>(base + off);
    off += (unsigned)(sizeof(T) * (unsigned)count);
    return r;
}

// number of occupied orbitals of spin s of d below orbital p
template <int NINT>
__device__ __forceinline__ int occ_below(const uint64_t *d, int s, int p)
{
    int c = 0;
#pragma unroll
    for (int q = 0; q < NINT; ++q) {
        const uint64_t wv = s ? d[NINT + q] : d[q];
        if (64 * q + 63 < p) c += popc64(wv);
        else if (64 * q <= p) c += popc64(wv & ((1ull << (p - 64 * q)) - 1ull));
    }
    return c;
}

__device__ __forceinline__ bool bit_of(const uint32_t *m, int i) { return (m[i >> 5] >> (i & 31)) & 1u; }

// a clean row: the row part of H_alpha,alpha, and orbital | virtual index << 8
struct __align__(16) RowE {
    double G;
    uint32_t info;
    uint32_t pad;
};

// an FP64 load through a buffer resource: per-lane byte offset, scalar offset
__device__ __forceinline__ double bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff)
{
    typedef unsigned int v2u __attribute__((ext_vector_type(2)));
    const v2u v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    return __builtin_bit_cast(double, v);
}

}  // namespace qplean

// LDS of one workgroup (nvm = largest virtual count of a spin)
size_t lean_lds_bytes(int n, int nvm)
{
    size_t b = 0;
    auto add = [&](size_t bytes) { b = ((b + 15) & ~(size_t)15) + bytes; };
    add(2 * 2 * n);     // sVidx
    add(2 * n);         // sVirt
    add(4 * 8);         // row flags
    add(4 * 8);         // column flags
    add(16 * nvm);      // clean rows
    add(4 * qplean::CL_CAP);   // cells passing the selection pretest
    return b + 16;
}

namespace qplean {

// waves per SIMD the register allocation aims for
template <int NINT, int NS, bool BWD, bool FP>
constexpr int lean_waves() { return FP || NS == 4 ? 3 : (NS == 1 ? 5 : 4); }

template <int NINT, int NS, bool BWD, bool FP>
__global__ __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(lean_waves<NINT, NS, BWD, FP>(), 8)))
void lean_kernel(const SweepArgs *__restrict__ sys,
                                                   const int64_t *__restrict__ item_end, int n_sys)
{
    extern __shared__ __align__(16) unsigned char lds[];
    const int lane = threadIdx.x;
    const int64_t total = item_end[n_sys - 1];
    int sid = 0;
    int64_t ibase = 0;
    int K = -1;
    int64_t kend = 0;
    double mind = __builtin_inf();
    // the smallest |delta| seen, flushed to the system's minimum when the wave
    // moves on to another system and at the end (cells with no alpha leave 1e300)
    auto flush_min = [&](unsigned long long *dst) {
        double m = mind;
        for (int o = 32; o > 0; o >>= 1) m = fmin(m, __shfl_xor(m, o));
        if (m >= 1e299) m = __builtin_inf();
        const unsigned long long mb = (unsigned long long)__double_as_longlong(m);
        if (lane == 0 && mb < __atomic_load_n(dst, __ATOMIC_RELAXED)) atomicMin(dst, mb);
        mind = __builtin_inf();
    };
    for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
        if (it >= item_end[sid]) {
            flush_min(((ConstSys *)sys)[sid].min_delta_bits);
            while (it >= item_end[sid]) ibase = item_end[sid++];
            K = -1;
        }
        ConstSys &a = ((ConstSys *)sys)[sid];
        const int64_t item = it - ibase;
        // lists shorter than n_gen * n_pairs only arise from inconsistent
        // electron counts under QP_FLAG_NOCHECK: such items are skipped
        if (item >= a.kl_off[a.n_keys]) continue;
        // the pair key of this item (a wave's items only increase)
        if (K < 0 || item >= kend) {
            if (K < 0 || item >= kend + (int64_t)WAVE * 1024) {
                int lo = 0, hi = a.n_keys;   // the largest K with kl_off[K] <= item
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (a.kl_off[mid] <= item) lo = mid; else hi = mid;
                }
                K = lo;
            }
            while (a.kl_off[K + 1] <= item) ++K;
            kend = a.kl_off[K + 1];
        }
        const int n = a.n;
        const int64_t n2 = (int64_t)n * n;
        const int P2 = n * (n - 1) / 2;
        const int nup = a.nup, ndn = a.ndn;
        const int nvm = n - (nup < ndn ? nup : ndn);
        const bool want_sel = a.n_select > 0;

        unsigned off = 0;
        uint16_t *sVidx = carve<uint16_t>(lds, off, 2 * n);
        uint8_t *sVirt = carve<uint8_t>(lds, off, 2 * n);
        uint32_t *sRowF = carve<uint32_t>(lds, off, 8);
        uint32_t *sColF = carve<uint32_t>(lds, off, 8);
        RowE *sRow = carve<RowE>(lds, off, nvm);
        uint32_t *sCl = carve<uint32_t>(lds, off, CL_CAP);

        const int64_t pos = a.kl_pos[item];                    // generator position in the call
        if (pos < 0 || pos >= a.n_gen) continue;
        const int64_t g = a.gen_list ? (int64_t)a.gen_list[pos] : pos;
        const int det = a.perm[g];
        uint64_t Ib[2 * NINT];
#pragma unroll
        for (int w = 0; w < 2 * NINT; ++w) Ib[w] = a.dets[(int64_t)det * 2 * NINT + w];

        // the batch: holes (s1, h1) and (s2, h2) in the generator's index order
        int type, s1, h1, s2, h2;
        if (K < n * n) {
            type = BT_OS; s1 = 0; h1 = K / n; s2 = 1; h2 = K - h1 * n;
        } else {
            const int t = K - n * n;
            const int s = t >= P2 ? 1 : 0;
            const int u = t - s * P2;
            int b = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)u)) * 0.5f);
            while (b * (b - 1) / 2 > u) --b;
            while ((b + 1) * b / 2 <= u) ++b;
            type = BT_SS; s1 = s2 = s; h1 = u - b * (b - 1) / 2; h2 = b;
        }
        // slot of the batch among the generator's hole pairs: holes are indexed
        // over the occupied orbitals, up spin first
        const int i1 = (s1 ? nup : 0) + occ_below<NINT>(Ib, s1, h1);
        const int i2 = (s2 ? nup : 0) + occ_below<NINT>(Ib, s2, h2);
        const int pb = i2 * (i2 - 1) / 2 + i1;
        if (pb >= a.n_pairs) continue;
        const int64_t slot = pos * a.n_pairs + pb;

        // per-generator tables: virtual index of every orbital and back
        for (int x = lane; x < 2 * n; x += WAVE) {
            const int s = x >= n ? 1 : 0, p = x - s * n;
            const int c = occ_below<NINT>(Ib, s, p);
            if (occ_bit<NINT>(Ib, s, p)) sVidx[x] = 0xFFFF;
            else { sVirt[s * n + p - c] = (uint8_t)p; sVidx[x] = (uint16_t)(p - c); }
        }
        if (lane < 8) { sRowF[lane] = 0u; sColF[lane] = 0u; }
        __syncthreads();

        int rs, cs, hrs, hro, hcs, hco;
        const double *blk;
        const double *Fg = a.F + g * 2 * n;
        const double HII = a.HII[g];
        double D0;
        if (type == BT_OS) {
            if (h1 <= h2) { rs = 0; cs = 1; hrs = h1; hro = h2; blk = a.I.X + qtri(h1, h2) * n2; }
            else { rs = 1; cs = 0; hrs = h2; hro = h1; blk = a.I.X + qtri(h2, h1) * n2; }
            hcs = hro; hco = hrs;
            D0 = HII - Fg[h1] - Fg[n + h2] + a.I.Jm[h1 * n + h2];
        } else {
            rs = cs = s1; hrs = h1; hro = h2; hcs = h1; hco = h2;
            blk = a.I.Y + qtris(h1, h2) * (int64_t)P2;
            D0 = HII - Fg[s1 * n + h1] - Fg[s1 * n + h2] + a.I.JK[h1 * n + h2];
        }
        const int nr = n - (rs ? ndn : nup), nc = n - (cs ? ndn : nup);
        const uint8_t *rvirt = sVirt + rs * n, *cvirt = sVirt + cs * n;
        const int hc0 = (s1 << 8) | h1, hc1 = (s2 << 8) | h2;

        // ------------------------------------------------ which cells are clean
        // The fine filter of the dense kernel: J of the generator's coarse list
        // with m = |(I - H) \ J| <= 2.  m = 0 (J touches every cell) takes the
        // batch away from this kernel, so do more entries than the dense
        // kernel's buffers hold; otherwise m = 2 entries flag the rows of their
        // cells and m = 1 entries their rows and columns (same spin: both on
        // each particle), exactly as the dense kernel flags them.
        bool take = true;
        {
            const int64_t cbeg = a.coff[g], cend = a.coff[g + 1];
            int nfine = 0, nl = 0, nrs = 0, ncs = 0;
            bool m0 = false;
            const int nv0 = n - nup, nv1 = n - ndn;
            for (int64_t base = cbeg; base < cend; base += WAVE) {
                const int64_t e = base + lane;
                bool keep = false;
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
                    keep = m <= 2;
                }
                nfine += __popcll(__ballot(keep));
                int ner = 0, nec = 0, er[4] = {0, 0, 0, 0}, ec[4] = {0, 0, 0, 0};
                if (keep) {
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
                        } else if (type == BT_OS) {
#pragma unroll
                            for (int q = 0; q < 4; ++q) if (q == nec) ec[q] = vi;
                            nec++;
                        }
                    }
                    if (m == 0) m0 = true;
                    else if (m == 2) {
                        if (type == BT_OS) {
                            nl += ner * nec;
                            if (nec > 0)
#pragma unroll
                                for (int q = 0; q < 4; ++q) if (q < ner) atomicOr(&sRowF[er[q] >> 5], 1u << (er[q] & 31));
                        } else {
                            nl += ner * (ner - 1) / 2;
                            // cells (u, v), u < v, of E's particles: each flags row max(u, v)
#pragma unroll
                            for (int q1 = 1; q1 < 4; ++q1)
#pragma unroll
                                for (int q0 = 0; q0 < 4; ++q0)
                                    if (q0 < q1 && q1 < ner) {
                                        const int r = er[q0] > er[q1] ? er[q0] : er[q1];
                                        atomicOr(&sRowF[r >> 5], 1u << (r & 31));
                                    }
                        }
                    } else {   // m == 1
                        if (type == BT_OS) {
                            nrs += ner;
                            ncs += nec;
#pragma unroll
                            for (int q = 0; q < 4; ++q) {
                                if (q < ner) atomicOr(&sRowF[er[q] >> 5], 1u << (er[q] & 31));
                                if (q < nec) atomicOr(&sColF[ec[q] >> 5], 1u << (ec[q] & 31));
                            }
                        } else {
                            nrs += ner;
                            ncs += ner;
#pragma unroll
                            for (int q = 0; q < 4; ++q)
                                if (q < ner) {
                                    atomicOr(&sRowF[er[q] >> 5], 1u << (er[q] & 31));
                                    atomicOr(&sColF[er[q] >> 5], 1u << (er[q] & 31));
                                }
                        }
                    }
                }
            }
            // wave totals
            for (int o = 32; o > 0; o >>= 1) {
                nl += __shfl_xor(nl, o);
                nrs += __shfl_xor(nrs, o);
                ncs += __shfl_xor(ncs, o);
            }
            const bool any_m0 = __ballot(m0) != 0ull;
            take = !any_m0 && nfine <= QPF_FCAP && nl <= QPF_L2CAP && nrs <= a.rscap && ncs <= a.cscap;
        }
        __syncthreads();
        if (!take) {
            if (lane < NS) {
                a.lean_eps[slot * NS + lane] = 0.0;
                a.lean_S[slot * NS + lane] = 0.0;
            }
            continue;
        }

        // clean rows (compact): orbital, virtual index and the row part of H_aa
        int nrow = 0;
        for (int r0 = 0; r0 < nr; r0 += WAVE) {
            const int r = r0 + lane;
            const bool ok = r < nr && !bit_of(sRowF, r);
            const uint64_t mk = __ballot(ok);
            if (ok) {
                const int p = rvirt[r];
                const int at = nrow + __popcll(mk & ((1ull << lane) - 1ull));
                double gv = Fg[rs * n + p] - a.I.JK[hrs * n + p];
                gv -= (type == BT_OS ? a.I.Jm : a.I.JK)[hro * n + p];
                RowE re;
                // H_alpha,alpha is summed in the dense kernel's order, so that
                // both kernels round every diagonal alike: opposite spins
                // Gcol + (Grow + pair), same spin ((D0 + Gsecond) + Gfirst) + pair
                re.G = type == BT_OS ? gv : D0 + gv;
                re.info = (uint32_t)(p | (r << 8));
                re.pad = 0u;
                sRow[at] = re;
            }
            nrow += __popcll(mk);
        }
        __syncthreads();

        double E0[NS], cc[NS], cw[NS], q[NS], sq[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            E0[k] = a.E0[k];
            const double c = a.coefs[(int64_t)k * a.n_det + det];
            cc[k] = c * c;
            cw[k] = cc[k] * a.inv_maxc2[k];
            q[k] = 0.0;
            sq[k] = 0.0;
        }
        const uint64_t tau_key = want_sel ? bin_edge(__atomic_load_n(a.tau_bin, __ATOMIC_RELAXED)) : ~0ull;
        const double tau_val = (want_sel ? __longlong_as_double((long long)tau_key) * (1.0 - 1e-12)
                                                : __builtin_inf());
        bool appended = false;
        uint64_t fpsum = 0;
        uint32_t ncell = 0;      // clean cells of this lane
        const double *Jp = type == BT_OS ? a.I.Jm : a.I.JK;

        auto fold = [&](int pa, int pb) {
            uint64_t al[2 * NINT];
#pragma unroll
            for (int w = 0; w < 2 * NINT; ++w) al[w] = alpha_word<NINT>(Ib, w, hc0, hc1, pa, rs, pb, cs);
            return det_fold<NINT>(al);
        };
        // the energy terms of one cell; true if its selection value passes the
        // running threshold's lower bound (the exact test comes later)
        auto cell = [&](double x, double D, bool live, int pa, int pb) -> bool {
            const double x2 = x * x;
            double tsel = 0.0;
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                const double delta = E0[k] - D;
                const double rc = rcp1(delta);
                const double t = x2 * rc;
                q[k] += t;
                sq[k] = fma(t, rc, sq[k]);
                mind = min_abs(mind, delta);
                tsel = k == 0 ? cw[0] * t : fma(cw[k], t, tsel);
            }
            if (FP && live) fpsum += fold(pa, pb);
            return fabs(tsel) >= tau_val;
        };

        // The cell loop.  Lanes run over a chunk of 64 columns (virtual indices
        // of the column spin; same spin: the first, lower particle), the loop
        // over the clean rows (same spin: the second particle, above the
        // chunk's first column).  A lane past the last column or on a flagged
        // column has no cell (okc false, diagonal DEAD_D).  Same spin, rows
        // inside the chunk's span (r < dlim) hold cells only for the lanes
        // below them.  The loads go through buffer resources (block, pair-term
        // matrix): the row offset is a scalar, the lane's column offset a
        // per-chunk constant; a row's loads are issued one row ahead, its
        // table entry two rows ahead.  Cells whose selection value passes the
        // threshold's lower bound are listed in LDS as (row, lane) and
        // appended after the loop, which keeps the loop's registers few.
        const bool os = type == BT_OS;
        const uint32_t xbytes = (uint32_t)((os ? n2 : (int64_t)P2) * 8);
        const __amdgpu_buffer_rsrc_t rX = __builtin_amdgcn_make_buffer_rsrc((void *)blk, (short)0, xbytes, 0x00020000);
        const __amdgpu_buffer_rsrc_t rJ =
            __builtin_amdgcn_make_buffer_rsrc((void *)Jp, (short)0, (uint32_t)(n2 * 8), 0x00020000);
        const double *Jco = os ? a.I.Jm : a.I.JK;
        auto xoff = [&](int pr) -> uint32_t { return (uint32_t)(os ? pr * n : pr * (pr - 1) / 2) * 8u; };
        auto col_G = [&](int pc) -> double {
            return os ? D0 + Fg[cs * n + pc] - a.I.JK[hcs * n + pc] - Jco[hco * n + pc]
                      : Fg[cs * n + pc] - a.I.JK[hcs * n + pc] - Jco[hco * n + pc];
        };
        auto diag = [&](double Gc, double Grow, double j) -> double {
            return os ? Gc + (Grow + j) : (Grow + Gc) + j;
        };
        int td = 0;
        for (int c0 = 0; os ? c0 < nc : c0 + 1 < nc; c0 += WAVE) {
            const int c = c0 + lane;
            const bool okc = c < nc && !bit_of(sColF, c);
            int dlim = -1;
            if (!os) {
                while (td < nrow && (int)(sRow[td].info >> 8) <= c0) ++td;
                dlim = c0 + WAVE;
            }
            if (__ballot(okc) == 0ull || td >= nrow) continue;
            // a lane past the last column reads a valid column: the last one, or
            // (same spin) the first virtual orbital, which lies below every row
            const int pc = cvirt[c < nc ? c : (os ? nc - 1 : 0)];
            const double Gcl = okc ? col_G(pc) : DEAD_D;
            const uint32_t off8 = (uint32_t)pc * 8u;
            auto lane_off = [&](int r) -> uint32_t { return (r >= dlim || c < r) ? off8 : 0u; };
            int t = td;
            while (t < nrow) {
                uint32_t ncand = 0;
                RowE e = sRow[t];
                uint32_t rp = rfl(e.info);
                double Gr = e.G;
                uint32_t o8 = lane_off((int)(rp >> 8));
                double xc = bload(rX, o8, xoff(rp & 255));
                double jc = bload(rJ, o8, (uint32_t)((rp & 255) * n) * 8u);
                e = sRow[t + 1 < nrow ? t + 1 : t];
                for (; t < nrow; ++t) {
                    const int pr = rp & 255, r = (int)(rp >> 8);
                    const double x = xc, j = jc, G = Gr;
                    if (t + 1 < nrow) {
                        rp = rfl(e.info);
                        Gr = e.G;
                        const int pn = rp & 255;
                        o8 = lane_off((int)(rp >> 8));
                        xc = bload(rX, o8, xoff(pn));
                        jc = bload(rJ, o8, (uint32_t)(pn * n) * 8u);
                        e = sRow[t + 2 < nrow ? t + 2 : t + 1];
                    }
                    double D = diag(Gcl, G, j);
                    bool ok = okc;
                    if (r < dlim) {
                        ok = okc && c < r;
                        D = ok ? D : DEAD_D;
                        ncell += ok ? 1u : 0u;
                    }
                    const bool cnd = cell(x, D, ok, os ? pr : pc, os ? pc : pr) && ok;
                    const uint64_t mk = __builtin_amdgcn_ballot_w64(cnd);
                    if (mk) {
                        if (cnd) sCl[ncand + __popcll(mk & ((1ull << lane) - 1ull))] = (uint32_t)t | ((uint32_t)lane << 16);
                        ncand += (uint32_t)__popcll(mk);
                        if (ncand > (uint32_t)(CL_CAP - WAVE)) { ++t; break; }
                    }
                }
                if (ncand) {
                    __syncthreads();
                    // the listed cells, recomputed with the loop's arithmetic: the
                    // exact key test and the append
                    for (uint32_t i0 = 0; i0 < ncand; i0 += WAVE) {
                        const uint32_t i = i0 + lane;
                        bool cand = false;
                        uint64_t key = 0;
                        double ek[NS];
                        int pa = 0, pb = 0;
                        if (i < ncand) {
                            const uint32_t en = sCl[i];
                            const int tt = (int)(en & 0xFFFF), cl = c0 + (int)(en >> 16);
                            const RowE re = sRow[tt];
                            const int pr = re.info & 255;
                            const int pcl = cvirt[cl];
                            const uint32_t ol = (uint32_t)pcl * 8u;
                            const double x = bload(rX, ol, xoff(pr)), j = bload(rJ, ol, (uint32_t)(pr * n) * 8u);
                            const double D = diag(col_G(pcl), re.G, j);
                            const double x2 = x * x;
                            double tsel = 0.0;
#pragma unroll
                            for (int k = 0; k < NS; ++k) {
                                const double rc = rcp1(E0[k] - D);
                                const double tk = x2 * rc;
                                ek[k] = cc[k] * tk;
                                tsel = k == 0 ? cw[0] * tk : fma(cw[k], tk, tsel);
                            }
                            key = (uint64_t)__double_as_longlong(fabs(tsel));
                            cand = key >= tau_key;
                            pa = os ? pr : pcl;
                            pb = os ? pcl : pr;
                        }
                        const uint64_t mask = __ballot(cand);
                        if (!mask) continue;
                        const int leader = ctz64(mask);
                        unsigned long long bse = 0;
                        if (lane == leader) bse = atomicAdd(a.cand_count, (unsigned long long)__popcll(mask));
                        bse = __shfl(bse, leader);
                        appended = true;
                        if (cand) {
                            const unsigned long long sc = bse + __popcll(mask & ((1ull << lane) - 1ull));
                            atomicAdd(&a.hist[key_bin(key)], 1u);
                            if ((int64_t)sc < a.cand_cap) {
                                Cand *cd = a.cand + sc;
                                const int up = os ? (rs == 0 ? pa : pb) : pa;
                                const int dn = os ? (rs == 0 ? pb : pa) : pb;
                                cd->key = key;
                                cd->code = pack_code(type, s1, h1, h2, up, dn);
                                cd->g = (uint32_t)g;
                                cd->pad = 0;
#pragma unroll
                                for (int k = 0; k < QPD_MAX_STATES; ++k) cd->e[k] = k < NS ? ek[k] : 0.0;
                            } else {
                                atomicOr(a.overflow, 1ull);
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            // rows at or above dlim: one cell per active lane each
            int tf = td;
            if (!os)
                while (tf < nrow && (int)(sRow[tf].info >> 8) < dlim) ++tf;
            ncell += okc ? (uint32_t)(nrow - tf) : 0u;
        }

        // batch sums: e = c^2 x^2 / delta, S = c^2 x^2 / delta^2
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const double qs = wsum(q[k]), ss = wsum(sq[k]);
            if (lane == 0) {
                a.lean_eps[slot * NS + k] = cc[k] * qs;
                a.lean_S[slot * NS + k] = cc[k] * ss;
            }
        }
        uint32_t ct = ncell;
        uint64_t ff = fpsum;
        for (int o = 32; o > 0; o >>= 1) {
            ct += __shfl_xor(ct, o);
            if (FP) ff += __shfl_xor(ff, o);
        }
        if (lane == 0) {
            if (ct) atomicAdd(&a.lean_cnt[pos], (unsigned long long)ct);
            if (FP && ff) atomicAdd(&a.lean_fp[pos], (unsigned long long)ff);
        }
        if (want_sel && __ballot(appended)) {
            // the running threshold: the highest histogram bin with at least
            // n_select candidates at or above it.  Lane l owns bins
            // [l PER, (l + 1) PER); counts are read twice rather than kept, so
            // that the pass needs no registers beyond a few counters.
            constexpr int PER = QP_HIST_BINS / WAVE;
            uint32_t tot = 0;
            const unsigned int *hb = a.hist + lane * PER;
#pragma unroll 1
            for (int t = 0; t < PER; ++t) tot += __atomic_load_n(hb + t, __ATOMIC_RELAXED);
            uint32_t incl = tot;
            for (int o = 1; o < WAVE; o <<= 1) {
                const uint32_t v = __shfl_down(incl, o);
                if (lane + o < WAVE) incl += v;
            }
            asm volatile("" ::: "memory");
            uint64_t cum = incl - tot;
            int best = -1;
            if (cum < (uint64_t)a.n_select && cum + tot >= (uint64_t)a.n_select) {
#pragma unroll 1
                for (int t = PER - 1; t >= 0; --t) {
                    cum += __atomic_load_n(hb + t, __ATOMIC_RELAXED);
                    if (cum >= (uint64_t)a.n_select) { best = lane * PER + t; break; }
                }
            }
            for (int o = 32; o > 0; o >>= 1) {
                const int ob = __shfl_xor(best, o);
                best = ob > best ? ob : best;
            }
            if (lane == 0 && best > 0) atomicMax(a.tau_bin, best);
        }
        __syncthreads();
    }
    if (total > 0) flush_min(((ConstSys *)sys)[sid < n_sys ? sid : n_sys - 1].min_delta_bits);
}

}  // namespace qplean

template <int NINT, int NS, bool BWD>
void launch_lean(const SweepArgs *sys, const int64_t *item_end, int n_sys, bool fp, size_t lds, int grid,
                 hipStream_t st)
{
    if (fp)
        hipLaunchKernelGGL((qplean::lean_kernel<NINT, NS, BWD, true>), dim3(grid), dim3(qplean::WAVE), lds, st, sys,
                           item_end, n_sys);
    else
        hipLaunchKernelGGL((qplean::lean_kernel<NINT, NS, BWD, false>), dim3(grid), dim3(qplean::WAVE), lds, st, sys,
                           item_end, n_sys);
}

template <int NINT, int NS, bool BWD>
int lean_occupancy(size_t lds, bool fp)
{
    int blocks = 0;
    const hipError_t e = fp ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                  &blocks, qplean::lean_kernel<NINT, NS, BWD, true>, qplean::WAVE, lds)
                            : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                  &blocks, qplean::lean_kernel<NINT, NS, BWD, false>, qplean::WAVE, lds);
    if (e != hipSuccess) return 8;
    return blocks > 0 ? blocks : 1;
}

#define QPL_INST(NI, NS)                                                                                        \
    template void launch_lean<NI, NS, false>(const SweepArgs *, const int64_t *, int, bool, size_t, int,         \
                                             hipStream_t);                                                       \
    template int lean_occupancy<NI, NS, false>(size_t, bool);

QPL_INST(1, 1) QPL_INST(1, 2) QPL_INST(1, 3) QPL_INST(1, 4)
QPL_INST(2, 1) QPL_INST(2, 2) QPL_INST(2, 3) QPL_INST(2, 4)
QPL_INST(3, 1) QPL_INST(3, 2) QPL_INST(3, 3) QPL_INST(3, 4)
QPL_INST(4, 1) QPL_INST(4, 2) QPL_INST(4, 3) QPL_INST(4, 4)
