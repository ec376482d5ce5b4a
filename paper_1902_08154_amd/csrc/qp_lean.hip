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

#include <type_traits>

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

// v moved DPP-wise across lanes (0 where the source lane is outside the row
// or the row is masked off)
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dppd(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROW_MASK, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// The sums over the wave of two values at once: one exchange of the wave's
// halves (lanes 32-63 of the first operand with lanes 0-31 of the second)
// leaves u's pairwise sums in lanes 0-31 and w's in lanes 32-63; a DPP scan
// within each half then puts u's total in lane 31 and w's in lane 63.
__device__ __forceinline__ double sum2(double u, double w)
{
    const long long ub = __double_as_longlong(u), wb = __double_as_longlong(w);
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)(ub & 0xffffffffll), (unsigned)(wb & 0xffffffffll),
                                                     false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ub >> 32), (unsigned)(wb >> 32), false, false);
    double v = __longlong_as_double(((long long)hi[0] << 32) | lo[0]) +
               __longlong_as_double(((long long)hi[1] << 32) | lo[1]);
    v += dppd<0x111, 0xf>(v);   // row_shr:1
    v += dppd<0x112, 0xf>(v);   // row_shr:2
    v += dppd<0x114, 0xf>(v);   // row_shr:4
    v += dppd<0x118, 0xf>(v);   // row_shr:8
    v += dppd<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
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

// The items of a launch in XCD-major shares: the workgroups that the
// hardware places on one XCD (block index mod 8, when the grid is a multiple
// of 8) form a group that owns one contiguous eighth of the item range, so
// that the items sharing a hole pair, which are consecutive, meet in that
// XCD's L2 instead of every XCD's.  The group's waves claim its items one at
// a time (a counter per group), so that they stay within a few hundred
// consecutive items of each other: statically dealt items let them drift
// apart over a launch until they span many hole pairs, whose integral blocks
// no longer fit in L2 together.
__device__ __forceinline__ void xcd_share(int64_t total, int64_t &lo, int64_t &end, int &group)
{
    const int nx = (gridDim.x % ITEM_CTR_GROUPS) == 0u ? ITEM_CTR_GROUPS : 1;
    const int64_t per = (total + nx - 1) / nx;
    group = (int)(blockIdx.x % nx);
    lo = (int64_t)group * per;
    end = lo + per < total ? lo + per : total;
}

__device__ __forceinline__ bool bit_of(const uint32_t *m, int i) { return (m[i >> 5] >> (i & 31)) & 1u; }

// a clean row: the row part of H_alpha,alpha and the byte offsets of the row
// in the integral block and in the pair-term matrix (its orbital and virtual
// index are kept apart, for the few places that need them)
struct __align__(16) RowE {
    double G;
    uint32_t xo;
    uint32_t jo;
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
size_t lean_lds_bytes(int n, int nvm, bool bwd)
{
    size_t b = bwd ? 8 * QPD_MAX_ORB : 0;   // adjoint: the wave's dE/dh_pp
    auto add = [&](size_t bytes) { b = ((b + 15) & ~(size_t)15) + bytes; };
    add(2 * 2 * n);     // sVidx
    add(2 * n);         // sVirt
    add(4 * 8);         // row flags
    add(4 * 8);         // column flags
    add(16 * nvm);      // clean rows
    add(4 * nvm);       // their orbital and virtual index
    add(4 * qplean::CL_CAP);   // cells passing the selection pretest
    return b + 16;
}

namespace qplean {

// waves per SIMD the register allocation aims for
template <int NINT, int NS, bool BWD, bool FP>
constexpr int lean_waves()
{
    if (BWD) return NS <= 2 ? 4 : 3;
    return FP && (NS == 4 || (NS == 3 && NINT == 4)) ? 2 : (FP || NS >= 3 ? 3 : 4);
}

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
    // adjoint: this wave's share of dE/dh_pp, kept in LDS across its items and
    // added to the system's dh when the wave moves on and at the end
    double *sDH = reinterpret_cast<double *>(lds);
    if (BWD)
        for (int p = lane; p < QPD_MAX_ORB; p += WAVE) sDH[p] = 0.0;
    auto flush_dh = [&](ConstSys &s) {
        if (!BWD) return;
        for (int p = lane; p < s.n; p += WAVE) {
            const double v = sDH[p];
            if (v != 0.0 && s.dh) atomicAdd(&s.dh[(int64_t)p * s.n + p], v);
            sDH[p] = 0.0;
        }
    };
    int64_t ilo, iend;
    int group;
    xcd_share(total, ilo, iend, group);
    unsigned long long *ctr = sys[0].item_ctr + group * ITEM_CTR_STRIDE;
    for (;;) {
        unsigned long long claim = 0;
        if (lane == 0) claim = atomicAdd(ctr, 1ull);
        // lane 0's claim, as a wave-uniform (scalar) value
        const uint32_t clo = __builtin_amdgcn_readfirstlane((uint32_t)claim);
        const uint32_t chi = __builtin_amdgcn_readfirstlane((uint32_t)(claim >> 32));
        const int64_t it = ilo + (int64_t)(((uint64_t)chi << 32) | clo);
        if (it >= iend) break;
        if (it >= item_end[sid]) {
            flush_min(((ConstSys *)sys)[sid].min_delta_bits);
            flush_dh(((ConstSys *)sys)[sid]);
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

        unsigned off = BWD ? 8u * QPD_MAX_ORB : 0u;
        uint16_t *sVidx = carve<uint16_t>(lds, off, 2 * n);
        uint8_t *sVirt = carve<uint8_t>(lds, off, 2 * n);
        uint32_t *sRowF = carve<uint32_t>(lds, off, 8);
        uint32_t *sColF = carve<uint32_t>(lds, off, 8);
        RowE *sRow = carve<RowE>(lds, off, nvm);
        uint32_t *sRi = carve<uint32_t>(lds, off, nvm);
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
        // the flags of the dense kernel's corrections (split_flags); a batch
        // with a determinant that touches every cell is not split
        const bool take = split_flags(a, g, n, nup, ndn, type == BT_OS, rs, hc0, hc1, sVidx, sRowF, sColF, lane);
        __syncthreads();
        if (!take) {
            if (lane < NS) {
                a.lean_eps[slot * NS + lane] = 0.0;
                a.lean_S[slot * NS + lane] = 0.0;
                if (BWD) a.lean_dc[slot * NS + lane] = 0.0;
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
                re.xo = (uint32_t)(type == BT_OS ? p * n : p * (p - 1) / 2) * 8u;
                re.jo = (uint32_t)(p * n) * 8u;
                sRow[at] = re;
                sRi[at] = (uint32_t)(p | (r << 8));
            }
            nrow += __popcll(mk);
        }
        __syncthreads();

        double E0[NS], cc[NS], cw[NS], q[NS], sq[NS], gc[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            E0[k] = a.E0[k];
            const double c = a.coefs[(int64_t)k * a.n_det + det];
            cc[k] = c * c;
            cw[k] = cc[k] * a.inv_maxc2[k];
            q[k] = 0.0;
            sq[k] = 0.0;
            gc[k] = BWD ? a.gup[k] * cc[k] : 0.0;
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
        // adjoint: v gains the cell's sum over states of g c^2 x^2 / delta^2, its
        // share of dE/dh_pp for every orbital the external determinant holds
        auto cell = [&](double x, double D, bool live, int pa, int pb, double thr, double &v) -> bool {
            const double x2 = x * x;
            double tsel = 0.0;
#pragma unroll
            for (int k = 0; k < NS; ++k) {
                const double delta = E0[k] - D;
                const double rc = rcp1(delta);
                const double t = x2 * rc;
                q[k] += t;
                sq[k] = fma(t, rc, sq[k]);
                if (BWD) v = fma(t * gc[k], rc, v);
                mind = min_abs(mind, delta);
                if (!BWD) tsel = k == 0 ? cw[0] * t : fma(cw[k], t, tsel);
            }
            if (FP && live) fpsum += fold(pa, pb);
            // (the adjoint selects nothing)
            return !BWD && fabs(tsel) >= thr;
        };

        // The cell loop.  Lanes run over a chunk of 64 columns (virtual indices
        // of the column spin; same spin: the first, lower particle), the loop
        // over the clean rows (same spin: the second particle, above the
        // chunk's first column).  A lane past the last column or on a flagged
        // column has no cell (okc false, diagonal DEAD_D).  Same spin, rows
        // inside the chunk's span hold cells only for the lanes below them and
        // take a simple loop of their own; every other row, a cell per active
        // lane, takes the main loop.  Loads go through buffer resources (block,
        // pair-term matrix): the row offset is a scalar, the lane's column
        // offset a per-chunk constant.  The main loop holds two rows in two
        // register sets that it refills in turn, one row ahead, and each row's
        // table entry one row before its loads.  Cells whose selection value
        // passes the threshold's lower bound are listed in LDS as (row, lane)
        // and appended after the rows (flush), which keeps the loop's registers
        // few; a list about to fill ends the loop early and restarts it.
        const bool os = type == BT_OS;
        const uint32_t xbytes = (uint32_t)((os ? n2 : (int64_t)P2) * 8);
        const __amdgpu_buffer_rsrc_t rX = __builtin_amdgcn_make_buffer_rsrc((void *)blk, (short)0, xbytes, 0x00020000);
        const __amdgpu_buffer_rsrc_t rJ =
            __builtin_amdgcn_make_buffer_rsrc((void *)Jp, (short)0, (uint32_t)(n2 * 8), 0x00020000);
        const double *Jco = os ? a.I.Jm : a.I.JK;
        auto col_G = [&](int pc) -> double {
            return os ? D0 + Fg[cs * n + pc] - a.I.JK[hcs * n + pc] - Jco[hco * n + pc]
                      : Fg[cs * n + pc] - a.I.JK[hcs * n + pc] - Jco[hco * n + pc];
        };
        auto diag = [&](double Gc, double Grow, double j) -> double {
            return os ? Gc + (Grow + j) : (Grow + Gc) + j;
        };
        // the listed cells of chunk c0, recomputed with the loop's arithmetic:
        // the exact key test and the append
        auto flush = [&](int c0, uint32_t ncand) {
            __syncthreads();
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
                    const int pr = (int)(sRi[tt] & 255u);
                    const int pcl = cvirt[cl];
                    const uint32_t ol = (uint32_t)pcl * 8u;
                    const double x = bload(rX, ol + re.xo, 0u), j = bload(rJ, ol + re.jo, 0u);
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
        };
        // list the lanes of row t whose cell passed the pretest
        auto note = [&](bool cnd, int t, uint32_t &ncand) {
            if (BWD) return;
            const uint64_t mk = __builtin_amdgcn_ballot_w64(cnd);
            if (mk) {
                if (cnd) sCl[ncand + __popcll(mk & ((1ull << lane) - 1ull))] = (uint32_t)t | ((uint32_t)lane << 16);
                ncand += (uint32_t)__popcll(mk);
            }
        };
        // the main loop over rows [tb, te), specialised on the batch type
        auto main_rows = [&](auto OSC, int c0, int tb, int te, double Gcl, uint32_t off8, bool okc, int pc,
                             double &colacc) {
            constexpr bool OS_ = decltype(OSC)::value;
            // a lane with no cell takes an infinite threshold: its value, x^2
            // times about 1e-300, never reaches it
            const double thr = okc ? tau_val : __builtin_inf();
            auto load = [&](const RowE &e, double &G, double &x, double &j) {
                G = e.G;
                x = bload(rX, off8, rfl(e.xo));
                j = bload(rJ, off8, rfl(e.jo));
            };
            // the row's orbital, for the fingerprint and the adjoint only
            auto orb = [&](int t) -> int { return FP || BWD ? (int)(rfl(sRi[t]) & 255u) : 0; };
            int t = tb;
            while (t < te) {
                uint32_t ncand = 0;
                // two register sets, each refilled right after its cell with the
                // row two ahead (the last row again past the end: no path through
                // the loop leaves one set's loads pending behind the other's);
                // the table entry of that row is read before the cell
                double GA, GB, xA, xB, jA, jB;
                load(sRow[t], GA, xA, jA);
                load(sRow[t + 1 < te ? t + 1 : t], GB, xB, jB);
                // pairs of rows: both cells first, so that their dependency
                // chains interleave, then the refills and the candidate lists
                bool full = false;
                for (; t + 1 < te; t += 2) {
                    const RowE nA = sRow[t + 2 < te ? t + 2 : te - 1];
                    const RowE nB = sRow[t + 3 < te ? t + 3 : te - 1];
                    const int prA = orb(t), prB = orb(t + 1);
                    double vA = 0.0, vB = 0.0;
                    const double DA = OS_ ? Gcl + (GA + jA) : (GA + Gcl) + jA;
                    const double DB = OS_ ? Gcl + (GB + jB) : (GB + Gcl) + jB;
                    const bool cA = cell(xA, DA, okc, OS_ ? prA : pc, OS_ ? pc : prA, thr, vA);
                    const bool cB = cell(xB, DB, okc, OS_ ? prB : pc, OS_ ? pc : prB, thr, vB);
                    load(nA, GA, xA, jA);
                    load(nB, GB, xB, jB);
                    note(cA, t, ncand);
                    note(cB, t + 1, ncand);
                    if (BWD) {
                        // the two rows' totals to their orbitals (lane 31 holds
                        // row t's, lane 63 row t + 1's), each lane's cells to its
                        // column
                        colacc += vA + vB;
                        const double rt = sum2(vA, vB);
                        if ((lane & 31) == 31) sDH[lane < 32 ? prA : prB] += rt;
                    }
                    if (ncand > (uint32_t)(CL_CAP - 2 * WAVE)) { t += 2; full = true; break; }
                }
                if (!full && t < te) {
                    // an odd row count: the last row, in the first set
                    const int prA = orb(t);
                    double vA = 0.0;
                    const double DA = OS_ ? Gcl + (GA + jA) : (GA + Gcl) + jA;
                    note(cell(xA, DA, okc, OS_ ? prA : pc, OS_ ? pc : prA, thr, vA), t, ncand);
                    if (BWD) {
                        colacc += vA;
                        const double rt = wsum(vA);
                        if (lane == 0) sDH[prA] += rt;
                    }
                    ++t;
                }
                if (ncand) flush(c0, ncand);
            }
            ncell += okc ? (uint32_t)(te - tb) : 0u;
        };
        int td = 0, tf = 0;   // same spin: the chunk's rows inside its span are [td, tf)
        for (int c0 = 0; os ? c0 < nc : c0 + 1 < nc; c0 += WAVE) {
            const int c = c0 + lane;
            const bool okc = c < nc && !bit_of(sColF, c);
            if (!os) {
                // the rows are in increasing virtual index: count, across the
                // lanes, those at or below the chunk's first column and those
                // below its end
                int nd = 0, nf = 0;
                for (int t0 = 0; t0 < nrow; t0 += WAVE) {
                    const int t = t0 + lane;
                    const int r = t < nrow ? (int)(sRi[t] >> 8) : 1 << 20;
                    nd += __popcll(__ballot(r <= c0));
                    nf += __popcll(__ballot(r < c0 + WAVE));
                }
                td = nd;
                tf = nf;
            }
            if (__ballot(okc) == 0ull || td >= nrow) continue;
            // a lane past the last column reads a valid column: the last one, or
            // (same spin) the first virtual orbital, which lies below every row
            const int pc = cvirt[c < nc ? c : (os ? nc - 1 : 0)];
            const double Gcl = okc ? col_G(pc) : DEAD_D;
            const uint32_t off8 = (uint32_t)pc * 8u;
            double colacc = 0.0;   // adjoint: this lane's cells, for its column's orbital
            if (os) {
                main_rows(std::integral_constant<bool, true>(), c0, 0, nrow, Gcl, off8, okc, pc, colacc);
                if (BWD && okc) sDH[pc] += colacc;
                continue;
            }
            // same spin, rows inside the chunk's span
            uint32_t ncand = 0;
            for (int t = td; t < tf; ++t) {
                const RowE e = sRow[t];
                const uint32_t rp = rfl(sRi[t]);
                const int pr = rp & 255, r = (int)(rp >> 8);
                const bool ok = okc && c < r;
                const uint32_t o8 = ok ? off8 : 0u;
                const double x = bload(rX, o8, rfl(e.xo));
                const double j = bload(rJ, o8, rfl(e.jo));
                const double D = ok ? diag(Gcl, e.G, j) : DEAD_D;
                ncell += ok ? 1u : 0u;
                double v = 0.0;
                note(cell(x, D, ok, pc, pr, ok ? tau_val : __builtin_inf(), v), t, ncand);
                if (BWD) {
                    colacc += v;
                    const double rt = wsum(v);
                    if (lane == 0) sDH[pr] += rt;
                }
                if (ncand > (uint32_t)(CL_CAP - WAVE)) { flush(c0, ncand); ncand = 0; }
            }
            if (ncand) flush(c0, ncand);
            main_rows(std::integral_constant<bool, false>(), c0, tf, nrow, Gcl, off8, okc, pc, colacc);
            if (BWD && okc) sDH[pc] += colacc;
        }

        // batch sums: e = c^2 x^2 / delta, S = c^2 x^2 / delta^2; adjoint: the
        // generator's dE/dc_I = 2 g c_I sum x^2 / delta (its cells have no
        // other determinant), and the batch's total of v for the orbitals
        // every cell holds, the generator's occupied ones but the two holes
        double vb = 0.0;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const double qs = wsum(q[k]), ss = wsum(sq[k]);
            if (BWD) vb = fma(gc[k], ss, vb);
            if (lane == 0) {
                a.lean_eps[slot * NS + k] = cc[k] * qs;
                a.lean_S[slot * NS + k] = cc[k] * ss;
                if (BWD) a.lean_dc[slot * NS + k] = 2.0 * a.gup[k] * a.coefs[(int64_t)k * a.n_det + det] * qs;
            }
        }
        if (BWD && vb != 0.0) {
            for (int p = lane; p < n; p += WAVE) {
                const int np = (sVidx[p] == 0xFFFF ? 1 : 0) + (sVidx[n + p] == 0xFFFF ? 1 : 0) -
                               ((s1 == 0 ? p == h1 : false) || (s2 == 0 ? p == h2 : false) ? 1 : 0) -
                               ((s1 == 1 ? p == h1 : false) || (s2 == 1 ? p == h2 : false) ? 1 : 0);
                if (np) sDH[p] += np * vb;
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
    if (total > 0) {
        flush_min(((ConstSys *)sys)[sid < n_sys ? sid : n_sys - 1].min_delta_bits);
        flush_dh(((ConstSys *)sys)[sid < n_sys ? sid : n_sys - 1]);
    }
}

// ---------------------------------------------------------------------------
// The split-correction kernel: the flagged cells of the batches the clean-cell
// kernel split, after it.  Items are the same (hole pair, generator) batches.
// A flagged cell's numerator is c_I <I|H|alpha> plus c_J <J|H|alpha> of every
// fine entry J of the generator's coarse list whose particles the cell holds
// (m = 1: one of them; m = 2: all), each evaluated by the Slater-Condon rules;
// J earlier in generator order, or J = alpha, bans the cell (alpha belongs to
// an earlier generator, or is internal).  The batch's sums are added to the
// slot the clean-cell kernel wrote.  A batch with more fine entries than the
// LDS list holds is handed to the general kernel (marked in def_bits), which
// then takes the same flagged cells.
// ---------------------------------------------------------------------------
constexpr int FCAPC = 64;   // fine entries a batch may have here

}  // namespace qplean

size_t corr_lds_bytes(int n, int ns, bool bwd)
{
    size_t b = bwd ? 8 * QPD_MAX_ORB : 0;   // adjoint: the wave's dE/dh_pp
    auto add = [&](size_t bytes) { b = ((b + 15) & ~(size_t)15) + bytes; };
    add(2 * 2 * n);                 // sVidx
    add(2 * n);                     // sVirt
    add(4 * 16);                    // row and column flags
    add(4 * qplean::FCAPC);         // fine: J
    add(4 * qplean::FCAPC);         // fine: E_J's row-spin particles (virtual indices, one per byte)
    add(4 * qplean::FCAPC);         // fine: E_J's column-spin particles
    add(4 * qplean::FCAPC);         // fine: m | earlier << 2 | ner << 4 | nec << 8
    add(8 * qplean::FCAPC * ns);    // fine: c_Jk
    if (bwd) add(8 * qplean::FCAPC * ns);   // adjoint: dE/dc_Jk
    return b + 16;
}

namespace qplean {

template <int NINT, int NS, bool BWD, bool FP>
__global__ __launch_bounds__(WAVE) void corr_kernel(const SweepArgs *__restrict__ sys,
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
    auto flush_min = [&](unsigned long long *dst) {
        double m = mind;
        for (int o = 32; o > 0; o >>= 1) m = fmin(m, __shfl_xor(m, o));
        if (m >= 1e299) m = __builtin_inf();
        const unsigned long long mb = (unsigned long long)__double_as_longlong(m);
        if (lane == 0 && mb < __atomic_load_n(dst, __ATOMIC_RELAXED)) atomicMin(dst, mb);
        mind = __builtin_inf();
    };
    double *sDH = reinterpret_cast<double *>(lds);   // adjoint: as in the clean-cell kernel
    if (BWD)
        for (int p = lane; p < QPD_MAX_ORB; p += WAVE) sDH[p] = 0.0;
    auto flush_dh = [&](ConstSys &s) {
        if (!BWD) return;
        for (int p = lane; p < s.n; p += WAVE) {
            const double v = sDH[p];
            if (v != 0.0 && s.dh) atomicAdd(&s.dh[(int64_t)p * s.n + p], v);
            sDH[p] = 0.0;
        }
    };
    // plain grid-stride order: its items differ widely in cost (most leave
    // at once), and contiguous per-XCD ranges balanced them worse (n_orb 256,
    // 16+16, 10^5 determinants: 928 ms against 734 ms); claiming them one at
    // a time, as the clean-cell kernel does, costs more per item than the
    // locality brings (forward 844 ms against 744 ms, adjoint 1341 against 1112)
    for (int64_t it = blockIdx.x; it < total; it += gridDim.x) {
        if (it >= item_end[sid]) {
            flush_min(((ConstSys *)sys)[sid].min_delta_bits);
            flush_dh(((ConstSys *)sys)[sid]);
            while (it >= item_end[sid]) ibase = item_end[sid++];
            K = -1;
        }
        ConstSys &a = ((ConstSys *)sys)[sid];
        const int64_t item = it - ibase;
        if (item >= a.kl_off[a.n_keys]) continue;
        if (K < 0 || item >= kend) {
            if (K < 0 || item >= kend + (int64_t)WAVE * 1024) {
                int lo = 0, hi = a.n_keys;
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
        const bool want_sel = a.n_select > 0;

        unsigned off = BWD ? 8u * QPD_MAX_ORB : 0u;
        uint16_t *sVidx = carve<uint16_t>(lds, off, 2 * n);
        uint8_t *sVirt = carve<uint8_t>(lds, off, 2 * n);
        uint32_t *sF = carve<uint32_t>(lds, off, 16);
        int32_t *sFJ = carve<int32_t>(lds, off, FCAPC);
        uint32_t *sFer = carve<uint32_t>(lds, off, FCAPC);
        uint32_t *sFec = carve<uint32_t>(lds, off, FCAPC);
        uint32_t *sFm = carve<uint32_t>(lds, off, FCAPC);
        double *sFC = carve<double>(lds, off, FCAPC * NS);
        double *sDCF = carve<double>(lds, off, BWD ? FCAPC * NS : 1);

        const int64_t pos = a.kl_pos[item];
        if (pos < 0 || pos >= a.n_gen) continue;
        const int64_t g = a.gen_list ? (int64_t)a.gen_list[pos] : pos;
        const int det = a.perm[g];
        uint64_t Ib[2 * NINT];
#pragma unroll
        for (int w = 0; w < 2 * NINT; ++w) Ib[w] = a.dets[(int64_t)det * 2 * NINT + w];

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
        const int i1h = (s1 ? nup : 0) + occ_below<NINT>(Ib, s1, h1);
        const int i2h = (s2 ? nup : 0) + occ_below<NINT>(Ib, s2, h2);
        const int pb = i2h * (i2h - 1) / 2 + i1h;
        if (pb >= a.n_pairs) continue;
        const int64_t slot = pos * a.n_pairs + pb;

        for (int x = lane; x < 2 * n; x += WAVE) {
            const int s = x >= n ? 1 : 0, p = x - s * n;
            const int c = occ_below<NINT>(Ib, s, p);
            if (occ_bit<NINT>(Ib, s, p)) sVidx[x] = 0xFFFF;
            else { sVirt[s * n + p - c] = (uint8_t)p; sVidx[x] = (uint16_t)(p - c); }
        }
        if (lane < 16) sF[lane] = 0u;
        __syncthreads();

        const bool os = type == BT_OS;
        int rs, cs;
        if (os) { rs = h1 <= h2 ? 0 : 1; cs = 1 - rs; }
        else { rs = cs = s1; }
        const int hc0 = (s1 << 8) | h1, hc1 = (s2 << 8) | h2;
        const bool take = split_flags(a, g, n, nup, ndn, os, rs, hc0, hc1, sVidx, sF, sF + 8, lane);
        __syncthreads();
        if (!take) continue;
        bool anyf = false;
#pragma unroll
        for (int w = 0; w < 16; ++w) anyf |= sF[w] != 0u;
        if (!anyf) continue;

        // the fine entries (m = 1 or 2; a taken batch has no m = 0 entry)
        const int nv0 = n - nup, nv1 = n - ndn;
        int nfine = 0;
        {
            const int64_t cbeg = a.coff[g], cend = a.coff[g + 1];
            for (int64_t base = cbeg; base < cend; base += WAVE) {
                const int64_t e = base + lane;
                bool keep = false;
                CoarseEnt ce;
                int m = 3;
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
                const uint64_t mk = __ballot(keep);
                const int at = nfine + __popcll(mk & ((1ull << lane) - 1ull));
                if (keep && at < FCAPC) {
                    uint32_t er = 0u, ec = 0u;
                    int ner = 0, nec = 0;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const int ecode = ce.E[t];
                        if (ecode == 0xFFFF) continue;
                        const int es = ecode >> 8, ep = ecode & 255;
                        if (ep >= n) continue;
                        const int vi = sVidx[es * n + ep];
                        if (vi >= (es == 0 ? nv0 : nv1)) continue;
                        if (es == rs) { er |= (uint32_t)vi << (8 * ner); ner++; }
                        else if (os) { ec |= (uint32_t)vi << (8 * nec); nec++; }
                    }
                    sFJ[at] = ce.j;
                    sFer[at] = er;
                    sFec[at] = ec;
                    sFm[at] = (uint32_t)m | ((uint32_t)(ce.flags & 1) << 2) | ((uint32_t)ner << 4) | ((uint32_t)nec << 8);
#pragma unroll
                    for (int k = 0; k < NS; ++k) sFC[at * NS + k] = a.coefs[(int64_t)k * a.n_det + ce.j];
                }
                nfine += __popcll(mk);
            }
        }
        if (nfine > FCAPC) {
            // the general kernel takes this batch's flagged cells
            if (lane == 0) {
                const int b = a.nel + pb;
                atomicOr(&a.def_bits[g * a.nbw + (b >> 5)], 1u << (b & 31));
            }
            continue;
        }
        if (BWD)
            for (int x = lane; x < nfine * NS; x += WAVE) sDCF[x] = 0.0;
        __syncthreads();

        const double *Fg = a.F + g * 2 * n;
        const double HII = a.HII[g];
        const uint8_t *rvirt = sVirt + rs * n, *cvirt = sVirt + cs * n;
        const int nr = n - (rs ? ndn : nup), nc = n - (cs ? ndn : nup);
        // holes of the row and column spins (opposite spins), or both holes
        const int hu = h1, hd = h2;   // opposite spins: h1 up, h2 down
        const int hrs = os ? (rs == 0 ? hu : hd) : h1, hro = os ? (rs == 0 ? hd : hu) : h2;
        const int hcs = os ? hro : h1, hco = os ? hrs : h2;
        const double *blk = os ? a.I.X + (h1 <= h2 ? qtri(h1, h2) : qtri(h2, h1)) * n2
                               : a.I.Y + qtris(h1, h2) * (int64_t)P2;
        const double D0 = os ? HII - Fg[h1] - Fg[n + h2] + a.I.Jm[h1 * n + h2]
                             : HII - Fg[s1 * n + h1] - Fg[s1 * n + h2] + a.I.JK[h1 * n + h2];
        double E0[NS], cI[NS], gup[NS], dcI[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            E0[k] = a.E0[k];
            cI[k] = a.coefs[(int64_t)k * a.n_det + det];
            gup[k] = BWD ? a.gup[k] : 0.0;
            dcI[k] = 0.0;
        }
        double vbat = 0.0;   // adjoint: the item's total of v
        const uint64_t tau_key = want_sel ? bin_edge(__atomic_load_n(a.tau_bin, __ATOMIC_RELAXED)) : ~0ull;
        double esum[NS], ssum[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) { esum[k] = 0.0; ssum[k] = 0.0; }
        uint32_t cnt = 0, conn = 0;
        uint64_t fpsum = 0;
        bool appended = false;
        auto has4 = [](uint32_t v, int nv, int x) {
            bool r = false;
#pragma unroll
            for (int t = 0; t < 4; ++t) r |= (t < nv) && ((int)((v >> (8 * t)) & 255u) == x);
            return r;
        };
        auto fl = [&](int which, int i) -> bool { return (sF[which * 8 + (i >> 5)] >> (i & 31)) & 1u; };

        // lines: flagged rows (opposite spins: every column; same spin: the cells
        // below the flagged second index), then flagged columns (opposite spins:
        // the unflagged rows; same spin: the cells above the flagged first index
        // whose second index is unflagged)
        // the set bits of the flag words, rows then columns, in ascending order
        for (int wi = 0; wi < 16; ++wi) {
          uint32_t bits = (uint32_t)__builtin_amdgcn_readfirstlane((int)sF[wi]);
          while (bits) {
            const bool colline = wi >= 8;
            const int idx = (wi & 7) * 32 + __builtin_ctz(bits);
            bits &= bits - 1u;
            if (idx >= (colline && os ? nc : nr)) continue;
            const int len = os ? (colline ? nr : nc) : (colline ? nr - 1 - idx : idx);
            for (int p0 = 0; p0 < len; p0 += WAVE) {
                const int p = p0 + lane;
                int ia, ib;   // opposite spins: row, column; same spin: first < second
                if (os) { ia = colline ? p : idx; ib = colline ? idx : p; }
                else { ia = colline ? idx : p; ib = colline ? idx + 1 + p : idx; }
                const bool act = p < len && !(colline && fl(0, os ? ia : ib));
                bool live = act;
                double A[NS], D = DEAD_D;
                int pa = 0, pbb = 0;
#pragma unroll
                for (int k = 0; k < NS; ++k) A[k] = 0.0;
                uint32_t nco = 0;
                double Hv0 = 0.0;   // <I|H|alpha>
                if (act) {
                    pa = rvirt[ia];
                    pbb = os ? cvirt[ib] : rvirt[ib];
                    double x, Ga, Gb;
                    int sg;
                    if (os) {
                        // pa: particle of the row spin, pbb: of the column spin
                        x = blk[(int64_t)pa * n + pbb];
                        Ga = Fg[rs * n + pa] - a.I.JK[hrs * n + pa];
                        Ga -= a.I.Jm[hro * n + pa];
                        Gb = D0 + Fg[cs * n + pbb] - a.I.JK[hcs * n + pbb] - a.I.Jm[hco * n + pbb];
                        D = Gb + (Ga + a.I.Jm[pa * n + pbb]);
                        sg = between_parity<NINT>(Ib, rs, hrs, pa) ^ between_parity<NINT>(Ib, cs, hcs, pbb);
                    } else {
                        // pa < pbb, holes h1 < h2 of spin s1
                        x = blk[(int64_t)pbb * (pbb - 1) / 2 + pa];
                        Ga = Fg[rs * n + pa] - a.I.JK[h1 * n + pa];
                        Ga -= a.I.JK[h2 * n + pa];
                        Gb = Fg[rs * n + pbb] - a.I.JK[h1 * n + pbb];
                        Gb -= a.I.JK[h2 * n + pbb];
                        D = ((D0 + Gb) + Ga) + a.I.JK[pbb * n + pa];
                        // h1 -> pa, then h2 -> pbb on the intermediate determinant
                        const int lo = h2 < pbb ? h2 : pbb, hi = h2 < pbb ? pbb : h2;
                        sg = between_parity<NINT>(Ib, s1, h1, pa) ^ between_parity<NINT>(Ib, s1, h2, pbb) ^
                             (int)(lo < h1 && h1 < hi) ^ (int)(lo < pa && pa < hi);
                    }
                    const double Hv = sg ? -x : x;
                    Hv0 = Hv;
#pragma unroll
                    for (int k = 0; k < NS; ++k) A[k] = cI[k] * Hv;
                    for (int f = 0; f < nfine; ++f) {
                        const uint32_t fm = sFm[f];
                        const int m = fm & 3, ner = (fm >> 4) & 15, nec = (fm >> 8) & 15;
                        const uint32_t er = sFer[f];
                        const bool inA = has4(er, ner, ia);
                        const bool inB = os ? has4(sFec[f], nec, ib) : has4(er, ner, ib);
                        const bool touch = m == 1 ? (inA || inB) : (inA && inB);
                        if (!touch || !live) continue;
                        if ((fm >> 2) & 1u) { live = false; continue; }
                        uint64_t al[2 * NINT], jb[2 * NINT];
                        const uint64_t *Jp = a.dets + (int64_t)sFJ[f] * 2 * NINT;
#pragma unroll
                        for (int w = 0; w < 2 * NINT; ++w) {
                            al[w] = alpha_word<NINT>(Ib, w, hc0, hc1, pa, rs, pbb, cs);
                            jb[w] = Jp[w];
                        }
                        int deg;
                        const double v = sc_offdiag<NINT>(a.I, al, jb, &deg, nullptr);
                        if (deg == 0) { live = false; continue; }
                        if (deg > 2) continue;
                        nco++;
#pragma unroll
                        for (int k = 0; k < NS; ++k) A[k] = fma(sFC[f * NS + k], v, A[k]);
                    }
                }
                double ek[NS];
                double tsel = 0.0;
                double vc = 0.0;   // adjoint: sum over states of g A^2 / delta^2
                if (live) {
                    cnt++;
                    conn += nco;
                    double w[NS];
#pragma unroll
                    for (int k = 0; k < NS; ++k) {
                        const double delta = E0[k] - D;
                        const double rc = rcp1(delta);
                        const double e = (A[k] * A[k]) * rc;
                        ek[k] = e;
                        esum[k] += e;
                        ssum[k] = fma(e, rc, ssum[k]);
                        mind = min_abs(mind, delta);
                        tsel += e / a.maxc2[k];
                        if (BWD) {
                            w[k] = 2.0 * gup[k] * A[k] * rc;
                            vc = fma(gup[k] * e, rc, vc);
                            dcI[k] = fma(w[k], Hv0, dcI[k]);
                        }
                    }
                    if (BWD) {
                        // dE/dc_J for the determinants connected to this cell,
                        // and the one-electron part of a single excitation J ->
                        // alpha for dE/dh_pq (the matrix elements again, now
                        // that the numerator is known)
                        for (int f = 0; f < nfine; ++f) {
                            const uint32_t fm = sFm[f];
                            const int m = fm & 3, ner = (fm >> 4) & 15, nec = (fm >> 8) & 15;
                            const uint32_t er = sFer[f];
                            const bool inA = has4(er, ner, ia);
                            const bool inB = os ? has4(sFec[f], nec, ib) : has4(er, ner, ib);
                            if (!(m == 1 ? (inA || inB) : (inA && inB))) continue;
                            uint64_t al[2 * NINT], jb[2 * NINT];
                            const uint64_t *Jp = a.dets + (int64_t)sFJ[f] * 2 * NINT;
#pragma unroll
                            for (int ww = 0; ww < 2 * NINT; ++ww) {
                                al[ww] = alpha_word<NINT>(Ib, ww, hc0, hc1, pa, rs, pbb, cs);
                                jb[ww] = Jp[ww];
                            }
                            int deg, sgl[4];
                            const double v = sc_offdiag<NINT>(a.I, al, jb, &deg, sgl);
                            if (deg < 1 || deg > 2) continue;
                            double gs = 0.0;
#pragma unroll
                            for (int k = 0; k < NS; ++k) {
                                atomicAdd(&sDCF[f * NS + k], w[k] * v);
                                gs = fma(w[k], sFC[f * NS + k], gs);
                            }
                            if (deg == 1 && sgl[0] >= 0 && a.dh) {
                                const double gg = 0.5 * (sgl[3] < 0 ? -gs : gs);
                                atomicAdd(&a.dh[(int64_t)sgl[0] * n + sgl[1]], gg);
                                atomicAdd(&a.dh[(int64_t)sgl[1] * n + sgl[0]], gg);
                            }
                        }
                    }
                    if (FP) {
                        uint64_t al[2 * NINT];
#pragma unroll
                        for (int w = 0; w < 2 * NINT; ++w) al[w] = alpha_word<NINT>(Ib, w, hc0, hc1, pa, rs, pbb, cs);
                        fpsum += det_fold<NINT>(al);
                    }
                }
                if (BWD) {
                    // v to the external determinant's two particles: the line's
                    // own orbital once per line chunk, the other one per lane
                    vbat += vc;
                    const bool pa_line = os != colline;
                    if (vc != 0.0) sDH[pa_line ? pbb : pa] += vc;
                    const double tl = wsum(vc);
                    if (lane == 0 && tl != 0.0) sDH[os && colline ? cvirt[idx] : rvirt[idx]] += tl;
                }
                const uint64_t key = (uint64_t)__double_as_longlong(fabs(tsel));
                const bool cand = want_sel && live && key >= tau_key;
                const uint64_t mask = __ballot(cand);
                if (mask) {
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
                            const int up = os ? (rs == 0 ? pa : pbb) : pa;
                            const int dn = os ? (rs == 0 ? pbb : pa) : pbb;
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
            }
          }
        }

        // add to the clean-cell kernel's slot (it ran before: one writer at a time)
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            const double es = wsum(esum[k]), ss = wsum(ssum[k]);
            const double ds = BWD ? wsum(dcI[k]) : 0.0;
            if (lane == 0) {
                a.lean_eps[slot * NS + k] += es;
                a.lean_S[slot * NS + k] += ss;
                if (BWD) a.lean_dc[slot * NS + k] += ds;
            }
        }
        if (BWD) {
            // v to the orbitals every cell holds, and dE/dc_J to the connected J
            const double vb = wsum(vbat);
            if (vb != 0.0) {
                for (int p = lane; p < n; p += WAVE) {
                    const int np = (sVidx[p] == 0xFFFF ? 1 : 0) + (sVidx[n + p] == 0xFFFF ? 1 : 0) -
                                   ((s1 == 0 ? p == h1 : false) || (s2 == 0 ? p == h2 : false) ? 1 : 0) -
                                   ((s1 == 1 ? p == h1 : false) || (s2 == 1 ? p == h2 : false) ? 1 : 0);
                    if (np) sDH[p] += np * vb;
                }
            }
            __syncthreads();
            for (int x = lane; x < nfine * NS; x += WAVE) {
                const double v = sDCF[x];
                if (v != 0.0 && a.dc) atomicAdd(&a.dc[(int64_t)(x % NS) * a.n_det + sFJ[x / NS]], v);
            }
        }
        uint32_t ct = cnt, cn = conn;
        uint64_t ff = fpsum;
        for (int o = 32; o > 0; o >>= 1) {
            ct += __shfl_xor(ct, o);
            cn += __shfl_xor(cn, o);
            if (FP) ff += __shfl_xor(ff, o);
        }
        if (lane == 0) {
            if (ct) atomicAdd(&a.lean_cnt[pos], (unsigned long long)ct);
            if (cn) atomicAdd(&a.lean_conn[pos], (unsigned long long)cn);
            if (FP && ff) atomicAdd(&a.lean_fp[pos], (unsigned long long)ff);
        }
        if (want_sel && __ballot(appended)) {
            constexpr int PER = QP_HIST_BINS / WAVE;
            const unsigned int *hb = a.hist + lane * PER;
            uint32_t tot = 0;
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
    if (total > 0) {
        flush_min(((ConstSys *)sys)[sid < n_sys ? sid : n_sys - 1].min_delta_bits);
        flush_dh(((ConstSys *)sys)[sid < n_sys ? sid : n_sys - 1]);
    }
}

}  // namespace qplean

// the adjoint has no fingerprint variant: a fingerprinted adjoint is not split
template <int NINT, int NS, bool BWD>
void launch_lean(const SweepArgs *sys, const int64_t *item_end, int n_sys, bool fp, size_t lds, int grid,
                 hipStream_t st)
{
    if constexpr (BWD)
        hipLaunchKernelGGL((qplean::lean_kernel<NINT, NS, true, false>), dim3(grid), dim3(qplean::WAVE), lds, st,
                           sys, item_end, n_sys);
    else if (fp)
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
    const hipError_t e = BWD ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                   &blocks, qplean::lean_kernel<NINT, NS, BWD, false>, qplean::WAVE, lds)
                       : fp ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                  &blocks, qplean::lean_kernel<NINT, NS, false, true>, qplean::WAVE, lds)
                            : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                  &blocks, qplean::lean_kernel<NINT, NS, false, false>, qplean::WAVE, lds);
    if (e != hipSuccess) return 8;
    return blocks > 0 ? blocks : 1;
}

template <int NINT, int NS, bool BWD>
void launch_corr(const SweepArgs *sys, const int64_t *item_end, int n_sys, bool fp, size_t lds, int grid,
                 hipStream_t st)
{
    if constexpr (BWD)
        hipLaunchKernelGGL((qplean::corr_kernel<NINT, NS, true, false>), dim3(grid), dim3(qplean::WAVE), lds, st,
                           sys, item_end, n_sys);
    else if (fp)
        hipLaunchKernelGGL((qplean::corr_kernel<NINT, NS, false, true>), dim3(grid), dim3(qplean::WAVE), lds, st,
                           sys, item_end, n_sys);
    else
        hipLaunchKernelGGL((qplean::corr_kernel<NINT, NS, false, false>), dim3(grid), dim3(qplean::WAVE), lds, st,
                           sys, item_end, n_sys);
}

template <int NINT, int NS, bool BWD>
int corr_occupancy(size_t lds, bool fp)
{
    int blocks = 0;
    const hipError_t e = BWD ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                   &blocks, qplean::corr_kernel<NINT, NS, BWD, false>, qplean::WAVE, lds)
                       : fp ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                  &blocks, qplean::corr_kernel<NINT, NS, false, true>, qplean::WAVE, lds)
                            : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                  &blocks, qplean::corr_kernel<NINT, NS, false, false>, qplean::WAVE, lds);
    if (e != hipSuccess) return 8;
    return blocks > 0 ? blocks : 1;
}

#define QPL_INST(NI, NS)                                                                                        \
    template void launch_lean<NI, NS, false>(const SweepArgs *, const int64_t *, int, bool, size_t, int,         \
                                             hipStream_t);                                                       \
    template int lean_occupancy<NI, NS, false>(size_t, bool);                                                   \
    template void launch_lean<NI, NS, true>(const SweepArgs *, const int64_t *, int, bool, size_t, int,          \
                                            hipStream_t);                                                        \
    template int lean_occupancy<NI, NS, true>(size_t, bool);                                                    \
    template void launch_corr<NI, NS, false>(const SweepArgs *, const int64_t *, int, bool, size_t, int,         \
                                             hipStream_t);                                                       \
    template int corr_occupancy<NI, NS, false>(size_t, bool);                                                   \
    template void launch_corr<NI, NS, true>(const SweepArgs *, const int64_t *, int, bool, size_t, int,          \
                                            hipStream_t);                                                        \
    template int corr_occupancy<NI, NS, true>(size_t, bool);

QPL_INST(1, 1) QPL_INST(1, 2) QPL_INST(1, 3) QPL_INST(1, 4)
QPL_INST(2, 1) QPL_INST(2, 2) QPL_INST(2, 3) QPL_INST(2, 4)
QPL_INST(3, 1) QPL_INST(3, 2) QPL_INST(3, 3) QPL_INST(3, 4)
QPL_INST(4, 1) QPL_INST(4, 2) QPL_INST(4, 3) QPL_INST(4, 4)
