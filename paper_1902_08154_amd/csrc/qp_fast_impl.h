// qp_fast_impl.h -- the dense EN-PT2 / selection sweep for gfx950 (forward and
// adjoint): the kernel that handles almost every (generator, hole set) batch.
// Included by the two translation units that instantiate it (forward,
// adjoint), so the instantiations compile in parallel.
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
// -- and the dense pass only reads those buffers, in a branch taken by the
// few cells whose row or column carries a correction flag.  Batches that need
// more (an m = 0 entry, whose J touches every cell and may equal alpha, or
// more corrections than the buffers hold) are appended to a deferred list and
// processed afterwards by the general kernel; the per-generator reduction
// adds them in batch order, so results stay deterministic.
//
// The dense pass has one loop per batch type (single, same-spin double,
// opposite-spin double) so that each keeps only its own values in registers.
// Per particle index a 16-byte LDS entry holds the Fock-diagonal part of
// H_alpha,alpha, the orbital, the phase bit and the correction flags; a cell
// reads at most one such entry, its two integrals, and nothing else.  A cell
// that must not count (a banned alpha, an idle lane of the adjoint) gets
// numerator 0 and a denominator of 1e300, which makes every sum it enters
// exact and leaves the minimum |delta| untouched.
#pragma once
#include "qp_dev.h"
#if __has_include("qp_fast_caps_gen.h")
#include "qp_fast_caps_gen.h"
#else
#include "qp_fast_caps.h"
#endif

namespace qpfast {

constexpr int WAVE = 64;
constexpr int FCAP = QPF_FCAP;     // fine entries per batch
constexpr int L2CAP = QPF_L2CAP;   // m = 2 cells per batch
constexpr int PCAP = QPF_PCAP;     // m = 0 entries (integral planes) per batch
constexpr uint32_t FR = 1u << 8;    // row (OS) / second index (SS) carries a row or list correction
constexpr uint32_t FC = 1u << 9;    // column (OS) / first index (SS) carries a column correction
constexpr uint32_t SGN = 1u << 31;  // phase bit
constexpr double DEAD_D = -1e300;   // H_alpha,alpha of a cell that contributes nothing

struct FE {
    int32_t j;
    uint8_t m;
    uint8_t earlier;   // bit 0: J precedes the generator; bits 1-2: holes of the batch in I \ J
    uint8_t ner, nec;
    uint32_t er;   // row-spin virtual indices of E = J \ I (one per byte)
    uint32_t ec;   // column-spin virtual indices of E
};

// per particle index of one spin: Fock-diagonal part, orbital | flags | phase
struct __align__(16) PEnt {
    double G;
    uint32_t info;
    uint32_t pad;
};

__device__ __forceinline__ double frcp(double d)
{
    // reciprocal: the hardware estimate (relative error below 2^-22) and one
    // Newton step, which squares the error (below 2^-44, far inside the
    // 1e-10 relative tolerance of E_PT2); where the estimate is infinite
    // (d = 0 or |d| below 2^-1024) it is kept
    const double r0 = __builtin_amdgcn_rcp(d);
    const double r = fma(r0, fma(-d, r0, 1.0), r0);
    return __builtin_isinf(r0) ? r0 : r;
}

// min(m, |x|) in one instruction: both are non-negative results of
// arithmetic, never signalling NaNs, so no canonicalisation is needed
__device__ __forceinline__ double min_abs(double m, double x)
{
    double r;
    asm("v_min_f64 %0, %1, |%2|" : "=v"(r) : "v"(m), "v"(x));
    return r;
}

// keeps a wave-uniform value in a vector register: values read by every
// cell are cheaper there than in scalar registers the kernel runs short of
template <typename T>
__device__ __forceinline__ T in_vgpr(T x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// x with its sign flipped when bit 31 of s is set
__device__ __forceinline__ double flip(double x, uint32_t s)
{
    return __longlong_as_double(__double_as_longlong(x) ^ ((long long)(s & SGN) << 32));
}

__device__ __forceinline__ uint32_t rfl(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double rfl(double v)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
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

// one DPP step on a double: lane i receives src from the lane the control
// names (0 where that lane is outside the row, or the row is masked off)
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROW_MASK, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// sum over the 64 lanes with cross-lane data moves inside the VALU (DPP)
// rather than through the LDS crossbar: a scan within each 16-lane row, then
// row 0 -> 1 and 2 -> 3, then rows 0-1 -> 2-3; lane 63 holds the total
__device__ __forceinline__ double wsum_dpp(double v)
{
    v += dpp_f64<0x111, 0xf>(v);   // row_shr:1
    v += dpp_f64<0x112, 0xf>(v);   // row_shr:2
    v += dpp_f64<0x114, 0xf>(v);   // row_shr:4
    v += dpp_f64<0x118, 0xf>(v);   // row_shr:8
    v += dpp_f64<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v += dpp_f64<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// <J|H|alpha> for alpha = I - holes + particles (generic Slater-Condon)
template <int NINT, class Ints>
__device__ __forceinline__ double celem(const Ints &I, const uint64_t *Ib, int hc0, int hc1, int pa, int sa,
                                        int pb, int sb, const uint64_t *J, int *deg, int *sgl)
{
    uint64_t al[2 * NINT], jb[2 * NINT];
#pragma unroll
    for (int w = 0; w < 2 * NINT; ++w) {
        al[w] = alpha_word<NINT>(Ib, w, hc0, hc1, pa, sa, pb, sb);
        jb[w] = J[w];
    }
    return sc_offdiag<NINT>(I, al, jb, deg, sgl);
}

// LDS of one workgroup; nvm = largest number of virtual orbitals of a spin.
// Kept small on purpose: it bounds how many one-wave workgroups a CU holds.
inline size_t lds_bytes(int n, int nvm, int ns, bool bwd, int rscap, int cscap)
{
    size_t b = 0;
    auto add = [&](size_t bytes) { b = ((b + 15) & ~(size_t)15) + bytes; };
    add(16 * nvm);                    // row-spin particle table
    add(16 * nvm);                    // column-spin particle table
    add(8 * rscap * nvm);             // row buffers
    add(4 * (bwd ? rscap * nvm : 1)); // row buffer single-excitation info (adjoint)
    add(4 * (bwd ? cscap * nvm : 1)); // column buffer single-excitation info (adjoint)
    add(8 * cscap * nvm);             // column buffers
    add(8 * FCAP * ns);             // fine coefficients
    add(8 * L2CAP);                 // list values
    add(8 * (bwd ? FCAP * ns : 1)); // adjoint per-entry accumulators
    add(8 * (bwd ? n : 1));         // adjoint diagonal of dE/dh
    add(sizeof(FE) * FCAP);
    add(4 * L2CAP);
    add(4 * PCAP);                  // plane descriptors
    add(4 * rscap);
    add(4 * cscap);
    add(2 * 2 * n);                 // vidx
    add(2 * n);                     // occ
    add(2 * n);                     // virt
    add(2 * n);                     // cnt
    return b + 16;
}

// waves per SIMD the register allocation aims for: the highest target at
// which the kernel needs no spill memory (see qp_fast_caps.h)
template <int NINT, int NS, bool BWD, bool FP>
constexpr int waves_target() { return qpf_caps[BWD ? 1 : 0][FP ? 1 : 0][NINT - 1][NS - 1]; }

template <int NINT, int NS, bool BWD, bool FP>
__global__ __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(waves_target<NINT, NS, BWD, FP>(), 8)))
void fast_kernel(const SweepArgs *__restrict__ sys, const int64_t *__restrict__ item_end, int n_sys)
{
    extern __shared__ __align__(16) unsigned char lds[];
    const int lane = threadIdx.x;
    // the items of all systems, system after system, are dealt round-robin
    // over the persistent grid: a shared counter would cost one contended
    // device-scope atomic per item.  item_end[s] is the end of system s's items.
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
        const int RSCAP = a.rscap, CSCAP = a.cscap;
        const bool want_sel = a.n_select > 0;
        const int nvm = n - (a.nup < a.ndn ? a.nup : a.ndn);

        unsigned off = 0;
        PEnt *sRT = carve<PEnt>(lds, off, nvm);
        PEnt *sCT = carve<PEnt>(lds, off, nvm);
        double *sRB = carve<double>(lds, off, RSCAP * nvm);
        uint32_t *sRI = carve<uint32_t>(lds, off, BWD ? RSCAP * nvm : 1);
        uint32_t *sCI = carve<uint32_t>(lds, off, BWD ? CSCAP * nvm : 1);
        double *sCB = carve<double>(lds, off, CSCAP * nvm);
        double *sFC = carve<double>(lds, off, FCAP * NS);
        double *sLH = carve<double>(lds, off, L2CAP);
        double *sDCF = carve<double>(lds, off, BWD ? FCAP * NS : 1);
        double *sDHD = carve<double>(lds, off, BWD ? n : 1);
        FE *sFine = carve<FE>(lds, off, FCAP);
        uint32_t *sL = carve<uint32_t>(lds, off, L2CAP);   // i1 | i2 << 8 | f << 16 | ban << 24
        uint32_t *sPL = carve<uint32_t>(lds, off, PCAP);   // q1 | q2 << 8 | f << 16 | normal << 24
        uint32_t *sRSg = carve<uint32_t>(lds, off, RSCAP); // row | f << 16 | ban << 24
        uint32_t *sCSg = carve<uint32_t>(lds, off, CSCAP); // col | f << 16 | ban << 24
        uint16_t *sVidx = carve<uint16_t>(lds, off, 2 * n);
        uint8_t *sOcc = carve<uint8_t>(lds, off, 2 * n);
        uint8_t *sVirt = carve<uint8_t>(lds, off, 2 * n);
        uint8_t *sCnt = carve<uint8_t>(lds, off, 2 * n);

        double E0[NS], gup[NS], cI[NS], invm[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            E0[k] = in_vgpr(a.E0[k]);
            invm[k] = in_vgpr(a.inv_maxc2[k]);
            gup[k] = BWD ? a.gup[k] : 0.0;
        }

        // items run q-major over the call's generators: every rank, or a list
        // of ranks; g is the generator's rank, slot the item's partials
        const int q = (int)(item / a.n_gen);
        const int64_t gi = item - (int64_t)q * a.n_gen;
        const int64_t g = a.gen_list ? (int64_t)a.gen_list[gi] : gi;
        const int64_t slot = gi * Q + q;
        const int det = a.perm[g];

        uint64_t Ib[2 * NINT];
#pragma unroll
        for (int w = 0; w < 2 * NINT; ++w) Ib[w] = a.dets[(int64_t)det * 2 * NINT + w];
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
            if (occ) { sOcc[s * n + c] = (uint8_t)p; sVidx[x] = 0xFFFF; }
            else { sVirt[s * n + p - c] = (uint8_t)p; sVidx[x] = (uint16_t)(p - c); }
            if (BWD && s == 0) sDHD[p] = 0.0;
        }
#pragma unroll
        for (int k = 0; k < NS; ++k) cI[k] = a.coefs[(int64_t)k * a.n_det + det];
        const double HII = a.HII[g];
        const double *Fg = a.F + g * 2 * n;   // Fock diagonal of the generator, both spins
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
                h1 = i1 < nup ? sOcc[i1] : sOcc[n + i1 - nup];
                if (i2 < 0) {
                    type = BT_SINGLE; rs = cs = s1; nr = nc = s1 == 0 ? nv0 : nv1; sH = 0;
                    D0 = HII - Fg[s1 * n + h1];
                } else {
                    s2 = i2 < nup ? 0 : 1;
                    h2 = i2 < nup ? sOcc[i2] : sOcc[n + i2 - nup];
                    if (s2 == s1) {
                        type = BT_SS; rs = cs = s1; nr = nc = s1 == 0 ? nv0 : nv1;
                        sH = (sCnt[s1 * n + h1] + sCnt[s1 * n + h2] - 1) & 1;
                        D0 = HII - Fg[s1 * n + h1] - Fg[s1 * n + h2] + a.I.JK[h1 * n + h2];
                        blk = a.I.Y + qtris(h1, h2) * (int64_t)P2;
                    } else {
                        type = BT_OS;
                        if (h1 <= h2) { rs = 0; cs = 1; blk = a.I.X + qtri(h1, h2) * n2; }
                        else { rs = 1; cs = 0; blk = a.I.X + qtri(h2, h1) * n2; }
                        nr = rs == 0 ? nv0 : nv1; nc = cs == 0 ? nv0 : nv1;
                        sH = (sCnt[h1] + sCnt[n + h2]) & 1;
                        D0 = HII - Fg[h1] - Fg[n + h2] + a.I.Jm[h1 * n + h2];
                    }
                }
            }
            const int hc0 = (s1 << 8) | h1;
            const int hc1 = type == BT_SINGLE ? -1 : ((s2 << 8) | h2);
            const uint8_t *rvirt = sVirt + rs * n;
            const uint8_t *cvirt = sVirt + cs * n;
            const int hrs = type == BT_OS ? (rs == 0 ? h1 : h2) : h1;
            const int hro = type == BT_OS ? (rs == 0 ? h2 : h1) : (type == BT_SS ? h2 : -1);

            // split sweep: a hole-pair batch that no determinant touches in every
            // cell belongs to the clean-cell and split-correction kernels; the
            // batches marked before the sweep stay here
            if (a.split && type != BT_SINGLE && !((a.split_keep[g * a.nbw + (b >> 5)] >> (b & 31)) & 1u))
                continue;

            // particle tables: Fock-diagonal part of H_alpha,alpha and phase
            for (int i = lane; i < nr; i += WAVE) {
                const int p = rvirt[i];
                int par = sCnt[rs * n + p] - (hrs < p);
                double gv = Fg[rs * n + p] - a.I.JK[hrs * n + p];
                if (type == BT_SINGLE) par += sCnt[rs * n + h1];
                else if (type == BT_SS) { par -= (hro < p); gv -= a.I.JK[hro * n + p]; }
                else gv -= a.I.Jm[hro * n + p];
                PEnt e;
                e.G = gv; e.info = (uint32_t)p | ((par & 1) ? SGN : 0u); e.pad = 0;
                sRT[i] = e;
            }
            if (type == BT_OS) {
                const int hcs = cs == 0 ? h1 : h2, hco = cs == 0 ? h2 : h1;
                for (int c = lane; c < nc; c += WAVE) {
                    const int p = cvirt[c];
                    const int csg = (sH + sCnt[cs * n + p] - (hcs < p)) & 1;
                    PEnt e;
                    e.G = D0 + Fg[cs * n + p] - a.I.JK[hcs * n + p] - a.I.Jm[hco * n + p];
                    e.info = (uint32_t)p | (csg ? SGN : 0u); e.pad = 0;
                    sCT[c] = e;
                }
            }

            // ------------------------------------------------- fine filter
            int nfine = 0;
            bool slow = false;
            for (int64_t base = cbeg; base < cend; base += WAVE) {
                const int64_t e = base + lane;
                bool keep = false;
                CoarseEnt ce;
                int m = 0, inmask = 0;
                if (e < cend) {
                    ce = a.cent[e];
                    int dc = 0;
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
                const uint64_t mask = __ballot(keep);
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
                    f.j = ce.j; f.m = (uint8_t)m; f.earlier = (uint8_t)((ce.flags & 1) | (inmask << 1));
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
            int nl = 0, nrs = 0, ncs = 0, npl = 0;
            bool allban = false;
            if (!slow) {
                for (int f = 0; f < nfine; ++f) {
                    const FE fe = sFine[f];
                    const uint32_t ban = (fe.earlier & 1) ? (1u << 24) : 0u;
                    if (fe.m == 0) {
                        // J lacks only holes of this batch: it is connected to every
                        // cell.  If it precedes the generator, it owns them all.
                        if (fe.earlier & 1) { allban = true; break; }
                        // the adjoint of two or more states, or of three or more
                        // words per spin, leaves integral planes to the general
                        // kernel: their code would cost it registers
                        if (BWD && !(NS == 1 && NINT <= 2)) { slow = true; break; }
                        // J = I - H + E_J is itself a cell when it lacks both holes:
                        // that cell is internal
                        const bool caseA = (fe.ner + fe.nec) == (type == BT_SINGLE ? 1 : 2);
                        if (caseA) {
                            uint32_t cell;
                            if (type == BT_SINGLE) cell = bat(fe.er, 0);
                            else if (type == BT_OS) cell = bat(fe.er, 0) | (bat(fe.ec, 0) << 8);
                            else {
                                const int u = bat(fe.er, 0), v = bat(fe.er, 1);
                                cell = (u < v ? u : v) | ((u < v ? v : u) << 8);
                            }
                            if (nl < L2CAP && lane == 0) sL[nl] = cell | (f << 16) | (1u << 24);
                            nl++;
                        }
                        // cells sharing no particle with E_J are double excitations of
                        // J: one integral block Q = (holes J keeps) + E_J, indexed by
                        // the cell's particles (the integral plane)
                        if (type != BT_SINGLE) {
                            uint32_t desc;
                            if (type == BT_OS) {
                                // Q as (row-spin orbital, column-spin orbital)
                                int qr, qc;
                                if (caseA) { qr = rvirt[bat(fe.er, 0)]; qc = cvirt[bat(fe.ec, 0)]; }
                                else if (fe.ner == 1) { qr = rvirt[bat(fe.er, 0)]; qc = hro; }
                                else { qr = hrs; qc = cvirt[bat(fe.ec, 0)]; }
                                desc = qr | (qc << 8) | (qr <= qc ? (1u << 24) : 0u);
                            } else {
                                const int qa = rvirt[bat(fe.er, 0)];
                                // case B: the hole J keeps is the one not in I \ J
                                const int qb = caseA ? rvirt[bat(fe.er, 1)] : (((fe.earlier >> 1) & 1) ? h2 : h1);
                                desc = (qa < qb ? qa : qb) | ((qa < qb ? qb : qa) << 8);
                            }
                            if (npl < PCAP && lane == 0) sPL[npl] = desc | (f << 16);
                            npl++;
                        }
                        // the cells sharing one particle with E_J: rows and columns,
                        // as for m = 1 below
                    }
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
                if (nl > L2CAP || nrs > RSCAP || ncs > CSCAP || npl > PCAP) slow = true;
            }
            if (allban) {
                // every alpha of the batch belongs to an earlier generator
                __syncthreads();
                continue;
            }
            if (slow) {
                // the general kernel takes this batch
                if (lane == 0) atomicOr(&a.def_bits[g * a.nbw + (b >> 5)], 1u << (b & 31));
                __syncthreads();
                continue;
            }
            __syncthreads();

            // --------------------------------- evaluate correction elements
            if (lane < nl) {
                const uint32_t e = sL[lane];
                double v = 0.0;
                const int i1 = e & 255, i2 = (e >> 8) & 255;
                if (!((e >> 24) & 1)) {
                    const int f = (e >> 16) & 255;
                    int pa, sa, pb = -1, sb = cs;
                    if (type == BT_OS) { pa = rvirt[i1]; sa = rs; pb = cvirt[i2]; }
                    else if (type == BT_SS) { pa = rvirt[i1]; pb = rvirt[i2]; sa = sb = rs; }
                    else { pa = rvirt[i1]; sa = rs; }
                    int deg;
                    v = celem<NINT>(a.I, Ib, hc0, hc1, pa, sa, pb, sb, a.dets + (int64_t)sFine[f].j * 2 * NINT,
                                    &deg, nullptr);
                }
                sLH[lane] = v;
                // flag the cell's row (OS: first index; SS: second index; single: its particle)
                atomicOr(&sRT[type == BT_SS ? i2 : i1].info, FR);
            }
            // integral planes: per particle index, the sign of J -> alpha on that
            // index's spin and whether the index is a particle of J (such cells
            // belong to rows/columns).  Bits 4k..4k+1: first index (sign, mask),
            // 4k+2..4k+3: second index.
            for (int k = 0; k < npl; ++k) {
                const uint32_t desc = sPL[k];
                const int q1 = desc & 255, q2 = (desc >> 8) & 255;
                const FE fe = sFine[(desc >> 16) & 255];
                const uint64_t *Jb = a.dets + (int64_t)fe.j * 2 * NINT;
                if (type == BT_OS) {
                    for (int i = lane; i < nr; i += WAVE) {
                        const uint32_t sg = (uint32_t)between_parity<NINT>(Jb, rs, q1, rvirt[i]);
                        sRT[i].pad |= (sg | (has(fe.er, fe.ner, i) ? 2u : 0u)) << (4 * k);
                    }
                    for (int c = lane; c < nc; c += WAVE) {
                        const uint32_t sg = (uint32_t)between_parity<NINT>(Jb, cs, q2, cvirt[c]);
                        sCT[c].pad |= (sg | (has(fe.ec, fe.nec, c) ? 2u : 0u)) << (4 * k + 2);
                    }
                } else {
                    // same spin, q1 < q2, cell p1 < p2: the second excitation sees
                    // q1 removed and p1 added, which moves the parity by
                    // [q1 inside (q2, p2)] and [p1 > q2]
                    for (int i = lane; i < nr; i += WAVE) {
                        const int p = rvirt[i];
                        const int lo = q2 < p ? q2 : p, hi = q2 < p ? p : q2;
                        const uint32_t t1 = (uint32_t)between_parity<NINT>(Jb, rs, q1, p) ^ (p > q2 ? 1u : 0u);
                        const uint32_t t2 = (uint32_t)between_parity<NINT>(Jb, rs, q2, p) ^ ((lo < q1 && q1 < hi) ? 1u : 0u);
                        const uint32_t mk = has(fe.er, fe.ner, i) ? 2u : 0u;
                        sRT[i].pad |= (t1 | mk | (t2 << 2) | (mk << 2)) << (4 * k);
                    }
                }
            }
            if (lane < nrs) atomicOr(&sRT[sRSg[lane] & 0xFFFF].info, FR);
            if (lane < ncs) atomicOr(type == BT_OS ? &sCT[sCSg[lane] & 0xFFFF].info : &sRT[sCSg[lane] & 0xFFFF].info, FC);
            for (int s = 0; s < nrs; ++s) {
                const uint32_t sg = sRSg[s];
                if ((sg >> 24) & 1) continue;
                const int row = sg & 0xFFFF, f = (sg >> 16) & 255;
                const uint64_t *Jb = a.dets + (int64_t)sFine[f].j * 2 * NINT;
                // cells of the row: OS (row, c) for all c; SS (i1, row) for i1 < row;
                // single: every particle
                const int len = type == BT_OS ? nc : (type == BT_SS ? row : nr);
                for (int x = lane; x < len; x += WAVE) {
                    int pa, sa, pb = -1, sb = cs;
                    if (type == BT_OS) { pa = rvirt[row]; sa = rs; pb = cvirt[x]; }
                    else if (type == BT_SS) { pa = rvirt[x]; pb = rvirt[row]; sa = sb = rs; }
                    else { pa = rvirt[x]; sa = rs; }
                    int deg, sgl[4] = {-1, -1, 0, 0};
                    const double v = celem<NINT>(a.I, Ib, hc0, hc1, pa, sa, pb, sb, Jb, &deg, BWD ? sgl : nullptr);
                    sRB[s * nvm + x] = v;
                    if (BWD) sRI[s * nvm + x] = deg == 1 ? (uint32_t)(sgl[0] | (sgl[1] << 8) | ((sgl[3] < 0) << 16) | (1u << 17)) : 0u;
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
                    uint32_t sci = 0u;
                    // OS: cells (r, col), r not in E_r; SS: cells (col, r), r > col, r not in E
                    const bool use = !has(fe.er, fe.ner, r) && (type == BT_OS || r > col);
                    if (use) {
                        int pa, sa, pb, sb;
                        if (type == BT_OS) { pa = rvirt[r]; sa = rs; pb = cvirt[col]; sb = cs; }
                        else { pa = rvirt[col]; pb = rvirt[r]; sa = sb = rs; }
                        int deg, sgl[4] = {-1, -1, 0, 0};
                        v = celem<NINT>(a.I, Ib, hc0, hc1, pa, sa, pb, sb, Jb, &deg, BWD ? sgl : nullptr);
                        if (BWD) sci = deg == 1 ? (uint32_t)(sgl[0] | (sgl[1] << 8) | ((sgl[3] < 0) << 16) | (1u << 17)) : 0u;
                    }
                    sCB[s * nvm + r] = v;
                    if (BWD) sCI[s * nvm + r] = sci;
                }
            }
            if (BWD) for (int x = lane; x < FCAP * NS; x += WAVE) sDCF[x] = 0.0;
            __syncthreads();

            // without selection no value passes either test (|t| has no sign bit)
            const uint64_t tau_key = want_sel ? bin_edge(__atomic_load_n(a.tau_bin, __ATOMIC_RELAXED)) : ~0ull;
            const double tau_val = in_vgpr(want_sel ? __longlong_as_double((long long)tau_key) * (1.0 - 1e-12)
                                                    : __builtin_inf());
            bool appended = false;
            double vbatch = 0.0;
            uint32_t nban = 0;

            // ------------------------------------------- per-cell helpers
            // corrections of cell (i1, i2): A += sum_J c_J <J|H|alpha>; true if banned
            auto gather = [&](int i1, int i2, double (&A)[NS], uint32_t &nco) -> bool {
                bool banned = false;
                for (int s = 0; s < nrs; ++s) {
                    const uint32_t sg = sRSg[s];
                    const int row = sg & 0xFFFF;
                    const bool hit = type == BT_OS ? row == i1 : (type == BT_SS ? row == i2 : true);
                    const int x_ = type == BT_OS ? i2 : i1;
                    if (hit) {
                        if ((sg >> 24) & 1) banned = true;
                        else {
                            const int f = (sg >> 16) & 255;
                            const double v = sRB[s * nvm + x_];
                            nco++;
#pragma unroll
                            for (int k = 0; k < NS; ++k) A[k] = fma(sFC[f * NS + k], v, A[k]);
                        }
                    }
                }
                for (int s = 0; s < ncs; ++s) {
                    const uint32_t sg = sCSg[s];
                    const int col = sg & 0xFFFF, f = (sg >> 16) & 255;
                    const int rowi = type == BT_OS ? i1 : i2;
                    const bool hit = (type == BT_OS ? i2 : i1) == col && !has(sFine[f].er, sFine[f].ner, rowi);
                    if (hit) {
                        if ((sg >> 24) & 1) banned = true;
                        else {
                            const double v = sCB[s * nvm + rowi];
                            nco++;
#pragma unroll
                            for (int k = 0; k < NS; ++k) A[k] = fma(sFC[f * NS + k], v, A[k]);
                        }
                    }
                }
                for (int t = 0; t < nl; ++t) {
                    const uint32_t e = sL[t];
                    if ((int)(e & 255) == i1 && (int)((e >> 8) & 255) == i2) {
                        if ((e >> 24) & 1) banned = true;
                        else {
                            const int f = (e >> 16) & 255;
                            nco++;
#pragma unroll
                            for (int k = 0; k < NS; ++k) A[k] = fma(sFC[f * NS + k], sLH[t], A[k]);
                        }
                    }
                }
                return banned;
            };
            // adjoint of the corrections: dE/dc_J += w <J|H|alpha>, and the
            // single-excitation elements' dependence on h
            auto gather_bwd = [&](int i1, int i2, const double (&w)[NS]) {
                for (int s = 0; s < nrs; ++s) {
                    const uint32_t sg = sRSg[s];
                    if ((sg >> 24) & 1) continue;
                    const int row = sg & 0xFFFF, f = (sg >> 16) & 255;
                    const bool hit = type == BT_OS ? row == i1 : (type == BT_SS ? row == i2 : true);
                    const int x_ = type == BT_OS ? i2 : i1;
                    if (!hit) continue;
                    const double hv = sRB[s * nvm + x_];
#pragma unroll
                    for (int k = 0; k < NS; ++k) atomicAdd(&sDCF[f * NS + k], w[k] * hv);
                    const uint32_t inf = sRI[s * nvm + x_];
                    if (((inf >> 17) & 1u) && a.dh) {
                        double gs = 0.0;
#pragma unroll
                        for (int k = 0; k < NS; ++k) gs += w[k] * sFC[f * NS + k];
                        const double gg = 0.5 * (((inf >> 16) & 1u) ? -gs : gs);
                        const int hh = inf & 255, pp = (inf >> 8) & 255;
                        atomicAdd(&a.dh[(int64_t)hh * n + pp], gg);
                        atomicAdd(&a.dh[(int64_t)pp * n + hh], gg);
                    }
                }
                for (int s = 0; s < ncs; ++s) {
                    const uint32_t sg = sCSg[s];
                    if ((sg >> 24) & 1) continue;
                    const int col = sg & 0xFFFF, f = (sg >> 16) & 255;
                    const int rowi = type == BT_OS ? i1 : i2;
                    if ((type == BT_OS ? i2 : i1) == col && !has(sFine[f].er, sFine[f].ner, rowi)) {
                        const double hv = sCB[s * nvm + rowi];
#pragma unroll
                        for (int k = 0; k < NS; ++k) atomicAdd(&sDCF[f * NS + k], w[k] * hv);
                        // a single excitation J -> alpha (the lines of an integral
                        // plane can be): its one-electron part feeds dE/dh
                        const uint32_t inf = sCI[s * nvm + rowi];
                        if (((inf >> 17) & 1u) && a.dh) {
                            double gs = 0.0;
#pragma unroll
                            for (int k = 0; k < NS; ++k) gs += w[k] * sFC[f * NS + k];
                            const double gg = 0.5 * (((inf >> 16) & 1u) ? -gs : gs);
                            const int hh = inf & 255, pp = (inf >> 8) & 255;
                            atomicAdd(&a.dh[(int64_t)hh * n + pp], gg);
                            atomicAdd(&a.dh[(int64_t)pp * n + hh], gg);
                        }
                    }
                }
                for (int t = 0; t < nl; ++t) {
                    const uint32_t e = sL[t];
                    if ((int)(e & 255) == i1 && (int)((e >> 8) & 255) == i2 && !((e >> 24) & 1)) {
                        const int f = (e >> 16) & 255;
#pragma unroll
                        for (int k = 0; k < NS; ++k) atomicAdd(&sDCF[f * NS + k], w[k] * sLH[t]);
                    }
                }
            };
            // energy, its accumulations and the selection pretest of one cell
            auto finish = [&](const double (&A)[NS], double D, double (&ek)[NS], double (&w)[NS], double &vsum) -> double {
                double tsel = 0.0;
                vsum = 0.0;
#pragma unroll
                for (int k = 0; k < NS; ++k) {
                    const double delta = E0[k] - D;
                    const double rc = frcp(delta);
                    const double e = (A[k] * A[k]) * rc;
                    ek[k] = e;
                    esum[k] += e;
                    ssum[k] = fma(e, rc, ssum[k]);
                    mind = min_abs(mind, delta);
                    tsel = fma(e, invm[k], tsel);
                    if (BWD) {
                        w[k] = 2.0 * gup[k] * A[k] * rc;
                        vsum += gup[k] * e * rc;
                    }
                }
                return tsel;
            };
            // exact key test and append of the lanes whose pretest passed
            auto select = [&](bool cand, const double (&ek)[NS], int pa, int pb) {
                uint64_t key = 0;
                if (cand) {
                    double t = 0.0;
#pragma unroll
                    for (int k = 0; k < NS; ++k) t += ek[k] / a.maxc2[k];
                    key = (uint64_t)__double_as_longlong(fabs(t));
                    cand = key >= tau_key;
                }
                const uint64_t mask = __ballot(cand);
                if (!mask) return;
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
            };
            auto fold = [&](int pa, int pb) {
                uint64_t al[2 * NINT];
#pragma unroll
                for (int w = 0; w < 2 * NINT; ++w) al[w] = alpha_word<NINT>(Ib, w, hc0, hc1, pa, rs, pb, cs);
                return det_fold<NINT>(al);
            };

            // one cell with all its corrections, outside the dense loops (the
            // column pass): element x with phase bits sg, diagonal D
            auto post_cell = [&](int i1, int i2, double x, uint32_t sg, double D, int pa, int pb) {
                const double Hv = flip(x, sg);
                double A[NS];
#pragma unroll
                for (int k = 0; k < NS; ++k) A[k] = cI[k] * Hv;
                bool live = true;
                uint32_t nco = 0;
                if (gather(i1, i2, A, nco)) {
                    live = false; D = DEAD_D; nban++;
#pragma unroll
                    for (int k = 0; k < NS; ++k) A[k] = 0.0;
                } else {
                    conn += nco;
                }
                double ek[NS], w[NS], vsum;
                const double tsel = finish(A, D, ek, w, vsum);
                if (FP && live) fpsum += fold(pa, pb);
                {
                    const bool c = live && fabs(tsel) >= tau_val;
                    if (__builtin_amdgcn_ballot_w64(c)) select(c, ek, pa, pb);
                }
                if (BWD) {
#pragma unroll
                    for (int k = 0; k < NS; ++k) dcI[k] = fma(w[k], Hv, dcI[k]);
                    vbatch += vsum;
                    if (vsum != 0.0) {
                        atomicAdd(&sDHD[pa], vsum);
                        atomicAdd(&sDHD[pb], vsum);
                    }
                    if (live) gather_bwd(i1, i2, w);
                }
            };

            // blocks of the integral planes
            const double *pblk[PCAP];
#pragma unroll
            for (int k = 0; k < PCAP; ++k) {
                pblk[k] = a.I.Y;
                if (k < npl) {
                    const uint32_t desc = sPL[k];
                    const int q1 = desc & 255, q2 = (desc >> 8) & 255;
                    pblk[k] = type == BT_OS ? a.I.X + qtri(q1 < q2 ? q1 : q2, q1 < q2 ? q2 : q1) * n2
                                            : a.I.Y + qtris(q1, q2) * (int64_t)P2;
                }
            }
            // one cell of a batch with integral planes, evaluated exactly: u1/u2
            // are the plane bits of its first/second index, o_norm/o_tran its
            // offset in a plane block read as [first][second] or transposed
            double pdc[PCAP][NS];
#pragma unroll
            for (int k = 0; k < PCAP; ++k)
#pragma unroll
                for (int t = 0; t < NS; ++t) pdc[k][t] = 0.0;
            auto plane_flush = [&]() {
                if (!BWD) return;
#pragma unroll
                for (int k = 0; k < PCAP; ++k)
#pragma unroll
                    for (int t = 0; t < NS; ++t) {
                        const double v = wsum_dpp(pdc[k][t]);
                        if (k < npl && lane == 0 && v != 0.0) sDCF[((sPL[k] >> 16) & 255) * NS + t] += v;
                    }
            };
            // act false: a lane with no cell (the adjoint runs every lane so that
            // row sums can be wave reductions); it adds nothing.  vs returns the
            // cell's sum over states of g A^2 / delta^2 for dE/dh's diagonal.
            auto plane_cell = [&](int i1, int i2, double x, uint32_t sg, double D, int pa, int pb, uint32_t u1,
                                  uint32_t u2, int o_norm, int o_tran, bool needg, bool act, double &vs) {
                const double Hv = act ? flip(x, sg) : 0.0;
                double A[NS], vv[PCAP];
#pragma unroll
                for (int k = 0; k < NS; ++k) A[k] = cI[k] * Hv;
                if (!act) D = DEAD_D;
                uint32_t nco = 0;
#pragma unroll
                for (int k = 0; k < PCAP; ++k) {
                    vv[k] = 0.0;
                    const uint32_t b1 = u1 >> (4 * k), b2 = u2 >> (4 * k);
                    if (act && k < npl && !((b1 & 2u) | (b2 & 8u))) {
                        const uint32_t desc = sPL[k];
                        const double v = pblk[k][((desc >> 24) & 1u) ? o_norm : o_tran];
                        vv[k] = ((b1 ^ (b2 >> 2)) & 1u) ? -v : v;
                        const int f = (desc >> 16) & 255;
#pragma unroll
                        for (int t = 0; t < NS; ++t) A[t] = fma(sFC[f * NS + t], vv[k], A[t]);
                        nco++;
                    }
                }
                bool live = act;
                if (act && needg && gather(i1, i2, A, nco)) {
                    live = false; D = DEAD_D; nban++;
#pragma unroll
                    for (int k = 0; k < NS; ++k) A[k] = 0.0;
                }
                if (live) conn += nco;
                double ek[NS], w[NS], vsum;
                const double tsel = finish(A, D, ek, w, vsum);
                vs = vsum;
                if (FP && live) fpsum += fold(pa, pb);
                {
                    const bool c = live && fabs(tsel) >= tau_val;
                    if (__builtin_amdgcn_ballot_w64(c)) select(c, ek, pa, pb);
                }
                if (BWD) {
#pragma unroll
                    for (int k = 0; k < NS; ++k) dcI[k] = fma(w[k], Hv, dcI[k]);
                    vbatch += vsum;
                    if (live) {
                        if (needg) gather_bwd(i1, i2, w);
                        // dE/dc of the planes' J: lane sums, reduced after the loop
#pragma unroll
                        for (int k = 0; k < PCAP; ++k)
#pragma unroll
                            for (int t = 0; t < NS; ++t) pdc[k][t] = fma(w[t], vv[k], pdc[k][t]);
                    }
                }
            };

            // --------------------------------------------------- dense pass
            if ((!BWD || (NS == 1 && NINT <= 2)) && type == BT_OS && npl > 0) {
                if (lane == 0) cnt += (uint32_t)(nr * nc);
                const double *Jm = a.I.Jm;
                for (int c0 = 0; c0 < nc; c0 += WAVE) {
                    const int l = c0 + lane;
                    const bool lok = l < nc;
                    if (BWD || lok) {
                        const PEnt ce = sCT[lok ? l : nc - 1];
                        const int pcol = ce.info & 255;
                        double colacc = 0.0;
                        for (int r = 0; r < nr; ++r) {
                            const PEnt re = sRT[r];
                            const int pr = re.info & 255;
                            const double xj = Jm[pr * n + pcol];
                            double vs;
                            plane_cell(r, l, blk[pr * n + pcol], re.info ^ ce.info, (ce.G + re.G) + xj, pr, pcol,
                                       re.pad, ce.pad, pr * n + pcol, pcol * n + pr,
                                       ((re.info & FR) | (ce.info & FC)) != 0u, lok, vs);
                            if (BWD) {
                                // the row's orbital is the same on every lane
                                const double rsum = wsum_dpp(vs);
                                if (lane == 0 && rsum != 0.0) sDHD[pr] += rsum;
                                colacc += vs;
                            }
                        }
                        if (BWD && lok && colacc != 0.0) atomicAdd(&sDHD[pcol], colacc);
                    }
                }
                plane_flush();
            } else if ((!BWD || (NS == 1 && NINT <= 2)) && type == BT_SS && npl > 0) {
                if (lane == 0) cnt += (uint32_t)(nr * (nr - 1) / 2);
                const double *JK = a.I.JK;
                const uint32_t shb = sH ? SGN : 0u;
                const int nfr = nr / 2;
                for (int c0 = 0; c0 < nr; c0 += WAVE) {
                    const int l = c0 + lane;
                    for (int r = 1; r <= nfr; ++r) {
                        const bool pA = l < r;
                        const bool act = l < nr && (pA || nr - r > r);
                        if (BWD || act) {
                            // folded row r: cells (l, r) for l < r, (l - r, nr - r) after
                            const bool useA = pA || !act;
                            const int i1 = act ? (pA ? l : l - r) : 0, i2 = useA ? r : nr - r;
                            const PEnt e1 = sRT[i1], e2 = sRT[i2];
                            const int p1 = e1.info & 255, p2 = e2.info & 255;
                            const int off = p2 * (p2 - 1) / 2 + p1;
                            const double xj = JK[p2 * n + p1];
                            double vs;
                            plane_cell(i1, i2, blk[off], e1.info ^ e2.info ^ shb, ((D0 + e2.G) + e1.G) + xj, p1, p2,
                                       e1.pad, e2.pad, off, off, ((e2.info & FR) | (e1.info & FC)) != 0u, act, vs);
                            if (BWD) {
                                // the second index is r on the lanes of part A and nr - r
                                // on those of part B
                                const double sA = wsum_dpp(useA ? vs : 0.0), sB = wsum_dpp(useA ? 0.0 : vs);
                                if (lane == 0) {
                                    if (sA != 0.0) sDHD[sRT[r].info & 255] += sA;
                                    if (sB != 0.0) sDHD[sRT[nr - r].info & 255] += sB;
                                }
                                if (vs != 0.0) atomicAdd(&sDHD[p1], vs);
                            }
                        }
                    }
                }
                plane_flush();
            } else if (type == BT_OS) {
                if (lane == 0) cnt += (uint32_t)(nr * nc);
                const double *Jm = a.I.Jm;
                for (int c0 = 0; c0 < nc; c0 += WAVE) {
                    const int l = c0 + lane;
                    const bool lok = l < nc;
                    const int lc = lok ? l : nc - 1;
                    const PEnt ce = sCT[lc];
                    const int pcol = ce.info & 255;
                    // a lane past the last column, or on a flagged column (the column
                    // pass finishes those), adds nothing in unflagged rows: a zero
                    // numerator and a diagonal that makes the denominator huge, set
                    // once here instead of per cell
                    const bool quiet = !lok || (ce.info & FC) != 0u;
                    const double Gq = quiet ? DEAD_D : ce.G;
                    double cq[NS];
#pragma unroll
                    for (int k = 0; k < NS; ++k) cq[k] = quiet ? 0.0 : cI[k];
                    double colacc = 0.0;
                    if (BWD || lok) {
                        // the next row's integrals are loaded as soon as this row's
                        // have been used, into the same registers, so that their
                        // latency overlaps the rest of the cell; each generator
                        // starts at its own row so that waves sharing a block do not
                        // all read the same lines at once
                        const unsigned uc = (unsigned)pcol;
                        int r = (int)(g % nr);
                        uint32_t rinfo = rfl(sRT[r].info);
                        double xc = (blk + (rinfo & 255) * n)[uc];
                        double xjc = (Jm + (rinfo & 255) * n)[uc];
                        for (int t = 0; t < nr; ++t, r = r + 1 == nr ? 0 : r + 1) {
                            const uint32_t ri = rinfo;
                            const int pr = ri & 255;
                            const double gx = rfl(sRT[r].G) + xjc;   // row part of H_aa
                            const double Hv = flip(xc, ri ^ ce.info);
                            {
                                const int rn = r + 1 == nr ? 0 : r + 1;
                                rinfo = rfl(sRT[rn].info);
                                xc = (blk + (rinfo & 255) * n)[uc];
                                xjc = (Jm + (rinfo & 255) * n)[uc];
                            }
                            double D = Gq + gx;
                            double A[NS];
#pragma unroll
                            for (int k = 0; k < NS; ++k) A[k] = cq[k] * Hv;
                            bool live = !quiet;
                            // a flagged row gathers its corrections here, all lanes at
                            // once, flagged columns included
                            const bool rowf = (ri & FR) != 0u;
                            if (rowf && lok) {
                                D = ce.G + gx;
#pragma unroll
                                for (int k = 0; k < NS; ++k) A[k] = cI[k] * Hv;
                                live = true;
                                uint32_t nco = 0;
                                if (gather(r, l, A, nco)) {
                                    live = false; D = DEAD_D; nban++;
#pragma unroll
                                    for (int k = 0; k < NS; ++k) A[k] = 0.0;
                                } else {
                                    conn += nco;
                                }
                            }
                            double ek[NS], w[NS], vsum;
                            const double tsel = finish(A, D, ek, w, vsum);
                            if (FP && live) fpsum += fold(pr, pcol);
                            {
                                const bool c = live && fabs(tsel) >= tau_val;
                                if (__builtin_amdgcn_ballot_w64(c)) select(c, ek, pr, pcol);
                            }
                            if (BWD) {
#pragma unroll
                                for (int k = 0; k < NS; ++k) dcI[k] = fma(w[k], Hv, dcI[k]);
                                vbatch += vsum;
                                const double rsum = wsum_dpp(vsum);
                                if (lane == 0 && rsum != 0.0) sDHD[pr] += rsum;
                                colacc += vsum;
                                if (live && rowf) gather_bwd(r, l, w);
                            }
                        }
                    }
                    if (BWD && lok && colacc != 0.0) atomicAdd(&sDHD[pcol], colacc);
                }
                // column pass: cells of flagged columns in unflagged rows
                for (int s = 0; s < ncs; ++s) {
                    const int col = sCSg[s] & 0xFFFF;
                    bool seen = false;
                    for (int t = 0; t < s; ++t) seen |= (int)(sCSg[t] & 0xFFFF) == col;
                    if (seen) continue;
                    const PEnt ce = sCT[col];
                    const int pcol = ce.info & 255;
                    for (int r0 = 0; r0 < nr; r0 += WAVE) {
                        const int r = r0 + lane;
                        const PEnt re = sRT[r < nr ? r : 0];
                        if (r < nr && !(re.info & FR)) {
                            const int pr = re.info & 255;
                            const double xj = Jm[pr * n + pcol];
                            post_cell(r, col, blk[pr * n + pcol], re.info ^ ce.info, (ce.G + re.G) + xj, pr, pcol);
                        }
                    }
                }
            } else if (type == BT_SS) {
                if (lane == 0) cnt += (uint32_t)(nr * (nr - 1) / 2);
                const double *JK = a.I.JK;
                const uint32_t shb = sH ? SGN : 0u;
                for (int c0 = 0; c0 < nr; c0 += WAVE) {
                    const int l = c0 + lane;
                    const bool lok = l < nr;
                    if (BWD || lok) {
                        // folded rows: row r holds cells (l, r) for l < r and
                        // (l - r, nr - r) for l >= r, so every row has nr cells.
                        // The lane's cell in folded row rr: first index, second
                        // index (A: rr itself, B: nr - rr), active or not.
                        auto pick = [&](int rr, int &i1, int &i2, bool &act, bool &useA) {
                            const bool pA = l < rr;
                            act = lok && (pA || nr - rr > rr);
                            useA = pA || !act;
                            i1 = act ? (pA ? l : l - rr) : 0;
                            i2 = useA ? rr : nr - rr;
                        };
                        // the next row's integrals are loaded as soon as this row's
                        // have been used, into the same registers
                        auto ss_offsets = [&](int rr, unsigned &ob, unsigned &oj) {
                            int i1, i2;
                            bool act, useA;
                            pick(rr, i1, i2, act, useA);
                            const int p1 = sRT[i1].info & 255, p2 = sRT[i2].info & 255;
                            ob = (unsigned)(p2 * (p2 - 1) / 2 + p1);
                            oj = (unsigned)(p2 * n + p1);
                        };
                        const int nfr = nr / 2;
                        int r = nfr > 0 ? 1 + (int)(g % nfr) : 1;
                        double xc = 0.0, xjc = 0.0;
                        if (nfr > 0) {
                            unsigned ob, oj;
                            ss_offsets(r, ob, oj);
                            xc = blk[ob];
                            xjc = JK[oj];
                        }
                        for (int t = 0; t < nfr; ++t, r = r == nfr ? 1 : r + 1) {
                            const bool validB = nr - r > r;
                            const uint32_t ia = rfl(sRT[r].info), ib = rfl(sRT[nr - r].info);
                            const double DA = D0 + rfl(sRT[r].G), DB = D0 + rfl(sRT[nr - r].G);
                            int i1, i2;
                            bool act, useA;
                            pick(r, i1, i2, act, useA);
                            const PEnt e1 = sRT[i1];
                            const uint32_t i2info = useA ? ia : ib;
                            const int p1 = e1.info & 255, p2 = i2info & 255;
                            const double Hv0 = flip(xc, e1.info ^ i2info ^ shb);
                            const double D0c = ((useA ? DA : DB) + e1.G) + xjc;
                            {
                                unsigned ob, oj;
                                ss_offsets(r == nfr ? 1 : r + 1, ob, oj);
                                xc = blk[ob];
                                xjc = JK[oj];
                            }
                            if (BWD || act) {
                                const double Hv = Hv0;
                                double D = D0c;
                                double A[NS];
#pragma unroll
                                for (int k = 0; k < NS; ++k) A[k] = cI[k] * Hv;
                                bool live = true;
                                if (BWD && !act) {
                                    live = false; D = DEAD_D;
#pragma unroll
                                    for (int k = 0; k < NS; ++k) A[k] = 0.0;
                                }
                                const bool rowf = (i2info & FR) != 0u;
                                if (live && rowf) {
                                    uint32_t nco = 0;
                                    if (gather(i1, i2, A, nco)) {
                                        live = false; D = DEAD_D; nban++;
#pragma unroll
                                        for (int k = 0; k < NS; ++k) A[k] = 0.0;
                                    } else {
                                        conn += nco;
                                    }
                                } else if ((e1.info & FC) != 0u) {
                                    live = false; D = DEAD_D;
#pragma unroll
                                    for (int k = 0; k < NS; ++k) A[k] = 0.0;
                                }
                                double ek[NS], w[NS], vsum;
                                const double tsel = finish(A, D, ek, w, vsum);
                                if (FP && live) fpsum += fold(p1, p2);
                                {
                                    const bool c = live && fabs(tsel) >= tau_val;
                                    if (__builtin_amdgcn_ballot_w64(c)) select(c, ek, p1, p2);
                                }
                                if (BWD) {
#pragma unroll
                                    for (int k = 0; k < NS; ++k) dcI[k] = fma(w[k], Hv, dcI[k]);
                                    vbatch += vsum;
                                    const double sA = wsum_dpp(useA ? vsum : 0.0), sB = wsum_dpp(useA ? 0.0 : vsum);
                                    if (lane == 0) {
                                        if (sA != 0.0) sDHD[ia & 255] += sA;
                                        if (sB != 0.0 && validB) sDHD[ib & 255] += sB;
                                    }
                                    if (vsum != 0.0) atomicAdd(&sDHD[p1], vsum);
                                    if (live && rowf) gather_bwd(i1, i2, w);
                                }
                            }
                        }
                    }
                }
                // column pass: cells (ie, i2), i2 > ie, of flagged first indices in
                // rows whose second index carries no flag
                for (int s = 0; s < ncs; ++s) {
                    const int ie = sCSg[s] & 0xFFFF;
                    bool seen = false;
                    for (int t = 0; t < s; ++t) seen |= (int)(sCSg[t] & 0xFFFF) == ie;
                    if (seen) continue;
                    const PEnt e1 = sRT[ie];
                    const int p1 = e1.info & 255;
                    for (int j0 = ie + 1; j0 < nr; j0 += WAVE) {
                        const int i2 = j0 + lane;
                        const PEnt e2 = sRT[i2 < nr ? i2 : ie];
                        if (i2 < nr && !(e2.info & FR)) {
                            const int p2 = e2.info & 255;
                            const double xj = JK[p2 * n + p1];
                            post_cell(ie, i2, blk[p2 * (p2 - 1) / 2 + p1], e1.info ^ e2.info ^ shb,
                                      ((D0 + e2.G) + e1.G) + xj, p1, p2);
                        }
                    }
                }
            } else {
                // single excitations: one row, lanes over the particle
                if (lane == 0) cnt += (uint32_t)nr;
                for (int c0 = 0; c0 < nr; c0 += WAVE) {
                    const int l = c0 + lane;
                    const bool lok = l < nr;
                    if (BWD || lok) {
                        const PEnt e1 = sRT[lok ? l : nr - 1];
                        const int pa = e1.info & 255;
                        const double Hv = flip(fock_offdiag<NINT>(a.I, Ib, s1, h1, pa), e1.info);
                        double D = D0 + e1.G;
                        double A[NS];
#pragma unroll
                        for (int k = 0; k < NS; ++k) A[k] = cI[k] * Hv;
                        bool live = true;
                        if (BWD && !lok) {
                            live = false; D = DEAD_D;
#pragma unroll
                            for (int k = 0; k < NS; ++k) A[k] = 0.0;
                        }
                        const bool flag = nrs > 0 || (e1.info & FR) != 0u;
                        if (live && flag) {
                            uint32_t nco = 0;
                            if (gather(l, 0, A, nco)) {
                                live = false; D = DEAD_D; nban++;
#pragma unroll
                                for (int k = 0; k < NS; ++k) A[k] = 0.0;
                            } else {
                                conn += nco;
                            }
                        }
                        double ek[NS], w[NS], vsum;
                        const double tsel = finish(A, D, ek, w, vsum);
                        if (FP && live) fpsum += fold(pa, -1);
                        {
                            const bool c = live && fabs(tsel) >= tau_val;
                            if (__builtin_amdgcn_ballot_w64(c)) select(c, ek, pa, -1);
                        }
                        if (BWD) {
                            double gs = 0.0;
#pragma unroll
                            for (int k = 0; k < NS; ++k) {
                                dcI[k] = fma(w[k], Hv, dcI[k]);
                                gs += w[k] * cI[k];
                            }
                            vbatch += vsum;
                            if (live) {
                                atomicAdd(&sDHD[pa], vsum);
                                if (a.dh && gs != 0.0) {
                                    const double gg = 0.5 * ((e1.info & SGN) ? -gs : gs);
                                    atomicAdd(&a.dh[(int64_t)h1 * n + pa], gg);
                                    atomicAdd(&a.dh[(int64_t)pa * n + h1], gg);
                                }
                                if (flag) gather_bwd(l, 0, w);
                            }
                        }
                    }
                }
            }
            cnt -= nban;

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
        // per-lane counts may wrap (banned cells are subtracted lane by lane);
        // their sum modulo 2^32 is the item's count
        uint32_t cc = cnt;
        uint64_t ff = fpsum, cn = conn;
        for (int o = 32; o > 0; o >>= 1) {
            cc += __shfl_xor(cc, o);
            ff += __shfl_xor(ff, o);
            cn += __shfl_xor(cn, o);
            mind = fmin(mind, __shfl_xor(mind, o));
        }
        // cells that did not count leave 1e300 behind
        if (mind >= 1e299) mind = __builtin_inf();
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

}  // namespace qpfast

template <int NINT, int NS, bool BWD>
void launch_fast(const SweepArgs *sys, const int64_t *item_end, int n_sys, bool fp, size_t lds, int grid,
                 hipStream_t st)
{
    if (fp)
        hipLaunchKernelGGL((qpfast::fast_kernel<NINT, NS, BWD, true>), dim3(grid), dim3(qpfast::WAVE), lds, st, sys,
                           item_end, n_sys);
    else
        hipLaunchKernelGGL((qpfast::fast_kernel<NINT, NS, BWD, false>), dim3(grid), dim3(qpfast::WAVE), lds, st, sys,
                           item_end, n_sys);
}

template <int NINT, int NS, bool BWD>
int fast_occupancy(size_t lds, bool fp)
{
    int blocks = 0;
    const hipError_t e = fp ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                  &blocks, qpfast::fast_kernel<NINT, NS, BWD, true>, qpfast::WAVE, lds)
                            : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                                  &blocks, qpfast::fast_kernel<NINT, NS, BWD, false>, qpfast::WAVE, lds);
    if (e != hipSuccess) return 8;
    return blocks > 0 ? blocks : 1;
}

#define QPF_INST(NI, NS, B)                                                                                  \
    template void launch_fast<NI, NS, B>(const SweepArgs *, const int64_t *, int, bool, size_t, int, hipStream_t); \
    template int fast_occupancy<NI, NS, B>(size_t, bool);
