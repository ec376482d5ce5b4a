/*
 * qp_oracle.c -- plain, slow FP64 reference for the Epstein-Nesbet PT2 and
 * CIPSI-selection sweep of Quantum Package 2.0 (arXiv:1902.08154).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes
 * or calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header, table or helper with the
 * HIP path.
 *
 * What it computes is the plain definition, written out:
 *   - Slater-Condon matrix elements between canonical determinants
 *     (sec. "Matrix elements of the Hamiltonian", the three rules for H_II,
 *     H_{I,I_p^r} and H_{I,I_pq^rs}); the phase is obtained by applying the
 *     creation/annihilation operators one at a time to the canonically ordered
 *     determinant (sec. "Internal representation of determinants": up
 *     spin-orbitals before down, increasing index within each spin);
 *   - the external set A = { alpha not in Psi, connected to Psi } where
 *     "connected" is read structurally: 1 <= excitation degree <= 2 from some
 *     J in Psi (sec. "CIPSI selection and PT2 energy", step 2);
 *   - e_alpha = <Psi|H|alpha>^2 / (E0 - H_alpha,alpha) and E_PT2 = sum e_alpha
 *     (eqs. e2 and PT2);
 *   - the generator partition E_PT2 = sum_I eps_I with A_I the alpha connected
 *     to I and to no earlier K (hybrid deterministic/stochastic PT2
 *     subsection); generators ordered by decreasing c_I^2 (sum over states),
 *     ties broken by ascending bit string;
 *   - the multi-state selection criterion sum_k e_{alpha k} / max_I c_{Ik}^2
 *     (Angeli-type criterion in the same subsection), ranked by absolute value,
 *     ties by ascending bit string;
 *   - gradients of E_PT2 with respect to c, E0 and the one-electron integrals
 *     (partial derivatives, A fixed, E0 independent).
 *
 * Two-electron integrals are read from the packed array through the paper's
 * Algorithm 1 ("HASH"), evaluated with 1-based orbital indices and shifted to
 * a 0-based offset.  Algorithm 1 pairs its 1st with its 3rd and its 2nd with
 * its 4th argument (physicist order), so the chemist integral (pq|rs) is
 * HASH(p, r, q, s).
 *
 * Summations over alpha use Neumaier compensation in ascending bit-string
 * order, so results do not depend on hash-table layout.
 *
 * Build:  gcc -O2 -fPIC -shared -fopenmp -ffp-contract=off
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

typedef uint64_t u64;

enum { ORC_MAX_STATES = 8 };

/* ------------------------------------------------------------------------ */
/* integrals                                                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n;             /* spatial orbitals */
    int nint;          /* 64-bit words per spin string */
    const double *h;   /* [n][n] */
    const double *eri; /* packed, Algorithm 1 order */
} orc_ints;

/* Algorithm 1: the integral "hash" of a quartet, 1-based indices. */
static u64 alg1_hash(u64 i, u64 j, u64 k, u64 l)
{
    u64 p = i < k ? i : k, r = i < k ? k : i;
    u64 t = p + r * (r - 1) / 2;
    u64 q = j < l ? j : l, s = j < l ? l : j;
    u64 u = q + s * (s - 1) / 2;
    u64 v = t < u ? t : u, w = t < u ? u : t;
    return v + w * (w - 1) / 2;
}

/* chemist (pq|rs), 0-based orbitals */
static double eri(const orc_ints *I, int p, int q, int r, int s)
{
    return I->eri[alg1_hash((u64)p + 1, (u64)r + 1, (u64)q + 1, (u64)s + 1) - 1];
}

static double hcore(const orc_ints *I, int p, int q) { return I->h[(size_t)p * I->n + q]; }

/* ------------------------------------------------------------------------ */
/* determinants: u64 d[2*nint]; word s*nint + w holds orbitals 64w..64w+63    */
/* of spin s (0 = up, 1 = down).  Spin-orbital index so = s*n + p.            */
/* ------------------------------------------------------------------------ */

static int occupied(const u64 *d, int nint, int s, int p)
{
    return (int)((d[s * nint + p / 64] >> (p % 64)) & 1u);
}

static void flip(u64 *d, int nint, int s, int p) { d[s * nint + p / 64] ^= (u64)1 << (p % 64); }

/* number of occupied spin-orbitals strictly before (s,p) in canonical order */
static int count_before(const u64 *d, int nint, int n, int s, int p)
{
    int c = 0;
    for (int ss = 0; ss <= s; ++ss) {
        int lim = (ss < s) ? n : p;
        for (int q = 0; q < lim; ++q) c += occupied(d, nint, ss, q);
    }
    return c;
}

/* Apply a (create=0) or a^dagger (create=1) on spin-orbital (s,p) in place.
 * Returns the sign (+1/-1) or 0 if the result vanishes. */
static int apply_op(u64 *d, int nint, int n, int create, int s, int p)
{
    int occ = occupied(d, nint, s, p);
    if (create == occ) return 0;
    int sign = (count_before(d, nint, n, s, p) & 1) ? -1 : 1;
    flip(d, nint, s, p);
    return sign;
}

static int popcount64(u64 x) { return __builtin_popcountll(x); }

/* key order: up words from high to low, then down words from high to low */
static int det_cmp(const u64 *a, const u64 *b, int nint)
{
    for (int s = 0; s < 2; ++s)
        for (int w = nint - 1; w >= 0; --w) {
            u64 x = a[s * nint + w], y = b[s * nint + w];
            if (x != y) return x < y ? -1 : 1;
        }
    return 0;
}

static int excitation_degree(const u64 *a, const u64 *b, int nint)
{
    int c = 0;
    for (int i = 0; i < 2 * nint; ++i) c += popcount64(a[i] ^ b[i]);
    return c / 2;
}

/* list the spin-orbitals (s*n+p) in x that are absent from y, canonical order */
static int set_minus(const u64 *x, const u64 *y, int nint, int n, int *out, int cap)
{
    int m = 0;
    for (int s = 0; s < 2; ++s)
        for (int p = 0; p < n; ++p)
            if (occupied(x, nint, s, p) && !occupied(y, nint, s, p)) {
                if (m < cap) out[m] = s * n + p;
                ++m;
            }
    return m;
}

/* Neumaier-compensated sum (the denominators E0 - H_aa of eq. e2 can be
 * small, so the diagonal is accumulated to within a few ulps) */
typedef struct { double s, c; } neumaier;
static void nm_add(neumaier *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double nm_val(const neumaier *a) { return a->s + a->c; }

/* Diagonal rule: sum_i h_ii + 1/2 sum_{i != j} [(ii|jj) - delta_spin (ij|ji)] */
double orc_diagonal(const orc_ints *I, const u64 *d)
{
    int n = I->n, nint = I->nint;
    neumaier acc = {0.0, 0.0};
    for (int si = 0; si < 2; ++si)
        for (int i = 0; i < n; ++i) {
            if (!occupied(d, nint, si, i)) continue;
            nm_add(&acc, hcore(I, i, i));
            for (int sj = 0; sj < 2; ++sj)
                for (int j = 0; j < n; ++j) {
                    if (!occupied(d, nint, sj, j)) continue;
                    if (si == sj && i == j) continue;
                    nm_add(&acc, 0.5 * eri(I, i, i, j, j));
                    if (si == sj) nm_add(&acc, -0.5 * eri(I, i, j, j, i));
                }
        }
    return nm_val(&acc);
}

/* Off-diagonal Slater-Condon element <bra|H|ket>, bra != ket.  Also returns
 * (through *single_hp, when non-NULL) the hole/particle spin-orbitals of a
 * single excitation and its operator sign, for the one-electron gradient. */
static double offdiag_element(const orc_ints *I, const u64 *bra, const u64 *ket,
                              int *deg_out, int *single_info)
{
    int n = I->n, nint = I->nint;
    int deg = excitation_degree(bra, ket, nint);
    if (deg_out) *deg_out = deg;
    if (deg == 0 || deg > 2) return 0.0;
    int holes[2], parts[2];
    set_minus(ket, bra, nint, n, holes, 2);  /* in ket, not in bra: annihilated */
    set_minus(bra, ket, nint, n, parts, 2);  /* in bra, not in ket: created */
    u64 work[2 * 8];
    memcpy(work, ket, sizeof(u64) * 2 * nint);
    if (deg == 1) {
        int sh = holes[0] / n, h = holes[0] % n, sp = parts[0] / n, p = parts[0] % n;
        if (sh != sp) return 0.0;
        int sign = apply_op(work, nint, n, 0, sh, h);
        sign *= apply_op(work, nint, n, 1, sp, p);
        /* <bra| a+_p a_h |ket> = sign ; element h_ph + sum_{i in ket} (ph|ii) - d (pi|ih) */
        double v = hcore(I, p, h);
        for (int si = 0; si < 2; ++si)
            for (int i = 0; i < n; ++i) {
                if (!occupied(ket, nint, si, i)) continue;
                v += eri(I, p, h, i, i);
                if (si == sh) v -= eri(I, p, i, i, h);
            }
        if (single_info) { single_info[0] = holes[0]; single_info[1] = parts[0]; single_info[2] = sign; }
        return sign * v;
    }
    /* deg == 2: sign of <bra| a+_p1 a+_p2 a_h2 a_h1 |ket>, h1<h2, p1<p2 canonical */
    int h1 = holes[0], h2 = holes[1], p1 = parts[0], p2 = parts[1];
    int sign = apply_op(work, nint, n, 0, h1 / n, h1 % n);
    sign *= apply_op(work, nint, n, 0, h2 / n, h2 % n);
    sign *= apply_op(work, nint, n, 1, p2 / n, p2 % n);
    sign *= apply_op(work, nint, n, 1, p1 / n, p1 % n);
    double v = 0.0;
    if (p1 / n == h1 / n && p2 / n == h2 / n)
        v += eri(I, p1 % n, h1 % n, p2 % n, h2 % n);
    if (p1 / n == h2 / n && p2 / n == h1 / n)
        v -= eri(I, p1 % n, h2 % n, p2 % n, h1 % n);
    return sign * v;
}

double orc_matrix_element(int n, int nint, const double *h, const double *eri_packed,
                          const u64 *bra, const u64 *ket)
{
    orc_ints I = {n, nint, h, eri_packed};
    if (excitation_degree(bra, ket, nint) == 0) return orc_diagonal(&I, bra);
    return offdiag_element(&I, bra, ket, NULL, NULL);
}

/* ------------------------------------------------------------------------ */
/* helpers: compensated sum, splitmix64 fingerprint, hash set of dets         */
/* ------------------------------------------------------------------------ */

/* splitmix64 output function (Steele, Lea & Flood 2014) */
static u64 mix64(u64 z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}
/* fingerprint of one determinant: fold mix64 over up words then down words */
u64 orc_det_fingerprint(const u64 *d, int nint)
{
    u64 hsh = 0;
    for (int i = 0; i < 2 * nint; ++i) hsh = mix64(hsh ^ d[i]);
    return hsh;
}

typedef struct {
    int nint;
    size_t cap;      /* power of two */
    size_t count;
    u64 *keys;       /* cap * 2*nint */
    int64_t *slot;   /* cap; -1 empty, else payload index */
} detmap;

static u64 det_hash(const u64 *d, int nint)
{
    u64 hsh = 0x12345678abcdefULL;
    for (int i = 0; i < 2 * nint; ++i) hsh = mix64(hsh + d[i] + 0x9e3779b97f4a7c15ULL);
    return hsh;
}

static int detmap_init(detmap *m, int nint, size_t expect)
{
    size_t cap = 64;
    while (cap < 2 * expect + 16) cap <<= 1;
    m->nint = nint; m->cap = cap; m->count = 0;
    m->keys = (u64 *)malloc(sizeof(u64) * 2 * nint * cap);
    m->slot = (int64_t *)malloc(sizeof(int64_t) * cap);
    if (!m->keys || !m->slot) return -1;
    for (size_t i = 0; i < cap; ++i) m->slot[i] = -1;
    return 0;
}
static void detmap_free(detmap *m) { free(m->keys); free(m->slot); }

static int64_t detmap_find(const detmap *m, const u64 *d)
{
    int w = 2 * m->nint;
    size_t i = det_hash(d, m->nint) & (m->cap - 1);
    while (m->slot[i] >= 0) {
        if (memcmp(m->keys + i * w, d, sizeof(u64) * w) == 0) return m->slot[i];
        i = (i + 1) & (m->cap - 1);
    }
    return -1;
}

static int detmap_grow(detmap *m);
/* insert with payload index; returns existing payload if present */
static int64_t detmap_insert(detmap *m, const u64 *d, int64_t payload, int *inserted)
{
    if (2 * (m->count + 1) > m->cap && detmap_grow(m) != 0) { *inserted = 0; return -2; }
    int w = 2 * m->nint;
    size_t i = det_hash(d, m->nint) & (m->cap - 1);
    while (m->slot[i] >= 0) {
        if (memcmp(m->keys + i * w, d, sizeof(u64) * w) == 0) { *inserted = 0; return m->slot[i]; }
        i = (i + 1) & (m->cap - 1);
    }
    memcpy(m->keys + i * w, d, sizeof(u64) * w);
    m->slot[i] = payload;
    m->count++;
    *inserted = 1;
    return payload;
}
static int detmap_grow(detmap *m)
{
    detmap n2;
    if (detmap_init(&n2, m->nint, m->cap) != 0) return -1;
    int w = 2 * m->nint, dummy;
    for (size_t i = 0; i < m->cap; ++i)
        if (m->slot[i] >= 0) detmap_insert(&n2, m->keys + i * w, m->slot[i], &dummy);
    detmap_free(m);
    *m = n2;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* excitation enumeration: every single and double of a determinant          */
/* ------------------------------------------------------------------------ */

/* Calls fn(ctx, alpha) for each distinct determinant that is a single or a
 * double excitation of d (same number of electrons per spin). */
typedef void (*exc_fn)(void *ctx, const u64 *alpha);

static void for_each_excitation(const u64 *d, int nint, int n, exc_fn fn, void *ctx)
{
    int occ[2][512], virt[2][512], no[2] = {0, 0}, nv[2] = {0, 0};
    for (int s = 0; s < 2; ++s)
        for (int p = 0; p < n; ++p) {
            if (occupied(d, nint, s, p)) occ[s][no[s]++] = p;
            else virt[s][nv[s]++] = p;
        }
    u64 a[16];
    /* singles */
    for (int s = 0; s < 2; ++s)
        for (int i = 0; i < no[s]; ++i)
            for (int x = 0; x < nv[s]; ++x) {
                memcpy(a, d, sizeof(u64) * 2 * nint);
                flip(a, nint, s, occ[s][i]);
                flip(a, nint, s, virt[s][x]);
                fn(ctx, a);
            }
    /* same-spin doubles */
    for (int s = 0; s < 2; ++s)
        for (int i = 0; i < no[s]; ++i)
            for (int j = i + 1; j < no[s]; ++j)
                for (int x = 0; x < nv[s]; ++x)
                    for (int y = x + 1; y < nv[s]; ++y) {
                        memcpy(a, d, sizeof(u64) * 2 * nint);
                        flip(a, nint, s, occ[s][i]); flip(a, nint, s, occ[s][j]);
                        flip(a, nint, s, virt[s][x]); flip(a, nint, s, virt[s][y]);
                        fn(ctx, a);
                    }
    /* opposite-spin doubles */
    for (int i = 0; i < no[0]; ++i)
        for (int x = 0; x < nv[0]; ++x)
            for (int j = 0; j < no[1]; ++j)
                for (int y = 0; y < nv[1]; ++y) {
                    memcpy(a, d, sizeof(u64) * 2 * nint);
                    flip(a, nint, 0, occ[0][i]); flip(a, nint, 0, virt[0][x]);
                    flip(a, nint, 1, occ[1][j]); flip(a, nint, 1, virt[1][y]);
                    fn(ctx, a);
                }
}

/* ------------------------------------------------------------------------ */
/* generator order: decreasing sum_k c_Ik^2, ties by ascending bit string     */
/* ------------------------------------------------------------------------ */

typedef struct { double w; const u64 *d; int nint; int64_t idx; } gen_key;
static int gen_cmp(const void *a, const void *b)
{
    const gen_key *x = (const gen_key *)a, *y = (const gen_key *)b;
    if (x->w != y->w) return x->w > y->w ? -1 : 1;
    return det_cmp(x->d, y->d, x->nint);
}

/* rank[J] = position of determinant J in the generator order */
int orc_generator_rank(const u64 *dets, const double *coefs, int64_t n_det, int n_states,
                       int nint, int64_t *rank)
{
    gen_key *k = (gen_key *)malloc(sizeof(gen_key) * (n_det ? n_det : 1));
    if (!k) return -1;
    for (int64_t j = 0; j < n_det; ++j) {
        double w = 0.0;
        for (int s = 0; s < n_states; ++s) w += coefs[(size_t)s * n_det + j] * coefs[(size_t)s * n_det + j];
        k[j].w = w; k[j].d = dets + (size_t)j * 2 * nint; k[j].nint = nint; k[j].idx = j;
    }
    qsort(k, n_det, sizeof(gen_key), gen_cmp);
    for (int64_t r = 0; r < n_det; ++r) rank[k[r].idx] = r;
    free(k);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* variational energy E0_k = <Psi_k|H|Psi_k> / <Psi_k|Psi_k>  (eq. evar)      */
/* ------------------------------------------------------------------------ */

int orc_energy(int n, int nint, const double *h, const double *eri_packed,
               const u64 *dets, const double *coefs, int64_t n_det, int n_states, double *E0)
{
    orc_ints I = {n, nint, h, eri_packed};
    double *row = (double *)malloc(sizeof(double) * (n_det ? n_det : 1) * n_states);
    if (!row) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t a = 0; a < n_det; ++a) {
        const u64 *da = dets + (size_t)a * 2 * nint;
        neumaier acc[ORC_MAX_STATES];
        memset(acc, 0, sizeof(acc));
        for (int64_t b = 0; b < n_det; ++b) {
            const u64 *db = dets + (size_t)b * 2 * nint;
            int deg = excitation_degree(da, db, nint);
            if (deg > 2) continue;
            double hab = deg == 0 ? orc_diagonal(&I, da) : offdiag_element(&I, da, db, NULL, NULL);
            for (int s = 0; s < n_states; ++s)
                nm_add(&acc[s], coefs[(size_t)s * n_det + a] * hab * coefs[(size_t)s * n_det + b]);
        }
        for (int s = 0; s < n_states; ++s) row[(size_t)s * n_det + a] = nm_val(&acc[s]);
    }
    for (int s = 0; s < n_states; ++s) {
        neumaier num = {0, 0}, den = {0, 0};
        for (int64_t a = 0; a < n_det; ++a) {
            nm_add(&num, row[(size_t)s * n_det + a]);
            double c = coefs[(size_t)s * n_det + a];
            nm_add(&den, c * c);
        }
        E0[s] = nm_val(&num) / nm_val(&den);
    }
    free(row);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* full definition: enumerate A, accumulate numerators, energies, partition,  */
/* selection and gradients                                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    const orc_ints *I;
    const u64 *dets;
    const double *coefs;
    int64_t n_det;
    int ns;
    const int64_t *rank;
    detmap *psi;
    detmap *amap;
    /* payload arrays indexed by alpha id */
    size_t acap, na;
    u64 *akeys;        /* na * 2nint */
    double *num;       /* na * ns */
    int64_t *owner;    /* na: min rank */
    int64_t *nconn;    /* na: connected internal dets */
    int nparts, part;
    /* current source determinant */
    int64_t j;
    int err;
    /* gradient pass */
    int grad_pass;
    const double *w;   /* na * ns : 2 g_k N/delta */
    double *dc;        /* ns * n_det */
    double *dh;        /* n * n */
} full_ctx;

static void full_visit(void *vctx, const u64 *a)
{
    full_ctx *C = (full_ctx *)vctx;
    int nint = C->I->nint;
    if (C->err) return;
    if (detmap_find(C->psi, a) >= 0) return;                     /* internal */
    if (C->nparts > 1 && (int)(orc_det_fingerprint(a, nint) % (u64)C->nparts) != C->part) return;
    const u64 *dj = C->dets + (size_t)C->j * 2 * nint;
    if (!C->grad_pass) {
        int ins;
        int64_t id = detmap_insert(C->amap, a, (int64_t)C->na, &ins);
        if (id == -2) { C->err = 1; return; }
        if (ins) {
            if (C->na == C->acap) {
                size_t nc = C->acap * 2 + 1024;
                u64 *k2 = (u64 *)realloc(C->akeys, sizeof(u64) * 2 * nint * nc);
                double *n2 = (double *)realloc(C->num, sizeof(double) * C->ns * nc);
                int64_t *o2 = (int64_t *)realloc(C->owner, sizeof(int64_t) * nc);
                int64_t *c2 = (int64_t *)realloc(C->nconn, sizeof(int64_t) * nc);
                if (!k2 || !n2 || !o2 || !c2) { C->err = 1; return; }
                C->akeys = k2; C->num = n2; C->owner = o2; C->nconn = c2; C->acap = nc;
            }
            memcpy(C->akeys + C->na * 2 * nint, a, sizeof(u64) * 2 * nint);
            for (int s = 0; s < C->ns; ++s) C->num[C->na * C->ns + s] = 0.0;
            C->owner[C->na] = INT64_MAX;
            C->nconn[C->na] = 0;
            C->na++;
        }
        double hja = offdiag_element(C->I, a, dj, NULL, NULL);
        for (int s = 0; s < C->ns; ++s)
            C->num[id * C->ns + s] += C->coefs[(size_t)s * C->n_det + C->j] * hja;
        if (C->rank[C->j] < C->owner[id]) C->owner[id] = C->rank[C->j];
        C->nconn[id]++;
    } else {
        int64_t id = detmap_find(C->amap, a);
        if (id < 0) return;
        int sinfo[3] = {-1, -1, 0};
        double hja = offdiag_element(C->I, a, dj, NULL, sinfo);
        int n = C->I->n;
        for (int s = 0; s < C->ns; ++s) {
            double w = C->w[id * C->ns + s];
            C->dc[(size_t)s * C->n_det + C->j] += w * hja;
            if (sinfo[0] >= 0 && C->dh) {
                /* d H_{alpha J} / d h_{pq} (symmetric variable) = sign for the
                 * single excitation hole x -> particle y; split over (x,y),(y,x) */
                int x = sinfo[0] % n, y = sinfo[1] % n;
                double g = 0.5 * w * C->coefs[(size_t)s * C->n_det + C->j] * sinfo[2];
                C->dh[(size_t)x * n + y] += g;
                C->dh[(size_t)y * n + x] += g;
            }
        }
    }
}

typedef struct { const u64 *keys; int nint; } sort_ctx_t;
static sort_ctx_t g_sort_ctx;
static int key_index_cmp(const void *a, const void *b)
{
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    return det_cmp(g_sort_ctx.keys + i * 2 * g_sort_ctx.nint, g_sort_ctx.keys + j * 2 * g_sort_ctx.nint,
                   g_sort_ctx.nint);
}

typedef struct { double key; int64_t id; } sel_item;
static const u64 *g_sel_keys; static int g_sel_nint;
static int sel_cmp(const void *a, const void *b)
{
    const sel_item *x = (const sel_item *)a, *y = (const sel_item *)b;
    if (x->key != y->key) return x->key > y->key ? -1 : 1;
    return det_cmp(g_sel_keys + x->id * 2 * g_sel_nint, g_sel_keys + y->id * 2 * g_sel_nint, g_sel_nint);
}

/*
 * orc_pt2_full: the whole definition for one partition of A.
 *
 * Inputs: h [n][n], packed ERIs, dets [n_det][2][nint], coefs [ns][n_det],
 * E0 [ns].  With nparts > 1 only alpha whose fingerprint % nparts == part are
 * considered (the union over parts is A; sums add up across parts).
 * Outputs (all optional except e_pt2):
 *   e_pt2[ns], S[ns] = sum N^2/delta^2, n_alpha, fp_sum (wrapping sum of
 *   per-alpha fingerprints), n_conn (sum over alpha of connected internal
 *   dets), min_abs_delta, eps_gen[ns][n_det] (caller's det index),
 *   selection: the first n_select alpha by (|e~| desc, key asc) ->
 *   sel_dets [n_select][2][nint], sel_e [n_select][ns], sel_key[n_select] (|e~|),
 *   sel_D [n_select] (H_alpha,alpha), *n_sel;
 *   conditioning sums for rounding-aware comparisons: abs_e[ns] = sum |e|,
 *   T[ns] = sum N^2/|delta|^3, and per generator S_gen, abs_gen [ns][n_det];
 *   all_dets/all_e/all_D/all_owner: every alpha in ascending key order when
 *   all_cap >= n_alpha (all_e [n][ns]; all_N [n][ns]);
 *   gradients when grad_up != NULL: dc [ns][n_det], dE0 [ns], dh [n][n].
 * Returns 0, or -1 on allocation failure.
 */
int orc_pt2_full(int n, int nint, const double *h, const double *eri_packed,
                 const u64 *dets, const double *coefs, int64_t n_det, int ns, const double *E0,
                 int nparts, int part,
                 double *e_pt2, double *S, int64_t *n_alpha, u64 *fp_sum, int64_t *n_conn,
                 double *min_abs_delta, double *eps_gen,
                 int64_t n_select, u64 *sel_dets, double *sel_e, double *sel_key, int64_t *n_sel,
                 int64_t all_cap, u64 *all_dets, double *all_e, double *all_N, double *all_D,
                 int64_t *all_owner,
                 const double *grad_up, double *dc, double *dE0, double *dh,
                 double *abs_e, double *T, double *S_gen, double *abs_gen, double *sel_D)
{
    if (ns < 1 || ns > ORC_MAX_STATES) return -1;
    orc_ints I = {n, nint, h, eri_packed};
    int64_t *rank = (int64_t *)malloc(sizeof(int64_t) * (n_det ? n_det : 1));
    int64_t *gen_of_rank = (int64_t *)malloc(sizeof(int64_t) * (n_det ? n_det : 1));
    if (!rank || !gen_of_rank) return -1;
    orc_generator_rank(dets, coefs, n_det, ns, nint, rank);
    for (int64_t j = 0; j < n_det; ++j) gen_of_rank[rank[j]] = j;

    detmap psi, amap;
    if (detmap_init(&psi, nint, (size_t)n_det) != 0) return -1;
    for (int64_t j = 0; j < n_det; ++j) {
        int ins;
        detmap_insert(&psi, dets + (size_t)j * 2 * nint, j, &ins);
    }
    if (detmap_init(&amap, nint, 1024) != 0) return -1;

    full_ctx C;
    memset(&C, 0, sizeof(C));
    C.I = &I; C.dets = dets; C.coefs = coefs; C.n_det = n_det; C.ns = ns; C.rank = rank;
    C.psi = &psi; C.amap = &amap; C.nparts = nparts; C.part = part;
    for (int64_t j = 0; j < n_det; ++j) {
        C.j = j;
        for_each_excitation(dets + (size_t)j * 2 * nint, nint, n, full_visit, &C);
        if (C.err) return -1;
    }
    size_t na = C.na;

    /* ascending key order for deterministic compensated sums */
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (na ? na : 1));
    double *D = (double *)malloc(sizeof(double) * (na ? na : 1));
    double *e = (double *)malloc(sizeof(double) * (na ? na : 1) * ns);
    if (!order || !D || !e) return -1;
    for (size_t i = 0; i < na; ++i) order[i] = (int64_t)i;
    g_sort_ctx.keys = C.akeys; g_sort_ctx.nint = nint;
    qsort(order, na, sizeof(int64_t), key_index_cmp);

    double maxc2[ORC_MAX_STATES];
    for (int s = 0; s < ns; ++s) {
        maxc2[s] = 0.0;
        for (int64_t j = 0; j < n_det; ++j) {
            double c = coefs[(size_t)s * n_det + j];
            if (c * c > maxc2[s]) maxc2[s] = c * c;
        }
    }

    neumaier accE[ORC_MAX_STATES], accS[ORC_MAX_STATES], accA[ORC_MAX_STATES], accT[ORC_MAX_STATES];
    memset(accE, 0, sizeof(accE)); memset(accS, 0, sizeof(accS));
    memset(accA, 0, sizeof(accA)); memset(accT, 0, sizeof(accT));
    neumaier *acc_gen = NULL, *accS_gen = NULL, *accA_gen = NULL;
    if (eps_gen || S_gen || abs_gen) {
        acc_gen = (neumaier *)calloc((size_t)ns * (n_det ? n_det : 1), sizeof(neumaier));
        accS_gen = (neumaier *)calloc((size_t)ns * (n_det ? n_det : 1), sizeof(neumaier));
        accA_gen = (neumaier *)calloc((size_t)ns * (n_det ? n_det : 1), sizeof(neumaier));
        if (!acc_gen || !accS_gen || !accA_gen) return -1;
    }
    u64 fps = 0;
    int64_t conn = 0;
    double mind = INFINITY;
    for (size_t oi = 0; oi < na; ++oi) {
        int64_t i = order[oi];
        const u64 *a = C.akeys + i * 2 * nint;
        D[i] = orc_diagonal(&I, a);
        int64_t owner_det = gen_of_rank[C.owner[i]];
        for (int s = 0; s < ns; ++s) {
            double N = C.num[i * ns + s];
            double delta = E0[s] - D[i];
            double ea = N * N / delta;
            e[i * ns + s] = ea;
            nm_add(&accE[s], ea);
            nm_add(&accS[s], N * N / (delta * delta));
            nm_add(&accA[s], fabs(ea));
            nm_add(&accT[s], N * N / fabs(delta * delta * delta));
            if (acc_gen) {
                nm_add(&acc_gen[(size_t)s * n_det + owner_det], ea);
                nm_add(&accS_gen[(size_t)s * n_det + owner_det], N * N / (delta * delta));
                nm_add(&accA_gen[(size_t)s * n_det + owner_det], fabs(ea));
            }
            if (fabs(delta) < mind) mind = fabs(delta);
        }
        fps += orc_det_fingerprint(a, nint);
        conn += C.nconn[i];
    }
    for (int s = 0; s < ns; ++s) {
        e_pt2[s] = nm_val(&accE[s]);
        if (S) S[s] = nm_val(&accS[s]);
        if (abs_e) abs_e[s] = nm_val(&accA[s]);
        if (T) T[s] = nm_val(&accT[s]);
    }
    for (int s = 0; s < ns && acc_gen; ++s)
        for (int64_t j = 0; j < n_det; ++j) {
            if (S_gen) S_gen[(size_t)s * n_det + j] = nm_val(&accS_gen[(size_t)s * n_det + j]);
            if (abs_gen) abs_gen[(size_t)s * n_det + j] = nm_val(&accA_gen[(size_t)s * n_det + j]);
        }
    if (n_alpha) *n_alpha = (int64_t)na;
    if (fp_sum) *fp_sum = fps;
    if (n_conn) *n_conn = conn;
    if (min_abs_delta) *min_abs_delta = mind;
    if (eps_gen)
        for (int s = 0; s < ns; ++s)
            for (int64_t j = 0; j < n_det; ++j)
                eps_gen[(size_t)s * n_det + j] = nm_val(&acc_gen[(size_t)s * n_det + j]);

    if (all_cap >= (int64_t)na) {
        for (size_t oi = 0; oi < na; ++oi) {
            int64_t i = order[oi];
            if (all_dets) memcpy(all_dets + oi * 2 * nint, C.akeys + i * 2 * nint, sizeof(u64) * 2 * nint);
            for (int s = 0; s < ns; ++s) {
                if (all_e) all_e[oi * ns + s] = e[i * ns + s];
                if (all_N) all_N[oi * ns + s] = C.num[i * ns + s];
            }
            if (all_D) all_D[oi] = D[i];
            if (all_owner) all_owner[oi] = gen_of_rank[C.owner[i]];
        }
    }

    if (n_select > 0 && n_sel) {
        sel_item *it = (sel_item *)malloc(sizeof(sel_item) * (na ? na : 1));
        if (!it) return -1;
        for (size_t i = 0; i < na; ++i) {
            double t = 0.0;
            for (int s = 0; s < ns; ++s) t += e[i * ns + s] / maxc2[s];
            it[i].key = fabs(t);
            it[i].id = (int64_t)i;
        }
        g_sel_keys = C.akeys; g_sel_nint = nint;
        qsort(it, na, sizeof(sel_item), sel_cmp);
        int64_t m = n_select < (int64_t)na ? n_select : (int64_t)na;
        for (int64_t r = 0; r < m; ++r) {
            int64_t i = it[r].id;
            if (sel_dets) memcpy(sel_dets + r * 2 * nint, C.akeys + i * 2 * nint, sizeof(u64) * 2 * nint);
            if (sel_e) for (int s = 0; s < ns; ++s) sel_e[r * ns + s] = e[i * ns + s];
            if (sel_key) sel_key[r] = it[r].key;
            if (sel_D) sel_D[r] = D[i];
        }
        *n_sel = m;
        free(it);
    }

    if (grad_up) {
        double *w = (double *)malloc(sizeof(double) * (na ? na : 1) * ns);
        if (!w) return -1;
        for (int s = 0; s < ns; ++s) {
            for (int64_t j = 0; j < n_det; ++j) dc[(size_t)s * n_det + j] = 0.0;
            dE0[s] = -grad_up[s] * nm_val(&accS[s]);
        }
        if (dh) for (int i = 0; i < n * n; ++i) dh[i] = 0.0;
        for (size_t i = 0; i < na; ++i)
            for (int s = 0; s < ns; ++s) {
                double delta = E0[s] - D[i];
                w[i * ns + s] = 2.0 * grad_up[s] * C.num[i * ns + s] / delta;
            }
        /* diagonal part of dE/dh: dD_alpha/dh_pp = spatial occupation n_p(alpha) */
        if (dh)
            for (size_t oi = 0; oi < na; ++oi) {
                int64_t i = order[oi];
                const u64 *a = C.akeys + i * 2 * nint;
                double v = 0.0;
                for (int s = 0; s < ns; ++s) {
                    double delta = E0[s] - D[i];
                    double N = C.num[i * ns + s];
                    v += grad_up[s] * N * N / (delta * delta);
                }
                for (int sp = 0; sp < 2; ++sp)
                    for (int p = 0; p < n; ++p)
                        if (occupied(a, nint, sp, p)) dh[(size_t)p * n + p] += v;
            }
        C.grad_pass = 1; C.w = w; C.dc = dc; C.dh = dh;
        for (int64_t j = 0; j < n_det; ++j) {
            C.j = j;
            for_each_excitation(dets + (size_t)j * 2 * nint, nint, n, full_visit, &C);
        }
        free(w);
    }

    free(order); free(D); free(e); free(acc_gen); free(accS_gen); free(accA_gen);
    free(C.akeys); free(C.num); free(C.owner); free(C.nconn);
    detmap_free(&psi); detmap_free(&amap);
    free(rank); free(gen_of_rank);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* per-alpha and per-generator evaluation (sampled checks at large sizes)     */
/* ------------------------------------------------------------------------ */

/* For one determinant alpha: numerators N_k = sum_J c_Jk <J|H|alpha> over all
 * of Psi, its diagonal, the minimum generator rank among connected J (or -1 if
 * none) and whether alpha itself is internal. */
int orc_alpha_eval(int n, int nint, const double *h, const double *eri_packed,
                   const u64 *dets, const double *coefs, int64_t n_det, int ns,
                   const int64_t *rank, const u64 *alpha,
                   double *N, double *D, int64_t *owner_rank, int *internal)
{
    orc_ints I = {n, nint, h, eri_packed};
    for (int s = 0; s < ns; ++s) N[s] = 0.0;
    *owner_rank = -1;
    *internal = 0;
    for (int64_t j = 0; j < n_det; ++j) {
        const u64 *dj = dets + (size_t)j * 2 * nint;
        int deg = excitation_degree(dj, alpha, nint);
        if (deg == 0) { *internal = 1; continue; }
        if (deg > 2) continue;
        double hja = offdiag_element(&I, alpha, dj, NULL, NULL);
        for (int s = 0; s < ns; ++s) N[s] += coefs[(size_t)s * n_det + j] * hja;
        if (*owner_rank < 0 || rank[j] < *owner_rank) *owner_rank = rank[j];
    }
    *D = orc_diagonal(&I, alpha);
    return 0;
}

typedef struct {
    const orc_ints *I;
    const u64 *dets;
    const double *coefs;
    int64_t n_det;
    int ns;
    const int64_t *rank;
    const detmap *psi;
    const int64_t *cand; int64_t ncand;   /* J with degree(J, I) <= 4 */
    int64_t gen;                          /* generator det index */
    const double *E0;
    const double *maxc2;
    neumaier acc[ORC_MAX_STATES], accS[ORC_MAX_STATES];
    int64_t count;
    u64 fp;
    /* optional dump of owned alpha with |e~| >= thr */
    double thr;
    int64_t dump_cap, ndump;
    u64 *dump_dets; double *dump_e; double *dump_key;
    /* a slice of the generator's excitations, in enumeration order: those
     * numbered [visit_start, visit_start + visit_cap) are evaluated (cap 0:
     * to the end).  Slices partition the generator's sums (a bounded timing
     * sample, or one generator split over threads). */
    int64_t visit_start, visit_cap, visits;
} gen_ctx;

static void gen_visit(void *vctx, const u64 *a)
{
    gen_ctx *G = (gen_ctx *)vctx;
    int nint = G->I->nint;
    const int64_t vi = G->visits++;
    if (vi < G->visit_start || (G->visit_cap > 0 && vi >= G->visit_start + G->visit_cap)) return;
    if (detmap_find(G->psi, a) >= 0) return;
    /* owner: lowest rank among connected J; only J within degree 4 of the
     * generator can be within degree 2 of alpha (triangle inequality) */
    int64_t best = INT64_MAX;
    double N[ORC_MAX_STATES] = {0};
    for (int64_t c = 0; c < G->ncand; ++c) {
        int64_t j = G->cand[c];
        const u64 *dj = G->dets + (size_t)j * 2 * nint;
        int deg = excitation_degree(dj, a, nint);
        if (deg == 0 || deg > 2) continue;
        if (G->rank[j] < best) best = G->rank[j];
        double hja = offdiag_element(G->I, a, dj, NULL, NULL);
        for (int s = 0; s < G->ns; ++s) N[s] += G->coefs[(size_t)s * G->n_det + j] * hja;
    }
    if (best != G->rank[G->gen]) return;
    double D = orc_diagonal(G->I, a);
    double t = 0.0, es[ORC_MAX_STATES];
    for (int s = 0; s < G->ns; ++s) {
        double delta = G->E0[s] - D;
        es[s] = N[s] * N[s] / delta;
        nm_add(&G->acc[s], es[s]);
        nm_add(&G->accS[s], N[s] * N[s] / (delta * delta));
        t += es[s] / G->maxc2[s];
    }
    G->count++;
    G->fp += orc_det_fingerprint(a, nint);
    if (G->dump_cap > 0 && fabs(t) >= G->thr) {
        if (G->ndump < G->dump_cap) {
            memcpy(G->dump_dets + G->ndump * 2 * nint, a, sizeof(u64) * 2 * nint);
            for (int s = 0; s < G->ns; ++s) G->dump_e[G->ndump * G->ns + s] = es[s];
            G->dump_key[G->ndump] = fabs(t);
        }
        G->ndump++;
    }
}

/*
 * orc_eps_generators: eps_I (per state) for the listed generators (caller's
 * det indices), plus per-generator |A_I|, fingerprint sum and S.  Optionally
 * dumps owned alpha with |e~| >= dump_thr (up to dump_cap per generator).
 * visit_start, visit_cap select a slice of each generator's excitations in
 * enumeration order: [visit_start, visit_start + visit_cap), cap 0 = to the
 * end (a bounded timing sample, or slices of one generator summed by the
 * caller).  nthreads > 0 sets the OpenMP
 * team's size (0: the runtime's default).
 * OpenMP over the listed generators; each generator is summed sequentially
 * (the enumeration order of for_each_excitation), so results are
 * deterministic.
 */
int orc_eps_generators(int n, int nint, const double *h, const double *eri_packed,
                       const u64 *dets, const double *coefs, int64_t n_det, int ns, const double *E0,
                       const int64_t *gens, int64_t n_gen,
                       double *eps, double *S, int64_t *count, u64 *fp,
                       double dump_thr, int64_t dump_cap, u64 *dump_dets, double *dump_e,
                       double *dump_key, int64_t *dump_n, int64_t visit_start, int64_t visit_cap,
                       int nthreads)
{
    if (ns < 1 || ns > ORC_MAX_STATES) return -1;
    orc_ints I = {n, nint, h, eri_packed};
    int64_t *rank = (int64_t *)malloc(sizeof(int64_t) * (n_det ? n_det : 1));
    if (!rank) return -1;
    orc_generator_rank(dets, coefs, n_det, ns, nint, rank);
    detmap psi;
    if (detmap_init(&psi, nint, (size_t)n_det) != 0) return -1;
    for (int64_t j = 0; j < n_det; ++j) {
        int ins;
        detmap_insert(&psi, dets + (size_t)j * 2 * nint, j, &ins);
    }
    double maxc2[ORC_MAX_STATES];
    for (int s = 0; s < ns; ++s) {
        maxc2[s] = 0.0;
        for (int64_t j = 0; j < n_det; ++j) {
            double c = coefs[(size_t)s * n_det + j];
            if (c * c > maxc2[s]) maxc2[s] = c * c;
        }
    }
    int fail = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : omp_get_max_threads())
    for (int64_t g = 0; g < n_gen; ++g) {
        int64_t gi = gens[g];
        const u64 *dg = dets + (size_t)gi * 2 * nint;
        int64_t *cand = (int64_t *)malloc(sizeof(int64_t) * (n_det ? n_det : 1));
        if (!cand) { fail = 1; continue; }
        int64_t nc = 0;
        for (int64_t j = 0; j < n_det; ++j)
            if (excitation_degree(dets + (size_t)j * 2 * nint, dg, nint) <= 4) cand[nc++] = j;
        gen_ctx G;
        memset(&G, 0, sizeof(G));
        G.I = &I; G.dets = dets; G.coefs = coefs; G.n_det = n_det; G.ns = ns; G.rank = rank;
        G.psi = &psi; G.cand = cand; G.ncand = nc; G.gen = gi; G.E0 = E0; G.maxc2 = maxc2;
        G.thr = dump_thr; G.dump_cap = dump_cap;
        G.visit_start = visit_start;
        G.visit_cap = visit_cap;
        if (dump_cap > 0) {
            G.dump_dets = dump_dets + (size_t)g * dump_cap * 2 * nint;
            G.dump_e = dump_e + (size_t)g * dump_cap * ns;
            G.dump_key = dump_key + (size_t)g * dump_cap;
        }
        for_each_excitation(dg, nint, n, gen_visit, &G);
        for (int s = 0; s < ns; ++s) {
            eps[(size_t)g * ns + s] = nm_val(&G.acc[s]);
            if (S) S[(size_t)g * ns + s] = nm_val(&G.accS[s]);
        }
        if (count) count[g] = G.count;
        if (fp) fp[g] = G.fp;
        if (dump_n) dump_n[g] = G.ndump;
        free(cand);
    }
    detmap_free(&psi);
    free(rank);
    return fail ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Dense H and S^2 over a determinant list (sec. "Davidson diagonalization":  */
/* the matrices whose lowest eigenpairs the Davidson iterations find).        */
/* ------------------------------------------------------------------------ */

/* H_IJ for every pair, from the Slater-Condon elements above; out [n_det][n_det] */
int orc_hamiltonian(int n, int nint, const double *h, const double *eri_packed, const u64 *dets,
                    int64_t n_det, double *out)
{
    orc_ints I = {n, nint, h, eri_packed};
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t i = 0; i < n_det; ++i)
        for (int64_t j = 0; j < n_det; ++j) {
            const u64 *a = dets + (size_t)i * 2 * nint, *b = dets + (size_t)j * 2 * nint;
            const int deg = excitation_degree(a, b, nint);
            double v = 0.0;
            if (deg == 0) v = orc_diagonal(&I, a);
            else if (deg <= 2) v = offdiag_element(&I, a, b, NULL, NULL);
            out[(size_t)i * n_det + j] = v;
        }
    return 0;
}

/* S^2 = S_- S_+ + S_z (S_z + 1), S_+ = sum_p a+(p,up) a(p,down),
 * S_- = sum_q a+(q,down) a(q,up), applied to each determinant by operator
 * application; out [n_det][n_det], <I|S^2|J> */
int orc_s2_matrix(int n, int nint, const u64 *dets, int64_t n_det, double *out)
{
    for (size_t x = 0; x < (size_t)n_det * n_det; ++x) out[x] = 0.0;
    u64 d[2 * 4], e[2 * 4];
    for (int64_t j = 0; j < n_det; ++j) {
        const u64 *ket = dets + (size_t)j * 2 * nint;
        int nup = 0, ndn = 0;
        for (int w = 0; w < nint; ++w) { nup += popcount64(ket[w]); ndn += popcount64(ket[nint + w]); }
        const double sz = 0.5 * (nup - ndn);
        out[(size_t)j * n_det + j] += sz * (sz + 1.0);
        for (int p = 0; p < n; ++p)
            for (int q = 0; q < n; ++q) {
                for (int w = 0; w < 2 * nint; ++w) d[w] = ket[w];
                int sg = apply_op(d, nint, n, 0, 1, p);          /* a(p, down)  */
                if (sg) sg *= apply_op(d, nint, n, 1, 0, p);     /* a+(p, up)   */
                if (sg) sg *= apply_op(d, nint, n, 0, 0, q);     /* a(q, up)    */
                if (sg) sg *= apply_op(d, nint, n, 1, 1, q);     /* a+(q, down) */
                if (!sg) continue;
                for (int64_t i = 0; i < n_det; ++i) {
                    const u64 *bra = dets + (size_t)i * 2 * nint;
                    int same = 1;
                    for (int w = 0; w < 2 * nint; ++w) if (bra[w] != d[w]) { same = 0; break; }
                    if (same) { out[(size_t)i * n_det + j] += sg; break; }
                }
                (void)e;
            }
    }
    return 0;
}
