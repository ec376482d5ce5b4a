/*
 * qp_pt2.h -- C ABI of the MI355X (gfx950) Epstein-Nesbet PT2 / CIPSI-selection
 * sweep of Quantum Package 2.0 (arXiv:1902.08154).
 *
 * For every external determinant alpha that is a single or double excitation
 * of the wave function Psi (and not in Psi), the sweep forms
 *     N_alpha,k = <Psi_k|H|alpha> = sum_J c_Jk <J|H|alpha>     (Slater-Condon)
 *     e_alpha,k = N_alpha,k^2 / (E0_k - <alpha|H|alpha>)        (eq. e2)
 *     E_PT2,k   = sum_alpha e_alpha,k                           (eq. PT2)
 * and keeps the alpha with the largest |sum_k e_alpha,k / max_J c_Jk^2|
 * (multi-state selection criterion of sec. "CIPSI selection and PT2 energy").
 * Each alpha is produced by exactly one generator: generators are the
 * determinants of Psi sorted by decreasing sum_k c_Jk^2 (ties: ascending bit
 * string), and alpha belongs to the first generator it is connected to
 * (generator decomposition E_PT2 = sum_I eps_I of the same section).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array arguments are DEVICE pointers on the context's device unless
 *    stated otherwise; they are owned by the caller.  Every call only enqueues
 *    work on `stream` (a hipStream_t; NULL = default stream), except where a
 *    host synchronisation is documented.  Outputs are valid once the stream
 *    has synchronised.
 *  - Orbitals are spatial, 0-based, n_orb in [1, 256].  A determinant is
 *    uint64_t[2][n_int], n_int = (n_orb-1)/64 + 1: the spin-up string (words
 *    0..n_int-1) then the spin-down string; bit b of word w is orbital
 *    64*w + b.  Bits at positions >= n_orb must be zero.  Every determinant of
 *    one call has the same number of up and of down electrons.  The sign
 *    convention is the paper's: up spin-orbitals before down ones, increasing
 *    index within each spin (sec. "Internal representation of determinants");
 *    any other phase is folded into the coefficients.
 *  - Bit-string order ("key"): up words from high to low, then down words from
 *    high to low, compared as unsigned integers.
 *  - h is the real symmetric one-electron matrix, row-major [n_orb][n_orb].
 *    Two-electron integrals are chemist-notation (pq|rs), real, 8-fold
 *    symmetric, packed at offset tri(tri(p,q), tri(r,s)) with
 *    tri(a,b) = M(M+1)/2 + m, M = max(a,b), m = min(a,b): the paper's
 *    Algorithm 1 evaluated on 1-based indices, minus one.  Length
 *    P(P+1)/2 with P = n_orb(n_orb+1)/2.
 *  - Coefficients are [n_states][n_det] row-major FP64; n_states in [1, 4].
 *    The library does not normalise them.
 *  - All arithmetic on energies is IEEE FP64.  A zero denominator
 *    E0 - H_alpha,alpha is not an error: IEEE results propagate and
 *    stats.min_abs_delta reports the smallest |denominator|.
 *  - Return value: QP_OK (0) or a negative QP_E_* code; qp_last_error() then
 *    holds a message.  A failed call leaves outputs unspecified.
 */
#ifndef QP_PT2_H
#define QP_PT2_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QP_OK            0
#define QP_E_ARG        -1  /* null pointer, negative size, bad flag            */
#define QP_E_NORB       -2  /* n_orb outside [1,256] or a bit set at >= n_orb   */
#define QP_E_ELEC       -3  /* per-spin electron counts differ between dets     */
#define QP_E_DUP        -4  /* the same determinant appears twice               */
#define QP_E_NOINT      -5  /* integrals not set, or n_orb mismatch             */
#define QP_E_OOM        -6  /* device allocation failed                         */
#define QP_E_HIP        -7  /* a HIP runtime call failed                        */
#define QP_E_STATES     -8  /* n_states outside [1,4]                           */
#define QP_E_OVERFLOW   -9  /* selection candidate buffer overflowed            */
#define QP_E_NOCONV    -10  /* Davidson: residual above tolerance at the limit  */

#define QP_MAX_STATES    4
#define QP_MAX_ORB       256
#define QP_MAX_SYSTEMS   4096
#define QP_NOALLOC_MAX_DET (1 << 18)   /* largest n_det of qp_generator_order_noalloc */
#define QP_SPLIT_NEVER   0
#define QP_SPLIT_AUTO    1
#define QP_SPLIT_ALWAYS  2
#define QP_SPLIT_MIN_VIRT 100              /* qp_set_split's automatic threshold */

/* qp_pt2 flags */
#define QP_FLAG_FINGERPRINT  1  /* also compute stats.fingerprint of the alpha set */
#define QP_FLAG_NOCHECK      2  /* skip input validation (duplicates, counts, bits,
                                   generator indices: an index outside [0, n_det)
                                   is then swept as generator rank 0)            */
#define QP_SIGMA_S2          8  /* qp_sigma: W = S^2 U instead of H U              */
#define QP_SIGMA_REUSE      16  /* qp_sigma: the determinants are those of the
                                   previous qp_sigma call on this context (same
                                   dets pointer and n_det, contents unchanged, no
                                   qp_set_integrals since, same stream): its
                                   generator order and coarse lists are reused;
                                   otherwise they are prepared again            */
#define QP_FLAG_REUSE_INTEGRALS 4 /* qp_pt2_batched: keep a system's integral layouts
                                     from the previous batched call when its h and
                                     eri_packed pointers and n_orb are the same, and
                                     the caller has not changed their contents      */

typedef struct qp_ctx qp_ctx;

/* Device-side statistics of one sweep (written by qp_pt2 / qp_pt2_backward). */
typedef struct {
    uint64_t n_alpha;        /* |A|: external determinants (each counted once)     */
    uint64_t n_cells;        /* (generator, alpha) candidate cells examined          */
    uint64_t fingerprint;    /* sum mod 2^64 over alpha of fold(alpha), see below  */
    uint64_t n_coarse;       /* total coarse-filter entries: pairs (I,J), J != I,
                                with excitation degree <= 4                        */
    uint64_t n_candidates;   /* selection candidates written before the final sort */
    uint64_t overflow;       /* nonzero: candidate buffer overflowed (QP_E_OVERFLOW)*/
    uint64_t n_connections;  /* (alpha, J != generator) pairs with degree <= 2
                                that contributed a matrix element                  */
    uint64_t n_alpha_general; /* of n_alpha, those evaluated by the general kernel
                                (batches the dense kernel hands over)             */
    double   S[QP_MAX_STATES];  /* sum_alpha N^2/(E0-H_aa)^2 = -dE_PT2/dE0 (rPT2) */
    double   min_abs_delta;     /* min over alpha, k of |E0_k - H_alpha,alpha|      */
    /* renormalised PT2 (sec. "Renormalized PT2", eq. Z): the self-energy
     * linearised about E0 has slope -S_k, so Z_k = 1/(1 + S_k) and the
     * renormalised energy is E0_k + Z_k E_PT2,k                             */
    double   Z[QP_MAX_STATES];
    double   e_rpt2[QP_MAX_STATES];
    /* fine filter (sec. "Fast filtering of determinants"): over every hole
     * batch evaluated, the coarse entries J of its generator that lack at
     * most two of the generator's electrons outside the batch's holes (the J
     * that can reach one of its cells)                                      */
    uint64_t n_fine;
    uint64_t n_alpha_clean;  /* of n_alpha, the cells no determinant but the
                                generator touches (split sweeps)              */
} qp_pt2_stats;
/* fold(alpha): h = 0; for each word x of alpha (up words 0..n_int-1, then down
 * words 0..n_int-1): h = splitmix64_mix(h ^ x), where splitmix64_mix is the
 * output function of SplitMix64 (Steele, Lea & Flood, 2014):
 *   z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9; z = (z ^ (z >> 27)) * 0x94d049bb133111eb;
 *   return z ^ (z >> 31). */

/* Create a context bound to HIP device `device`.  Allocates nothing on the
 * device until the first call that needs it.  *ctx is owned by the caller and
 * released with qp_destroy. */
int  qp_create(qp_ctx **ctx, int device);
void qp_destroy(qp_ctx *ctx);
/* Message of the last failed call on ctx (never NULL; "" if none). */
const char *qp_last_error(const qp_ctx *ctx);

/*
 * qp_set_integrals -- one-electron matrix and two-electron integrals
 * (sec. "Matrix elements of the Hamiltonian"; storage: sec. "Storage of the
 * two-electron integrals", Algorithm 1).
 *   h          device [n_orb][n_orb], symmetric.
 *   eri_packed device, length P(P+1)/2, layout above.
 * The context builds its own device layouts from these and does not keep the
 * caller's pointers: a dense block per hole pair, n(n+1)/2 opposite-spin
 * blocks of n^2 and (n(n-1)/2)^2 same-spin entries, plus 2 n^3 + 4 n^2 tables
 * (doubles): at n_orb = 256 about 26 GB, six times the packed array.
 * Host synchronisation: the call synchronises `stream` twice, before it
 * releases the previous layouts and after it has built the new ones; the
 * caller may free h and eri_packed when it returns.
 * Replaces any previous integrals.  Errors: QP_E_ARG, QP_E_NORB, QP_E_OOM,
 * QP_E_HIP.
 */
int qp_set_integrals(qp_ctx *ctx, const double *h, const double *eri_packed, int n_orb,
                     void *stream);

/*
 * qp_pt2 -- the forward sweep: E_PT2 per state, the selected alpha, optional
 * per-generator partition (eqs. e2, PT2; generator decomposition and
 * selection of sec. "CIPSI selection and PT2 energy").
 *   dets      device uint64 [n_det][2][n_int]    (distinct determinants)
 *   coefs     device double [n_states][n_det]
 *   E0        device double [n_states]            (independent input)
 *   n_select  >= 0: number of alpha to keep (fewer if |A| < n_select)
 *   flags     QP_FLAG_*
 * Outputs (device):
 *   e_pt2     double [n_states]                   (required)
 *   sel_dets  uint64 [n_select][2][n_int]         (required if n_select > 0)
 *   sel_e     double [n_select][n_states]: e_alpha,k of each selected alpha,
 *             ordered by |sum_k e_k/max_J c_Jk^2| descending, ties by key
 *             ascending                            (required if n_select > 0)
 *   n_sel     int64 [1]                           (required if n_select > 0)
 *   stats     qp_pt2_stats [1]                    (optional, NULL)
 *   eps_gen   double [n_states][n_det]: eps_I of determinant I (caller's index)
 *                                                 (optional, NULL)
 * Host synchronisation: the call synchronises `stream` up to three times:
 * after the preparation (coarse-filter list sizes and input checks), after
 * the dense kernel when it handed batches over (their count), and before
 * the selection sort when n_select > 0.  A call that needs more pinned
 * host staging than earlier calls first waits for the device.
 * Errors: QP_E_ARG, QP_E_STATES, QP_E_NOINT, QP_E_NORB, QP_E_ELEC, QP_E_DUP,
 * QP_E_OOM, QP_E_HIP, QP_E_OVERFLOW.
 */
int qp_pt2(qp_ctx *ctx, const uint64_t *dets, const double *coefs, int64_t n_det,
           int n_states, const double *E0, int64_t n_select, int flags,
           double *e_pt2, uint64_t *sel_dets, double *sel_e, int64_t *n_sel,
           qp_pt2_stats *stats, double *eps_gen, void *stream);

/*
 * qp_pt2_backward -- adjoint of qp_pt2's E_PT2 output.  Recomputes every
 * numerator N_alpha,k (nothing is stored by the forward call) and returns the
 * partial derivatives of L = sum_k g_k E_PT2,k with A and E0 held as
 * independent inputs:
 *   grad_coefs[k][J] = 2 g_k sum_alpha (N_alpha,k / delta_alpha,k) <J|H|alpha>
 *   grad_E0[k]       = -g_k sum_alpha N_alpha,k^2 / delta_alpha,k^2
 *   grad_h[p][q]     symmetric G with dL = sum_pq G_pq dh_pq for symmetric dh:
 *                    diagonal terms from d<alpha|H|alpha>/dh_pp (occupation of
 *                    p in alpha), off-diagonal terms from the single-excitation
 *                    elements (d<J|H|alpha>/dh_xy = phase).
 *   grad_e_pt2 device double [n_states] (g_k); outputs device, overwritten:
 *   grad_coefs [n_states][n_det], grad_E0 [n_states], grad_h [n_orb][n_orb]
 *   (any output may be NULL to skip it).  stats as in qp_pt2 (optional).
 * Gradient accumulation uses FP64 atomics: results agree between runs to
 * rounding, not bitwise.  Errors as qp_pt2.
 */
int qp_pt2_backward(qp_ctx *ctx, const uint64_t *dets, const double *coefs, int64_t n_det,
                    int n_states, const double *E0, const double *grad_e_pt2, int flags,
                    double *grad_coefs, double *grad_E0, double *grad_h,
                    qp_pt2_stats *stats, void *stream);

/*
 * qp_generator_order -- the generator order used by every sweep (sec. "CIPSI
 * selection and PT2 energy"): determinant indices sorted by decreasing
 * sum_k c_Ik^2, ties by key ascending.  order_out device int32 [n_det].
 * Synchronises the stream once.  Errors as qp_pt2.
 */
int qp_generator_order(qp_ctx *ctx, const uint64_t *dets, const double *coefs, int64_t n_det,
                       int n_states, int flags, int32_t *order_out, void *stream);

/*
 * qp_generator_order_noalloc -- qp_generator_order for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments and the same order_out,
 * bit for bit, for n_det <= QP_NOALLOC_MAX_DET (2^18); larger n_det:
 * QP_E_ARG, nothing launched.  It calls no hipMalloc or hipFree and allocates
 * nothing else: its scratch (the weights sum_k c_Ik^2 and the index array of
 * the sort, 12 bytes per determinant up to the limit, 3 MiB in all) is a
 * file-scope device array that every GPU the library runs on holds until the
 * process ends, its address taken once per device when a context is
 * created.  Every call on a GPU shares that GPU's array: calls that overlap
 * on one GPU (other streams, other contexts, other threads) race and must be
 * serialised by the caller.  The inputs are not validated beyond pointers and
 * sizes (as under QP_FLAG_NOCHECK; flags is otherwise unused), and the stream
 * is not synchronised: order_out is complete when the stream's work is.
 * Errors: QP_E_ARG, QP_E_NOINT, QP_E_STATES, QP_E_HIP.
 */
int qp_generator_order_noalloc(qp_ctx *ctx, const uint64_t *dets, const double *coefs, int64_t n_det,
                               int n_states, int flags, int32_t *order_out, void *stream);

/*
 * qp_pt2_generators -- the generator decomposition E_PT2 = sum_I eps_I (same
 * section) evaluated for a list of generators only: eps_I,k of each listed
 * determinant I, with alpha owned by the first generator (in the generator
 * order of the whole wave function) it is connected to.
 *   gens     device int32 [n_gen]: distinct determinant indices
 *   eps_out  device double [n_states][n_gen] (position i: generator gens[i])
 *   n_select, sel_dets, sel_e, n_sel: as qp_pt2, over the alpha owned by the
 *            listed generators
 *   stats    optional; n_alpha, S, ... summed over the listed generators,
 *            n_cells counts their candidate cells
 * A listed generator's eps_I is the same, bit for bit, as qp_pt2's eps_gen
 * entry for it.  Errors as qp_pt2; QP_E_ARG for an index outside [0, n_det)
 * (not checked under QP_FLAG_NOCHECK).
 */
int qp_pt2_generators(qp_ctx *ctx, const uint64_t *dets, const double *coefs, int64_t n_det,
                      int n_states, const double *E0, const int32_t *gens, int64_t n_gen,
                      int64_t n_select, int flags, double *eps_out, uint64_t *sel_dets,
                      double *sel_e, int64_t *n_sel, qp_pt2_stats *stats, void *stream);

/*
 * qp_pt2_stochastic -- semi-stochastic E_PT2 (sec. "CIPSI selection and PT2
 * energy", the hybrid deterministic/stochastic scheme): E_PT2 = sum_{I in D}
 * eps_I + sum_{K in S} eps_K, with D the first d generators in generator order
 * (computed exactly) and the rest estimated from generators drawn with
 * probability w_K / W, w_K = sum_k c_Kk^2.  eps of a drawn generator is
 * computed once and reused when it is drawn again.  Rounds: D grows by
 * det_chunk generators and draws_per_round generators are drawn, then the
 * listed new generators are swept on the GPU together.  The estimate of
 * state k is sum_{D} eps + mean over the draws that fall outside D of
 * W_S eps_K / w_K (W_S the weight outside D), its error the standard error of
 * that mean.  Stops when every state has error <= rel_err |estimate| (the
 * paper's default is 0.002), when D holds every generator (exact, error 0),
 * or when the random numbers run out.  The generator order, per-generator
 * tables and coarse lists are prepared once per call; each round is one sweep
 * of its list followed by a host decision, and lasts at least one work item's
 * time, so rounds of a few hundred generators keep the device busy.
 * Selection on the fly (sec. "CIPSI selection and PT2 energy", the new
 * stochastic selection): with n_select > 0 every round also selects among the
 * alpha owned by the generators it sweeps, and the rounds' lists are merged,
 * so the call returns the top n_select alpha of every generator it computed,
 * ordered as qp_pt2 orders its selection -- the same list, bit for bit, as
 * qp_pt2_generators over those generators gives.  No generator is swept twice.
 *   uniforms   HOST double [n_uniforms] in [0, 1): the random numbers, one per
 *              draw, consumed in order (the caller owns the generator)
 *   e_est, e_err  HOST double [n_states]; n_computed, n_rounds HOST int64 [1]
 *   n_select, sel_dets, sel_e, n_sel: as qp_pt2 (device), over the alpha owned
 *              by the computed generators; unused when n_select = 0
 *   computed_out  optional device uint8 [n_det]: 1 for each determinant whose
 *              eps was computed (in the caller's order), else 0
 * The call is synchronous.  Errors as qp_pt2; QP_E_ARG for det_chunk < 1,
 * draws_per_round < 0, rel_err < 0 or n_select < 0.
 */
int qp_pt2_stochastic(qp_ctx *ctx, const uint64_t *dets, const double *coefs, int64_t n_det,
                      int n_states, const double *E0, const double *uniforms, int64_t n_uniforms,
                      double rel_err, int64_t det_chunk, int64_t draws_per_round, int64_t n_select,
                      int flags, double *e_est, double *e_err, int64_t *n_computed, int64_t *n_rounds,
                      uint64_t *sel_dets, double *sel_e, int64_t *n_sel, uint8_t *computed_out,
                      void *stream);

/*
 * qp_pt2_batched -- many independent wave functions in one sweep call: every
 * system's (generator, batch) work items go into one work list, and each of
 * the two sweep kernels runs as one persistent launch per (n_int, n_states)
 * class over the items of all systems of that class (the generator
 * decomposition of sec. "CIPSI selection and PT2 energy" applied system by
 * system; each system is the computation of qp_pt2, or of qp_pt2_backward).
 *   n_sys          number of systems, 0..QP_MAX_SYSTEMS
 *   sys            host array [n_sys] of qp_system (below)
 *   with_backward  0: the forward sweep (qp_pt2's outputs per system);
 *                  1: the adjoint sweep, which yields E_PT2 and the gradients
 *                  of qp_pt2_backward in one pass over the alpha (selection is
 *                  then not available: n_select must be 0)
 *   flags          QP_FLAG_* (FINGERPRINT, NOCHECK, REUSE_INTEGRALS)
 * The context builds each system's integral layouts (as qp_set_integrals
 * does) into storage of its own; it keeps them, and its other per-system
 * scratch, until qp_destroy.  Results of a system are those qp_pt2 /
 * qp_pt2_backward give for it alone.  The integrals set by qp_set_integrals
 * are neither used nor changed.
 * Host synchronisation: once per system with n_det > 0 (coarse-list sizes,
 * validation), once after the dense kernel (sizes of the handed-over batch
 * lists) and once before the selection sort.
 * Errors: as qp_pt2; a message names the failing system.
 */
typedef struct {
    int n_orb;                  /* 1..256                                           */
    int n_states;               /* 1..4                                             */
    int64_t n_det;              /* >= 0                                             */
    const double *h;            /* device [n_orb][n_orb]                            */
    const double *eri_packed;   /* device, packed as for qp_set_integrals           */
    const uint64_t *dets;       /* device [n_det][2][n_int]                         */
    const double *coefs;        /* device [n_states][n_det]                         */
    const double *E0;           /* device [n_states]                                */
    int64_t n_select;           /* forward only; 0 = no selection                   */
    double *e_pt2;              /* out device [n_states] (required)                 */
    uint64_t *sel_dets;         /* out device [n_select][2][n_int] (n_select > 0)   */
    double *sel_e;              /* out device [n_select][n_states] (n_select > 0)   */
    int64_t *n_sel;             /* out device [1] (n_select > 0)                    */
    qp_pt2_stats *stats;        /* out device [1], optional                         */
    double *eps_gen;            /* out device [n_states][n_det], optional, forward  */
    const double *grad_e_pt2;   /* with_backward: device [n_states] (required)      */
    double *grad_coefs;         /* with_backward: out [n_states][n_det], optional   */
    double *grad_E0;            /* with_backward: out [n_states], optional          */
    double *grad_h;             /* with_backward: out [n_orb][n_orb], optional      */
} qp_system;

int qp_pt2_batched(qp_ctx *ctx, int n_sys, const qp_system *sys, int with_backward, int flags,
                   void *stream);

/*
 * qp_sigma -- sigma vectors of a Davidson iteration over the determinant
 * space of Psi (sec. "Davidson diagonalization", the H U product that
 * dominates it): W = H U, or with QP_SIGMA_S2 in flags W = S^2 U, with
 * S^2 = S_- S_+ + S_z (S_z + 1) applied by second quantisation in the
 * canonical order (up spin-orbitals first).
 *   U, W  device double [n_vec][n_det] (W overwritten)
 * Matrix elements by the Slater-Condon rules as in qp_pt2.  Synchronises
 * once (coarse-list sizes) to prepare the determinant space; with
 * QP_SIGMA_REUSE and the same dets pointer, n_det, integrals and stream as
 * the previous qp_sigma call, the preparation is reused and the call only
 * launches the sigma kernel.  Errors: QP_E_ARG, QP_E_NOINT, QP_E_NORB,
 * QP_E_ELEC, QP_E_DUP, QP_E_OOM, QP_E_HIP.
 */
int qp_sigma(qp_ctx *ctx, const uint64_t *dets, int64_t n_det, int n_vec, const double *U,
             int flags, double *W, void *stream);

/*
 * qp_davidson -- n_states eigenpairs of H in the space of the given
 * determinants (sec. "Davidson diagonalization"): Davidson iterations with
 * the diagonal preconditioner, converged on the lowest Ritz pairs of the
 * subspace.  From the default start these are the lowest eigenpairs in the
 * spaces the tests check against a dense eigensolver; from a guess far from
 * the ground state the iteration can settle on eigenpairs near the guess's
 * energy instead, as Davidson does.  The basis, its sigma vectors (as
 * qp_sigma), the Ritz vectors, residuals and Gram-Schmidt steps stay on the
 * device; only the m x m Rayleigh matrix (m <= max(8 n_states, 24)) and the
 * norms reach the host, which solves the subspace problem.  Converged when
 * every residual ||H x - theta x|| < tol.
 *   guess   device double [n_states][n_det] start vectors, or NULL (unit
 *           vectors on the lowest diagonal elements)
 *   E_out   HOST double [n_states] eigenvalues, ascending
 *   C_out   device double [n_states][n_det] normalised eigenvectors, largest
 *           component positive
 *   s2_out  HOST double [n_states] <S^2> of each vector, or NULL
 *   n_iter  HOST int [1] iterations used, or NULL
 * The call is synchronous.  Errors: as qp_sigma, QP_E_STATES, QP_E_ARG when
 * the guess spans fewer than n_states directions, and QP_E_NOCONV when
 * max_iter iterations leave a residual above tol (the outputs then hold the
 * last iterate).
 */
int qp_davidson(qp_ctx *ctx, const uint64_t *dets, int64_t n_det, int n_states, const double *guess,
                double tol, int max_iter, int flags, double *E_out, double *C_out, double *s2_out,
                int *n_iter, void *stream);

/*
 * qp_energy -- variational energy E0_k = <Psi_k|H|Psi_k> / <Psi_k|Psi_k>
 * (eq. evar) over the determinant list, for preparing the E0 input.
 *   E0_out device double [n_states].  Errors as qp_pt2.
 */
int qp_energy(qp_ctx *ctx, const uint64_t *dets, const double *coefs, int64_t n_det,
              int n_states, int flags, double *E0_out, void *stream);

/*
 * qp_set_timing / qp_last_timing -- diagnostics.  When enabled, every
 * qp_pt2 / qp_pt2_backward call records HIP events on its stream around the
 * sweep kernels (the per-generator batch kernels, the dominant cost).
 * qp_last_timing waits for the last recorded event and writes, in ms:
 * out_ms[0] = the dense sweep kernel, out_ms[1] = the general kernel on the
 * batches handed over to it, out_ms[2] = the call's first enqueued kernel to
 * its last, out_ms[3] = the clean-cell and split-correction kernels of a
 * split sweep (0 when the call did not split), out_ms[4] = the clean-cell
 * kernel alone.  out_ms must hold 5 doubles.  Errors: QP_E_ARG when
 * timing is off or no call has been timed, QP_E_HIP.
 */
int qp_set_timing(qp_ctx *ctx, int enable);
int qp_last_timing(qp_ctx *ctx, double *out_ms);

/*
 * qp_alu_probe -- diagnostic: the vector-ALU issue rate this device reaches,
 * the ceiling against which the sweep kernels' lane operations are priced.
 * Launches 8 workgroups of 256 lanes per compute unit (8 waves per SIMD),
 * each lane running eight independent chains of one instruction:
 * kind = QP_PROBE_F64_FMA (v_fma_f64), QP_PROBE_I32_ADD (v_add_u32) or
 * QP_PROBE_MIXED (the two alternating), iters x 64 instructions per chain
 * set (x 128 for QP_PROBE_MIXED).  One untimed launch, then one launch timed
 * with HIP events on `stream`; blocks until it ends.
 *   out_lane_ops_per_s  host double: instructions x 64 lanes per second.
 * The first call allocates 8 bytes of device memory, freed by qp_destroy.
 * Errors: QP_E_ARG (unknown kind, iters outside [1, 2^24]), QP_E_OOM,
 * QP_E_HIP.
 */
#define QP_PROBE_F64_FMA 0
#define QP_PROBE_I32_ADD 1
#define QP_PROBE_MIXED   2
int qp_alu_probe(qp_ctx *ctx, int kind, int64_t iters, void *stream, double *out_lane_ops_per_s);

/*
 * qp_set_split -- how sweeps (qp_pt2, qp_pt2_backward, qp_pt2_generators,
 * qp_pt2_batched and the rounds of qp_pt2_stochastic) divide their cells
 * between kernels.  A split sweep gives the hole-pair batches that no
 * determinant touches in every cell to the clean-cell kernel, in
 * hole-pair-major order, for the cells no other determinant touches, and to
 * the split-correction kernel for the rest; the dense kernel keeps the other
 * batches.  mode = QP_SPLIT_AUTO (the default) splits a system whose batches
 * hold at least QP_SPLIT_MIN_VIRT particles per spin (n_orb minus the larger
 * electron count), QP_SPLIT_ALWAYS every system, QP_SPLIT_NEVER none.  All
 * give the same alpha set, counts and selection, and energies and gradients
 * equal to rounding (the sums run in another order).  An adjoint call with
 * QP_FLAG_FINGERPRINT is not split.  No device work.  Errors: QP_E_ARG (an
 * unknown mode).
 */
int qp_set_split(qp_ctx *ctx, int mode);

#ifdef __cplusplus
}
#endif
#endif /* QP_PT2_H */
