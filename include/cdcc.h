/*
 * cdcc.h -- C ABI of the MI355X (gfx950) particle-particle ladder library for
 * closed-shell CCSD with Cholesky-decomposed two-electron integrals and
 * Abelian point-group symmetry (arXiv 2512.21909).
 *
 * Operations (paper section "Stationarity with respect to cluster amplitudes:
 * Lambda equations", the PPL equations, plus Appendix A):
 *
 *   T2 ladder      R_ij^ab = sum_cd tau_ij^cd (ac|bd),
 *                  (ac|bd) = sum_P B^P_ac B^P_bd          (CD of eq. 1)
 *   Lambda ladder  Z_ij^ab = sum_ef lambda_ij^ef W_efab,
 *                  W_efab  = sum_P [(B^P_ea - t^P_ea) B^P_fb - B^P_ea t^P_fb],
 *                  t^P_xy  = sum_m t_m^x L^P_ym           (Appendix A)
 *
 * both evaluated with the symmetric-antisymmetric split (S + A, stored halves
 * a>=b, i>=j, c>=d) and blocked by irreducible representation (direct-product
 * decomposition, symmetry section).  (ac|bd) is assembled on the fly in
 * bounded batches; the v^4 tensor never exists.
 *
 * Symmetry: h in {1,2,4,8} irreps labelled 0..h-1; the product of two irreps
 * is their bitwise XOR (D2h and its subgroups in the standard ordering).
 * Orbitals and Cholesky vectors are sorted by irrep, then by local index.
 *
 * Memory: every tensor pointer in cdcc_problem_t is a caller-owned DEVICE
 * pointer to FP64 data in the layout described by cdcc_layout_t (all counts
 * and offsets in elements, not bytes).  The library never frees or keeps a
 * caller pointer after the call's work has completed on the stream.  It owns
 * an internal workspace cache (device memory, per stream) and a plan cache,
 * both released by cdcc_release() or at process exit.
 *
 * Errors: functions return CDCC_OK (0) or a negative status; nothing else
 * crosses the ABI.  Ladder calls are asynchronous on the given stream; an
 * error in argument checking is reported before anything is enqueued.
 */
#ifndef CDCC_H
#define CDCC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CDCC_MAX_IRREP 8

#define CDCC_OK            0
#define CDCC_EINVAL       -1  /* bad layout, pointer, size or option            */
#define CDCC_ENOMEM       -2  /* device workspace could not be allocated        */
#define CDCC_EUNSUPPORTED -3  /* e.g. irrep count not in {1,2,4,8}              */
#define CDCC_EDEVICE      -4  /* HIP runtime error, or no gfx950 device         */
#define CDCC_ESCRATCH     -5  /* needs more than the static scratch of         */
                              /* cdcc_ladder_t2_noalloc                          */

#define CDCC_FP64  0  /* FP64 MFMA throughout                                     */
#define CDCC_MIXED 1  /* split-BF16 MFMA, FP32 accumulation, FP64 combination     */
#define CDCC_MIXED_I8 2  /* four signed 8-bit digits per operand element, int8  */
                         /* MFMA with exact int32 accumulation, FP64 combination */

/* Orbital and Cholesky-vector counts per irrep (entries >= nirrep ignored). */
typedef struct {
  int32_t nirrep;
  int32_t nocc[CDCC_MAX_IRREP];
  int32_t nvir[CDCC_MAX_IRREP];
  int32_t ncd[CDCC_MAX_IRREP];
} cdcc_sym_t;

/*
 * Flat storage of every tensor, filled by cdcc_irrep_layout.
 *
 * Amplitudes (tau, lambda, R, Z, delta): one block per pair irrep G, at
 *   amp_off[G], row-major n_oo[G] x n_vv[G].  Row of (i,j), Gi^Gj = G:
 *   oo_off[G][Gi] + i*nocc[Gj] + j.  Column of (a,b), Ga^Gb = G:
 *   vv_off[G][Ga] + a*nvir[Gb] + b   (i, j, a, b local to their irrep).
 * Cholesky vectors of the vv block, B^P_ac with Ga^Gc = GP: block at
 *   b_off[GP][Ga], dense [a][c][P] (P fastest), nvir[Ga] x nvir[Gc] x ncd[GP].
 * Cholesky vectors of the vo block, L^P_am with Ga^Gm = GP: block at
 *   bvo_off[GP][Ga], dense [a][m][P].
 * Singles t_m^e (Gm == Ge): block at t1_off[G], dense [m][e].
 * Orbital energies: eps_occ[occ_off[G] + i], eps_vir[vir_off[G] + a].
 * Pair energies: dense nocc_tot x nocc_tot matrix, [I][J] with global
 *   occupied indices I = occ_off[Gi] + i.
 * n_oo_pk / n_vv_pk: number of pairs with i>=j / a>=b (orbital order above)
 *   in pair irrep G, i.e. the stored halves of the symmetric-antisymmetric
 *   algorithm.
 */
typedef struct {
  cdcc_sym_t sym;
  int64_t n_oo[CDCC_MAX_IRREP], n_vv[CDCC_MAX_IRREP];
  int64_t n_oo_pk[CDCC_MAX_IRREP], n_vv_pk[CDCC_MAX_IRREP];
  int64_t amp_off[CDCC_MAX_IRREP];
  int64_t oo_off[CDCC_MAX_IRREP][CDCC_MAX_IRREP];
  int64_t vv_off[CDCC_MAX_IRREP][CDCC_MAX_IRREP];
  int64_t b_off[CDCC_MAX_IRREP][CDCC_MAX_IRREP];
  int64_t bvo_off[CDCC_MAX_IRREP][CDCC_MAX_IRREP];
  int64_t t1_off[CDCC_MAX_IRREP];
  int64_t occ_off[CDCC_MAX_IRREP], vir_off[CDCC_MAX_IRREP], cd_off[CDCC_MAX_IRREP];
  int64_t amp_size, b_size, bvo_size, t1_size;
  int64_t nocc_tot, nvir_tot, ncd_tot;
} cdcc_layout_t;

/*
 * One ladder evaluation.  Required: lay, B, X, R.  X is tau (T2) or lambda
 * (Lambda) and must be pair-symmetric, X_ij^ab = X_ji^ba; only its rows with
 * i >= j are read.  R receives the full result (every stored element is
 * written).  Optional outputs (NULL = skip): delta = R / D with
 * D_ij^ab = eps_i + eps_j - eps_a - eps_b (needs eps_occ, eps_vir), and
 * pair_energy e_IJ = sum_ab (2 T_ij^ab - T_ij^ba) R_ij^ab with T = X, or
 * T = energy_amps when that is given (for instance the T2 amplitudes with
 * the Lambda residual).  Lambda only:
 * Bvo and t1 enable the T1 dressing of Appendix A; both NULL gives the
 * undressed W_efab = (ea|fb).  Input buffers must not overlap R/delta.
 */
typedef struct {
  const cdcc_layout_t *lay;  /* host pointer, read during the call only        */
  const double *B;           /* device, lay->b_size                             */
  const double *X;           /* device, lay->amp_size                           */
  double *R;                 /* device out, lay->amp_size                       */
  const double *Bvo;         /* device, lay->bvo_size, or NULL                  */
  const double *t1;          /* device, lay->t1_size, or NULL                   */
  const double *eps_occ;     /* device, lay->nocc_tot, or NULL                  */
  const double *eps_vir;     /* device, lay->nvir_tot, or NULL                  */
  double *delta;             /* device out, lay->amp_size, or NULL              */
  double *pair_energy;       /* device out, nocc_tot*nocc_tot, or NULL          */
  const double *U;           /* Lambda only: device, 2*lay->b_size, the dressed */
                             /* stack of cdcc_lambda_dress (Bvo, t1 unused), or */
                             /* NULL; must be NULL for the T2 ladder            */
  const double *energy_amps; /* device, lay->amp_size, pair-symmetric, or NULL */
                             /* (= X): the T of the pair energies              */
} cdcc_problem_t;

typedef struct {
  int32_t precision;         /* CDCC_FP64, CDCC_MIXED or CDCC_MIXED_I8          */
  int32_t tile_policy;       /* 0 = tile table, k = force assembly class k-1:   */
                             /* 1..3 (FP64), 1..4 (the two split precisions)   */
  int64_t batch_bytes;       /* cap of the (ac|bd) batch buffer, 0 = default:  */
                             /* CDCC_BATCH_MB megabytes if set, else one batch */
                             /* when the whole intermediate fits 16 GiB and    */
                             /* batches of at most 4 GiB otherwise; the vvvv   */
                             /* density's default is 4 GiB                     */
  int32_t contract_kseg;     /* K-table entries per contraction segment (split */
                             /* K), 0 = tile table, else the built-in rule;    */
                             /* changes the rounding order of S and A only     */
  int32_t pad0;
} cdcc_opts_t;

/*
 * Fill *out with the offsets above.  Host only, no device access.  Returns
 * CDCC_EUNSUPPORTED unless nirrep is 1, 2, 4 or 8, CDCC_EINVAL for a NULL
 * pointer or a negative count.
 */
int cdcc_irrep_layout(const cdcc_sym_t *sym, cdcc_layout_t *out);

/*
 * T2 ladder R_ij^ab = sum_cd tau_ij^cd sum_P B^P_ac B^P_bd for nsys >= 1
 * independent systems (each with its own layout) in one batched, persistent
 * launch sequence on `stream` (a hipStream_t, NULL = default stream).
 * opts may be NULL (FP64, default batch size).  Returns CDCC_EINVAL for
 * nsys < 1, NULL probs, a NULL required pointer, or eps missing while delta
 * is requested; CDCC_ENOMEM if the workspace cannot be allocated;
 * CDCC_EDEVICE on a HIP error.
 */
int cdcc_ladder_t2(int32_t nsys, const cdcc_problem_t *probs,
                   const cdcc_opts_t *opts, void *stream);

/*
 * Lambda ladder Z_ij^ab = sum_ef lambda_ij^ef W_efab with the Appendix-A
 * W_efab (X = lambda, R = Z).  Same conventions and errors as cdcc_ladder_t2;
 * Bvo and t1 must be both set or both NULL.  With U set (the stack of
 * cdcc_lambda_dress for these B, Bvo and t1) the dressing is not rebuilt:
 * the result is the dressed ladder, bitwise the same as with Bvo and t1 in
 * FP64.  All problems of one call use the same kind of dressing (none,
 * Bvo/t1, or U).
 */
int cdcc_ladder_lambda(int32_t nsys, const cdcc_problem_t *probs,
                       const cdcc_opts_t *opts, void *stream);

/*
 * The T1-dressed operand of the Lambda ladder (Appendix A, the
 * lambda-independent intermediates t^P_ab = sum_m t_m^a L^P_bm and the
 * W_AbEf they enter; the paper computes them once per Lambda solve).  For
 * every (GP, Ga) block, rows (a, e) with e in Ge = Ga ^ GP (e fastest), each
 * row of 2 N_GP doubles:
 *
 *   U[a][e][P]        = B^P_ea - t^P_ea,   U[a][e][N_GP + P] = t^P_ea,
 *   t^P_ea = sum_m t_m^e L^P_am            (m in Ge),
 *
 * block (GP, Ga) at element 2 * b_off[GP][Ga], so that
 * W_efab = sum_P [U^P_(a,e) U^P_(b,f)] - sum_P [U^(N+P)_(a,e) U^(N+P)_(b,f)]
 * is the ladder's operand product (the second half subtracted).  Blocks with
 * N_GP = 0 or an empty irrep are not written.  B, Bvo, t1 as in
 * cdcc_problem_t (device, read only); U is a caller-owned device buffer of
 * 2 * lay->b_size doubles, written asynchronously on `stream`.  Pass it as
 * cdcc_problem_t.U to every cdcc_ladder_lambda call of the solve (valid
 * while B, Bvo and t1 are unchanged).  CDCC_EINVAL for nsys < 0, a NULL
 * pointer or a bad layout; CDCC_ENOMEM, CDCC_EDEVICE as for the ladder.
 */
typedef struct {
  const cdcc_layout_t *lay;  /* host pointer, read during the call only        */
  const double *B;           /* device, lay->b_size                             */
  const double *Bvo;         /* device, lay->bvo_size                           */
  const double *t1;          /* device, lay->t1_size                            */
  double *U;                 /* device out, 2 * lay->b_size                     */
} cdcc_dress_problem_t;

int cdcc_lambda_dress(int32_t nsys, const cdcc_dress_problem_t *probs, void *stream);

/*
 * One vvvv two-body-density contraction (Appendix "CCSD two-body density
 * matrices": Gamma_AbCd = 1/2 P_+(ab,cd) V_AbCd, V_AbCd = sum_mn
 * tau~_Mn^Cd lambda_Ab^Mn; section "CCSD density matrices": for an RHF
 * reference the spin-adapted Gamma~_pqrs = 2 Gamma_PqRs - Gamma_PqSr;
 * gradient section, eq. for Gamma^P_pr: Gamma^P_pr = sum_qs Gamma~_pqrs
 * L~^P_qs, contracted on the fly), closed-shell spatial form with
 * p = a, q = b, r = c, s = d:
 *
 *   V_abcd  = sum_mn Y_mn^ab X_mn^cd,   Gamma_abcd = 1/2 (V_abcd + V_cdab)
 *   G^P_ac  = sum_bd (2 Gamma_abcd - Gamma_abdc) L^P_bd
 *
 * X = tau~ and Y = lambda in the amplitude layout (any values; the paper
 * leaves tau~ to the caller; no pair symmetry is assumed), L = the
 * transformed Cholesky vectors L~^P_bd and G = the result G^P_ac, both in the
 * Cholesky-vector layout of B (block (GP, Ga) = [a][c][P]).  G receives every
 * stored element.
 */
typedef struct {
  const cdcc_layout_t *lay;  /* host pointer, read during the call only        */
  const double *L;           /* device, lay->b_size                             */
  const double *X;           /* device, lay->amp_size                           */
  const double *Y;           /* device, lay->amp_size                           */
  double *G;                 /* device out, lay->b_size                         */
} cdcc_density_problem_t;

/*
 * vvvv density contraction for nsys >= 0 independent systems, FP64 MFMA,
 * asynchronous on `stream`.  The (ab|cd) intermediate exists only in bounded
 * batches (opts->batch_bytes, default 4 GiB).  opts may be NULL; precision
 * must be CDCC_FP64 (the split precisions return CDCC_EUNSUPPORTED); tile_policy is
 * ignored.  Errors as for cdcc_ladder_t2 (CDCC_EINVAL for a NULL required
 * pointer); inputs must not overlap G.
 */
int cdcc_vvvv_density(int32_t nsys, const cdcc_density_problem_t *probs,
                      const cdcc_opts_t *opts, void *stream);

/*
 * Algorithmic flop count of one vvvv density contraction (host only):
 * flops[0] = the (ab|cd) products (2 flops per (a,b,c,d,m,n) term, both
 * orders of the P_+ pair), flops[1] = the contraction with L (2 flops per
 * (a,c,b,d,P) term); symmetry-allowed blocks only.
 */
int cdcc_density_flops(const cdcc_layout_t *lay, double flops[2]);

/*
 * Layout of tensors whose first index pair is (virtual b, occupied i), filled
 * by cdcc_vo_layout from a layout of cdcc_irrep_layout.  One block per pair
 * irrep G (Gb^Gi = G), row-major with rows (b,i): row
 * vo_off[G][Gb] + b*nocc[Gi] + i (b, i local to their irrep), n_vo[G] rows.
 *   lambda_bi^mn: block at lam_off[G], n_vo[G] x n_oo[G], columns (m,n) as
 *     the rows of the amplitude layout (oo_off[G][Gm] + m*nocc[Gn] + n);
 *   M_bi^dc:      block at m_off[G],   n_vo[G] x n_vv[G], columns (d,c) as
 *     the columns of the amplitude layout (vv_off[G][Gd] + d*nvir[Gc] + c).
 * Host only; CDCC_EINVAL for a NULL pointer.
 */
typedef struct {
  int64_t n_vo[CDCC_MAX_IRREP];
  int64_t vo_off[CDCC_MAX_IRREP][CDCC_MAX_IRREP];
  int64_t lam_off[CDCC_MAX_IRREP];
  int64_t m_off[CDCC_MAX_IRREP];
  int64_t lam_size, m_size;
} cdcc_vo_layout_t;

int cdcc_vo_layout(const cdcc_layout_t *lay, cdcc_vo_layout_t *out);

/*
 * O(O^3 V^3) contraction with the partial symmetric-antisymmetric algorithm
 * (paper: the paragraph closing the section on the I_pq multipliers, example
 * M_bi^dc = sum_mn lambda_Bi^Mn tau~_mn^dc, half the flops of the plain
 * contraction):
 *
 *   M_bi^dc = sum_mn lambda_bi^mn tau_mn^dc
 *
 * lam = lambda_bi^mn (vo layout, lam_off; any values, no symmetry assumed),
 * tau = tau~_mn^dc in the amplitude layout, which must be pair symmetric
 * (tau_mn^dc = tau_nm^cd; only its rows with m >= n are read), M = the
 * result in the vo layout (m_off); every element of M is written.
 */
typedef struct {
  const cdcc_layout_t *lay;  /* host pointer, read during the call only        */
  const double *lam;         /* device, cdcc_vo_layout lam_size                 */
  const double *tau;         /* device, lay->amp_size                           */
  double *M;                 /* device out, cdcc_vo_layout m_size               */
} cdcc_partial_problem_t;

/*
 * The contraction above for nsys >= 0 independent systems, FP64 MFMA,
 * asynchronous on `stream`.  opts may be NULL; precision must be CDCC_FP64
 * (the split precisions return CDCC_EUNSUPPORTED); the other options are ignored.
 * CDCC_EINVAL for nsys < 0, NULL probs with nsys > 0 or a NULL required
 * pointer; CDCC_ENOMEM, CDCC_EDEVICE as for cdcc_ladder_t2.  Inputs must not
 * overlap M.
 */
int cdcc_partial_contract(int32_t nsys, const cdcc_partial_problem_t *probs,
                          const cdcc_opts_t *opts, void *stream);

/*
 * Algorithmic flop count of one partial contraction (host only): flops[0] =
 * the symmetric half S (2 flops per (b,i), m>=n, d>=c term), flops[1] = the
 * antisymmetric half A (2 flops per (b,i), m>n, d>c term); symmetry-allowed
 * blocks only.  The plain contraction costs 2 n_vo n_oo n_vv per irrep.
 */
int cdcc_partial_flops(const cdcc_layout_t *lay, double flops[2]);

/*
 * Symmetry-adapted two-step Cholesky decomposition (paper: section
 * "Symmetry-adapted two-step CD algorithm", Algorithm 1, and the equation
 * L^P_rs = sum_R K^-1_PR (R|rs) of the CD/DF section) of a symmetric
 * positive semidefinite integral matrix given per irrep: V[g] is the dense
 * row-major n[g] x n[g] block of the basis-function pairs of irrep g (device,
 * read only; pairs of different irreps do not couple).
 */
typedef struct {
  int32_t nirrep;                  /* 1, 2, 4 or 8                              */
  int32_t pad0;
  int64_t n[CDCC_MAX_IRREP];       /* pairs per irrep                           */
  const double *V[CDCC_MAX_IRREP]; /* device, n[g] * n[g], or NULL if n[g] = 0  */
} cdcc_cd_matrix_t;

typedef struct {
  double tau;    /* decomposition threshold (> 0): every residual diagonal ends below it */
  double sigma;  /* span factor (0 < sigma <= 1), the paper uses 1e-2                   */
  int32_t qmax;  /* qualified pairs per macro iteration (1 .. 2048), the paper uses 1000 */
  int32_t pad0;
} cdcc_cd_params_t;

/*
 * First step: the Cholesky basis.  Pairs with Diag >= tau form P; each macro
 * iteration qualifies the (at most qmax) largest diagonals of P that are
 * >= sigma * D_max, forms their residual columns, and decomposes them in
 * micro iterations (pivot = the largest qualified diagonal) while that
 * diagonal is >= max(tau, sigma * D_max); pairs whose diagonal falls below
 * tau leave P.  On return piv[g][0 .. npiv[g]) holds the pivots of irrep g
 * (pair indices, in the order chosen); piv[g] is a host array of capacity
 * n[g].  Synchronous: waits for `stream`.  Device workspace is allocated and
 * freed inside the call.  CDCC_EINVAL for a bad argument (NULL pointer,
 * negative n, tau <= 0, sigma outside (0, 1], qmax outside 1 .. 2048),
 * CDCC_EUNSUPPORTED for an irrep count other than 1, 2, 4, 8.
 */
int cdcc_cd_basis(const cdcc_cd_matrix_t *mat, const cdcc_cd_params_t *params,
                  int64_t *const piv[CDCC_MAX_IRREP], int64_t npiv[CDCC_MAX_IRREP],
                  void *stream);

/*
 * Second step: for each irrep, K = the lower Cholesky factor of the metric
 * V[g][piv][piv] and the vectors L^P_r = (K^-1 V[g][piv][:])_Pr, written to
 * L[g] (device, row-major n[g] x npiv[g]: element [r][P], vector index
 * fastest).  piv as returned by cdcc_cd_basis (host arrays).  Asynchronous on
 * `stream` except for the final check of the factorisation, which waits.
 * CDCC_EINVAL for a bad argument, a pivot out of range, or a metric that is
 * not numerically positive definite.
 */
int cdcc_cd_vectors(const cdcc_cd_matrix_t *mat, const int64_t *const piv[CDCC_MAX_IRREP],
                    const int64_t npiv[CDCC_MAX_IRREP], double *const L[CDCC_MAX_IRREP],
                    void *stream);

/*
 * Tile choice (host only).  cdcc_tile_key writes the size class of a shape
 * ("<precision> <t2|lambda> b<h> <T> <K> <M>": the half-octave buckets of
 * its 64 x 64 assembly tile count, their mean Cholesky length and its
 * largest packed occupied pair count) into buf (len bytes); the tile table
 * (tile_table.txt next to the library, or $CDCC_TILE_TABLE) maps exact shapes
 * and size classes to "<assembly class>[:<contraction segment>]", exact
 * entries first, and the autotuner writes it.  cdcc_tile_table_reload makes
 * plans built afterwards read the table again, from path (NULL: the default
 * location).  Tile choices never change an element's arithmetic in the
 * assembly; the contraction segment fixes the order in which S and A are
 * summed.  CDCC_EINVAL for a NULL pointer, a short buffer or a bad
 * precision, CDCC_EUNSUPPORTED for an irrep count other than 1, 2, 4, 8.
 */
int cdcc_tile_key(const cdcc_sym_t *sym, int32_t precision, int32_t lambda, char *buf, int32_t len);
int cdcc_tile_table_reload(const char *path);

/*
 * Algorithmic flop count of one evaluation (host only): flops[0] = (ac|bd)
 * assembly, flops[1] = contraction, flops[2] = T1 dressing (Lambda with t1).
 * kind: 0 = T2, 1 = Lambda, 2 = Lambda with dressing.  Counts the stored
 * halves (a>=b for the assembly; i>=j, a>=b, c>=d for the contraction) and
 * only symmetry-allowed blocks, with 2 flops per multiply-add.
 */
int cdcc_ladder_flops(const cdcc_layout_t *lay, int32_t kind, double flops[3]);

/*
 * Device bytes the library allocates for a call with these problems and
 * options (workspace only; excludes the caller's buffers).  Host only.
 */
int cdcc_workspace_bytes(int32_t nsys, const cdcc_problem_t *probs,
                         const cdcc_opts_t *opts, int32_t lambda, int64_t *bytes);

/*
 * Kernel timing (instrumentation for benchmarks).  While enabled, every ladder
 * call records a HIP event pair on its own stream around each kernel class:
 * 0 = T1 dressing, 1 = amplitude packing, 2 = (ac|bd) batch assembly,
 * 3 = contraction + unpack, 4 = pair energies, 5 = operand slicing (mixed),
 * 6 = vvvv density (ab|cd) batch, 7 = vvvv density contraction with L,
 * 8 = vvvv density split-K reduction, 9 = partial contraction +/- packing,
 * 10 = partial contraction GEMM, 11 = Cholesky basis: diagonals and
 * residual columns, 12 = Cholesky basis: micro iterations, 13 = Cholesky
 * vectors (second step).
 * cdcc_timing_read waits for the recorded events, returns the summed elapsed
 * milliseconds and launch counts per class (arrays of CDCC_TIMING_CLASSES)
 * and clears the record.
 */
#define CDCC_TIMING_CLASSES 14
int cdcc_timing_enable(int32_t on);
int cdcc_timing_read(double ms[CDCC_TIMING_CLASSES], int64_t launches[CDCC_TIMING_CLASSES]);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the T2
 * ladder of cdcc_ladder_t2, same arguments, results and errors, computed
 * without any device or pinned-host allocation.  Plan tables and workspace
 * live in a static device array of CDCC_NOALLOC_SCRATCH_BYTES that every GPU
 * the library runs on holds until the process ends; the (ac|bd) batch is
 * sized to what is left of it.  A call whose tables and workspace do not fit
 * returns CDCC_ESCRATCH before anything is enqueued.  The launches are
 * enqueued directly (no graph); plans are cached on the host.  All calls on
 * one GPU share the array: calls that overlap in time on one GPU (other
 * streams, or unordered host threads) race and must be serialised by the
 * caller; consecutive calls on one stream are ordered and each call writes
 * every byte it reads.
 */
#define CDCC_NOALLOC_SCRATCH_BYTES (256ll << 20)
int cdcc_ladder_t2_noalloc(int32_t nsys, const cdcc_problem_t *probs,
                           const cdcc_opts_t *opts, void *stream);

/* Static, human-readable text for a status code. */
const char *cdcc_status_string(int status);

/* Free the workspace and plan caches of every device (waits for the device). */
int cdcc_release(void);

#ifdef __cplusplus
}
#endif
#endif /* CDCC_H */
