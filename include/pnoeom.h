/*
 * pnoeom -- closed-shell EOM-CCSD sigma vectors and a Davidson eigensolver with
 * state-averaged PNO truncation of the doubles, for one AMD Instinct MI355X (gfx950).
 *
 * The operations follow Peng, Clement & Valeev, "Exploration of Reduced Scaling
 * Formulation of EOM-CCSD Based on State-Averaged Pair Natural Orbitals"
 * (arXiv:1802.06738):
 *   - H-bar = exp(-T) H exp(T) and the EOM eigenproblem H-bar R|0> = E R|0> with
 *     T = T1 + T2, R = R1 + R2 parameterised by the spin-summed excitation
 *     operators E_i^a, E_ij^ab (Methods section, the EOM ansatz and its operator
 *     parameterisation);
 *   - the Hamiltonian is given by density-fitting factors (Computational Details);
 *   - first-order (MP1) amplitudes as the default T2 (Methods, eq. T1);
 *   - the ladder intermediate W_ab^cd (Methods, the largest intermediate);
 *   - CIS(D) doubles, state-specific pair densities and their state average
 *     (Methods, the CIS(D) doubles equation, the pair-density equation and the
 *     state-averaged density equation), PNO truncation at T_CutPNO and OSVs from
 *     diagonal pairs at T_CutOSV = T_CutPNO/10 (Methods; Computational Details);
 *   - the PNO-modified Davidson step: residuals transformed to the semicanonical
 *     OSV/PNO bases, preconditioned there and back-transformed (Methods, the
 *     state-averaged PNO simulation in the Davidson solver).
 *
 * Conventions
 *   o = active occupied orbitals, v = virtual orbitals, nmo = o + v, naux = DF rank.
 *   Orbitals are indexed occupied first.  All floating-point arguments are FP64.
 *   R1 / sigma1 layout [o][v];  R2 / sigma2 layout [o][o][v][v] (full array) with
 *   R2[i][j][a][b] = R2[j][i][b][a] (the singlet space).
 *   Device pointers are HIP device addresses on the context's device; host pointers
 *   are ordinary CPU memory.  The caller owns every buffer it passes; pointers must
 *   stay valid only for the duration of the call.  The library copies what it
 *   keeps into memory owned by the context (freed by pnoeom_destroy).
 *   All device work is ordered on the stream given to pnoeom_create; host outputs
 *   are complete when a call returns.  One context per host thread.
 *   Every entry point returns a status code (0 = success); no C++ exception
 *   crosses this boundary.  pnoeom_last_error() gives the message of the last
 *   failure on a context.
 */
#ifndef PNOEOM_H
#define PNOEOM_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pnoeom_ctx pnoeom_ctx;

enum {
  PNOEOM_OK = 0,
  PNOEOM_EINVAL = -1,   /* bad argument (sizes, null pointers, unknown enum) */
  PNOEOM_ENOMEM = -2,   /* device allocation failed */
  PNOEOM_EHIP = -3,     /* HIP runtime error (message has the HIP error string) */
  PNOEOM_ENOTCONV = -4, /* Davidson reached max_iter without convergence */
  PNOEOM_ESTATE = -5,   /* call out of order (e.g. sigma before build_df) */
  PNOEOM_ECOMPLEX = -6, /* converged with a complex Ritz pair (real parts returned) */
  PNOEOM_EABORTED = -7  /* stopped by abort_after_iter (checkpoint written if requested) */
};

enum { PNOEOM_FP64 = 0, PNOEOM_FP32 = 1, PNOEOM_BF16 = 2 }; /* contraction precision */
enum { PNOEOM_CANONICAL = 0, PNOEOM_PNO = 1 };              /* vector space */

/* Create a context for o occupied, v virtual orbitals and naux fitting functions.
 * hip_stream: a hipStream_t (NULL = the default stream).  Allocates nothing large. */
int pnoeom_create(int o, int v, int naux, void* hip_stream, pnoeom_ctx** out);

/* Free every device buffer of the context.  Accepts NULL. */
void pnoeom_destroy(pnoeom_ctx* ctx);

/* Message of the last failed call on ctx ("" if none).  Owned by ctx. */
const char* pnoeom_last_error(const pnoeom_ctx* ctx);

/* Build the T-dependent intermediates of sigma (H-bar pieces, dressed DF factors,
 * the ladder intermediate W_ab^cd of the Methods section).
 *   B    : device [naux][nmo][nmo], B[Q][p][q] = B[Q][q][p]; (pq|rs) = sum_Q B[Q][p][q] B[Q][r][s]
 *   eps  : device [nmo], orbital energies; the Fock matrix is diag(eps)
 *   t1   : device [o][v] or NULL (T1 = 0)
 *   t2   : device [o][o][v][v] or NULL (first-order amplitudes (ia|jb)/(e_i+e_j-e_a-e_b))
 *   precision : PNOEOM_FP64, PNOEOM_FP32 or PNOEOM_BF16 (precision of the large
 *               contractions used by later sigma calls; FP64 copies are always kept).
 *               BF16: the particle ladder runs on bfloat16 operands (W+/- and the
 *               packed trial amplitudes, rounded to nearest even) with FP32
 *               accumulation; the other large contractions run in FP32.
 * Discards the workspaces and SA-PNOs of an earlier build_df (build_sapno again).
 * Errors: EINVAL (null B/eps, bad precision), ENOMEM, EHIP. */
int pnoeom_build_df(pnoeom_ctx* ctx, const double* B, const double* eps, const double* t1,
                    const double* t2, int precision);

/* Lowest nroots CIS excitation energies and unit-norm singles vectors of the bare
 * Hamiltonian, A_{ia,jb} = d_ij d_ab (e_a - e_i) + 2(ia|jb) - (ij|ab).
 *   omega_out : host [nroots];  vec_out : device [nroots][o][v] or NULL.
 * Requires build_df.  Errors: ESTATE, EINVAL, ENOTCONV. */
int pnoeom_cis(pnoeom_ctx* ctx, int nroots, double* omega_out, double* vec_out);

/* Build state-averaged PNOs / OSVs (Methods: CIS(D) doubles of the lowest
 * nstates CIS roots, pair densities averaged over the states, per-pair
 * eigenvectors kept when |occupation| >= tcut_pno; OSVs from diagonal pairs with
 * tcut_osv (tcut_osv < 0 selects tcut_pno/10)), rotated to the semicanonical basis.
 *   npno_out : host [o(o+1)/2] (pairs i <= j, row-major) or NULL
 *   nosv_out : host [o] or NULL
 * Requires build_df.  Errors: ESTATE, EINVAL, ENOMEM, EHIP. */
int pnoeom_build_sapno(pnoeom_ctx* ctx, int nstates, double tcut_pno, double tcut_osv, int* npno_out,
                       int* nosv_out);

/* Length of one PNO-space vector and its layout: singles block [sum_i nosv_i]
 * followed by the pair blocks i <= j, each n_p x n_p row-major.
 *   offsets : host [o + o(o+1)/2 + 1] start of each block (singles of i = 0..o-1,
 *             then pairs; the last entry is the end of the blocks) or NULL;
 *   len : host, total length: the end of the blocks rounded up to an even count (an odd
 *         total is followed by one padding element, which compress sets to zero).
 * Off-diagonal pair blocks are stored multiplied by sqrt(2), so the plain dot
 * product of two PNO-space vectors is the full-array Frobenius inner product.
 * Requires build_sapno.  Errors: ESTATE. */
int pnoeom_pno_layout(const pnoeom_ctx* ctx, long long* offsets, long long* len);

/* PNO projection and back-transformation of nvec vectors (Methods: the residual
 * transformation into the OSV / PNO bases and the projection back to the canonical
 * space of the PNO simulation), in the semicanonical bases built by build_sapno.
 *   direction 0 (compress): x[q] = ( U^i^T r1[q]_i , w_p U^{ij}^T r2[q]^{ij} U^{ij} )
 *                           reading r1 [nvec][o][v] and r2 [nvec][o][o][v][v] (device)
 *   direction 1 (expand):   r1[q]_i = U^i x_i, r2[q]^{ij} = U^{ij} x_p U^{ij}^T / w_p and
 *                           r2[q]^{ji} = (r2[q]^{ij})^T, writing r1, r2 (device)
 * x is device [nvec][len] (pnoeom_pno_layout); w_p = sqrt(2) for i < j, 1 for i = j.
 * expand(compress(r)) is the orthogonal projector P of the PNO space applied to r.
 * Requires build_sapno.  Errors: ESTATE, EINVAL, EHIP. */
int pnoeom_pno_transform(pnoeom_ctx* ctx, int nvec, int direction, double* r1, double* r2, double* x);

/* sigma = <mu|[H-bar, R]|0> for nvec trial vectors.
 *   space = PNOEOM_CANONICAL: r1 device [nvec][o][v], r2 device [nvec][o][o][v][v]
 *           with the closed-shell pair symmetry r2[q][i][j][a][b] = r2[q][j][i][b][a]
 *           (the doubles space of the method; the contractions rely on it);
 *           s1, s2 the same shapes (outputs).
 *   space = PNOEOM_PNO: r1 = device [nvec][len] PNO-space vectors (r2 ignored, may be
 *           NULL); s1 = device [nvec][len] receives P sigma in the same layout.
 *   precision : PNOEOM_FP64, PNOEOM_FP32 or PNOEOM_BF16 for the large contractions
 *               (FP32 / BF16 need build_df with the same precision; FP64 always works).
 * Requires build_df (and build_sapno for PNO).  Errors: ESTATE, EINVAL, ENOMEM, EHIP. */
int pnoeom_apply_sigma(pnoeom_ctx* ctx, int nvec, const double* r1, const double* r2, double* s1,
                       double* s2, int space, int precision);

/* States whose CIS(D) pair densities pnoeom_build_sapno averages (Methods: the
 * state-specific density of one state and the state average over several).
 *   states : host [n] distinct CIS state indices, 0 = the lowest root; n = 1 gives the
 *            state-specific PNOs of that state; n = 0 restores the default (the lowest
 *            nstates of the build_sapno call, whose nstates is ignored while a list is set).
 * Errors: EINVAL (null ctx, negative or repeated index, states NULL with n > 0). */
int pnoeom_set_pno_states(pnoeom_ctx* ctx, int n, const int* states);

/* Ladder of the PNO-space sigma, for the next pnoeom_build_sapno.  The projected ladder of
 * a pair is U^T [sum_cd W_ab^cd (U Rbar U^T)_cd] U = sum_Q Bbar^Q Rbar Bbar^Q^T with the
 * pair's factors Bbar^Q = U^T B~^Q U (W_ab^cd = sum_Q B~^Q_ac B~^Q_bd; Methods, the PNO
 * simulation of the Davidson step): 4 n_p^3 naux flop per pair and vector instead of the
 * pair's rows of the canonical ladder (about v^4).  Pairs with n_p <= max_native take that
 * route (their per-pair factors, n_p^2 naux words each, are built by build_sapno); the others
 * keep the canonical ladder.  max_native = -1 (default): automatic, the n_p where
 * 128 n_p^3 naux = v^4, lowered until the factors fit in a fifth of the free memory;
 * 0: every pair canonical.  Results equal up to rounding order.
 * Errors: EINVAL (null ctx, max_native < -1). */
int pnoeom_set_pno_ladder(pnoeom_ctx* ctx, int max_native);

/* The split chosen by the last build_sapno: the n_p bound, the number of pairs with the
 * PNO-space ladder and with the canonical one, and the PNO-space ladder's flops per vector.
 * Any output may be NULL.  Errors: EINVAL (null ctx), ESTATE (before build_sapno). */
int pnoeom_pno_ladder_stats(const pnoeom_ctx* ctx, int* cut, int* native_pairs, int* canonical_pairs,
                            double* native_flops);

/* Storage of the particle-particle ladder W_ab^cd = sum_Q B~^Q_ac B~^Q_bd (Methods: the
 * largest intermediate; B~ the T1-dressed factors), for the next pnoeom_build_df:
 *   mode PNOEOM_LADDER_AUTO (0): cached when the packed W+/- fit in 60% of the free
 *        device memory, else streamed;
 *   mode PNOEOM_LADDER_CACHED (1): W+/- (v^4/2 words) built once and kept;
 *   mode PNOEOM_LADDER_STREAMED (2): never stored; every sigma rebuilds the rows of
 *        W+/- from B~_vv one slab of a-values at a time (an MFMA GEMM over Q per slab)
 *        and contracts them at once with all trial vectors of the call.  The results
 *        equal those of the cached mode up to rounding order.
 *   max_slab : upper bound on the a-values per slab (0 = from the memory budget: 30%
 *        of the free device memory, 256 MB to 64 GB).
 * Errors: EINVAL (null ctx, bad mode, max_slab < 0). */
enum { PNOEOM_LADDER_AUTO = 0, PNOEOM_LADDER_CACHED = 1, PNOEOM_LADDER_STREAMED = 2 };
int pnoeom_set_ladder_mode(pnoeom_ctx* ctx, int mode, int max_slab);

/* Evaluation of the R1-driven three-body ring terms of sigma2 (Methods: the EOM sigma
 * equations of the cited Stanton-Bartlett formalism), for the next pnoeom_build_df.  The
 * integrals (ij|ab)' of the R1-transformed factors are sum_c r_j^c (ic|ab)~ - sum_l r_l^a
 * (ij|lb)~, so their products with T2 can go through two T-only intermediates built
 * once per T: Y = (ic|ab)~ T (v^2 x 2ov words) and Z = (ij|lb)~ T (o^2 x 2ov words),
 * at 4 o^2 v^3 + 4 o^3 v^2 flop per trial vector, or through (ij|ab)' itself as an
 * ov x ov operand of the ring product (4 (ov)^3 flop per vector, no extra storage).
 *   mode 0: the intermediates when they take at most a third of the free device memory;
 *   mode 1: never;  mode 2: always (ENOMEM at build_df if they do not fit).
 * pnoeom_ring_mode_used returns 2 (intermediates) or 1 for the current build, ESTATE
 * before build_df.  Errors: EINVAL (null ctx, bad mode). */
int pnoeom_set_ring_mode(pnoeom_ctx* ctx, int mode);
int pnoeom_ring_mode_used(const pnoeom_ctx* ctx);

/* Passes of the bfloat16 ring products of PNOEOM_BF16 contractions (next pnoeom_build_df;
 * only with the T-only ring intermediates, else those products run on FP32 MFMA): 1 = one
 * bfloat16 product (inputs rounded to bfloat16, relative error ~2^-8), 3 = each operand
 * split as hi + lo (both bfloat16) and hi hi + hi lo + lo hi summed in FP32 by one GEMM of
 * three times the depth (relative error ~2^-16).  Default 1.  Errors: EINVAL. */
int pnoeom_set_bf16_passes(pnoeom_ctx* ctx, int passes);

/* Which contractions PNOEOM_BF16 puts on bfloat16 MFMA (next pnoeom_build_df); all of them
 * accumulate in FP32, and the small / R1-one-index products stay FP64 in every scope.
 *   scope 0: the particle ladder and (with the T-only ring intermediates) the ring products
 *            R^s [Dr | Xr] and R_ia DX2; the other large contractions run on FP32 MFMA;
 *   scope 1: also the hole ladder W_klij R_kl^ab, X_klij = sum_cd R_ij^cd (kc|ld) and its
 *            product with T, M1 = U(R) B~_ov, the DF-factorised ring terms and the R1 ring
 *            term through Yr (when their bfloat16 staging fits: o <= v, o v naux <= o^2 v^2).
 * Default 1.  The bfloat16 rounding of both operands of a product term (relative 2^-9 each)
 * bounds each product's error by 2^-8 sum |a||b|.  Errors: EINVAL. */
int pnoeom_set_bf16_scope(pnoeom_ctx* ctx, int scope);

/* Prepare the context for pnoeom_ladder_apply alone: the dressed virtual factors
 * B~^Q_ac = B^Q_ac - sum_k t_k^a B^Q_kc (the virtual block of the T1 similarity
 * transformation of the Methods section) and the streamed-ladder workspace, without
 * the other intermediates of build_df.  For workloads whose W does not fit one GPU
 * (v = 900: W+/- take 1.3 TB in FP64): each GPU of a pair-sharded sigma applies the
 * ladder to the pair blocks it owns.
 *   B  : device [naux][nmo][nmo] as in pnoeom_build_df (read during the call only)
 *   t1 : device [o][v] or NULL (T1 = 0)
 *   precision : as in pnoeom_build_df (FP32 / BF16 copies of B~ for those precisions)
 * Discards the intermediates of an earlier build_df (apply_sigma then needs build_df
 * again).  Device memory held: B~ (v^2 naux words FP64, plus the low-precision copy)
 * and the slab workspace.  Errors: EINVAL, ENOMEM, EHIP. */
int pnoeom_build_ladder(pnoeom_ctx* ctx, const double* B, const double* t1, int precision);

/* The particle-particle ladder of nmat doubles blocks:
 *   Y[m][a][b] = sum_cd W_ab^cd X[m][c][d],   W_ab^cd = sum_Q B~^Q_ac B~^Q_bd,
 * i.e. the ladder term of sigma2 for the pair blocks X[m] = R_ij (any pairs, any
 * vectors).  X, Y : device [nmat][v][v] FP64 (may not overlap).  precision as in
 * pnoeom_apply_sigma: FP32 / BF16 contract in that precision (BF16: bfloat16
 * operands, FP32 accumulation) and need the same precision at build time.
 * Uses the cached W+/- when build_df cached them, else streams W from B~.
 * Requires build_df or build_ladder.  Errors: ESTATE, EINVAL, ENOMEM, EHIP. */
int pnoeom_ladder_apply(pnoeom_ctx* ctx, int nmat, const double* X, double* Y, int precision);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): pnoeom_ladder_apply without any
 * device allocation, hipFree or allocating library call.  Same arguments, layout and
 * result as pnoeom_ladder_apply (same kernels; K is never split, so FP64 / FP32 results
 * may differ from it in the last bits of the summation order; BF16 results are equal).
 * The packed operands and sigma+/- rows of the call are staged in a fixed device array
 * of 128 MiB per GPU (a global of the library's device code: the HIP runtime places one
 * copy on each GPU the library runs on, held until the process ends), so calls that overlap on one GPU (other streams,
 * other threads, other contexts) race for it: serialise them.  The array keeps what the
 * last call left; each call clears what it needs cleared.  Needs W+/- cached by build_df
 * (EINVAL when the ladder is streamed, which needs its slab workspace).  EINVAL when
 * nmat v^2 exceeds the array (pnoeom_ladder_noalloc_limit gives the largest nmat).
 * Errors: ESTATE, EINVAL, EHIP. */
int pnoeom_ladder_apply_noalloc(pnoeom_ctx* ctx, int nmat, const double* X, double* Y, int precision);

/* Largest nmat pnoeom_ladder_apply_noalloc accepts for this context's v in a precision
 * (host arithmetic only); -1 for a null context or an unknown precision. */
long long pnoeom_ladder_noalloc_limit(const pnoeom_ctx* ctx, int precision);

/* The phases of the last pnoeom_davidson call on this context: phase 0 = the main run
 * (with precision FP32 / BF16 and refine_fp64 the mixed-precision run before the
 * refinement, else the whole run), phase 1 = the FP64 refinement.  Copies up to cap
 * Ritz values and residual norms (host), the iterations, sigma evaluations and the wall
 * seconds of that phase.  ESTATE when the phase did not run; EINVAL for bad arguments. */
int pnoeom_davidson_phase(const pnoeom_ctx* ctx, int phase, int cap, double* omega_out, double* resnorm_out,
                          int* iters_out, int* nsigma_out, double* seconds_out);

typedef struct {
  int space;           /* PNOEOM_CANONICAL or PNOEOM_PNO */
  int precision;       /* PNOEOM_FP64, PNOEOM_FP32 or PNOEOM_BF16 contractions; subspace work is FP64 */
  double tol_e;        /* |theta_k - theta_k(previous)| bound (Eh) */
  double tol_r;        /* residual 2-norm bound; <= 0 selects 0.1*sqrt(tol_e) */
  int max_sub;         /* largest subspace before collapse to the Ritz vectors */
  int max_iter;        /* iteration limit (ENOTCONV when reached) */
  int refine_fp64;     /* precision FP32/BF16: finish with FP64 sigma from the converged roots */
  int verbose;         /* 1: print one line per iteration to stderr */
  int nextra;          /* further Ritz pairs tracked and kept at collapse (need not converge) */
  double mixed_tol_e;  /* refine_fp64: bounds of the FP32/BF16 phase before the FP64 refinement; */
  double mixed_tol_r;  /*   <= 0 selects tol_e / tol_r (the final bounds are always tol_e, tol_r) */
  /* Checkpoint / resume (host files).  A checkpoint holds the Ritz values and Ritz vectors
   * of all tracked roots after an iteration, in the layout of the space (canonical
   * [r1 | r2] or compressed PNO vectors), plus the phase (main run or FP64 refinement). */
  int ckpt_every;          /* > 0: write ckpt_path every ckpt_every iterations (counted over both phases) */
  int abort_after_iter;    /* > 0: after that iteration write ckpt_path (if set) and return PNOEOM_EABORTED */
  const char* ckpt_path;   /* checkpoint file, or NULL */
  const char* resume_path; /* NULL, or a checkpoint of the same space and vector length: its Ritz
                              vectors replace the CIS guess (a refinement-phase checkpoint resumes
                              in the FP64 refinement) */
  const char* log_path;    /* NULL, or a file to which one JSON line per iteration is appended:
                              phase, iteration, subspace size, sigma count, Ritz values, residual
                              norms, changes of the Ritz values, seconds since the call began and
                              seconds spent in sigma so far (the stream is synchronised around
                              each sigma block only when a log is written) */
} pnoeom_davidson_opts;

/* Fill opts with the defaults (canonical, FP64, tol_e 1e-8, tol_r 1e-5, max_sub 60,
 * max_iter 200, nextra 0, mixed_tol_e = mixed_tol_r = 0, no checkpoints, no resume, no log). */
void pnoeom_davidson_defaults(pnoeom_davidson_opts* opts);

/* Lowest-real-part EOM-CCSD roots by the Davidson method with the PNO
 * modification of the correction step (Methods).  Guess: the nroots lowest CIS
 * vectors projected onto the space.
 *   omega_out   : host [nroots] excitation energies (Eh)
 *   resnorm_out : host [nroots] final residual norms or NULL
 *   iters_out   : host, iterations used, or NULL
 *   nsigma_out  : host, number of sigma vectors evaluated, or NULL
 * Requires build_df (and build_sapno for PNO).
 * Errors: ESTATE, EINVAL (also an unreadable or mismatched resume file), ENOMEM, EHIP,
 * ENOTCONV (omega_out holds the last Ritz values), ECOMPLEX (converged; real parts
 * returned), EABORTED (abort_after_iter reached; omega_out holds that iteration's Ritz
 * values and the checkpoint, if asked for, is written). */
int pnoeom_davidson(pnoeom_ctx* ctx, int nroots, const pnoeom_davidson_opts* opts, double* omega_out,
                    double* resnorm_out, int* iters_out, int* nsigma_out);

/* ---------------------------------------------------------------- CCSD ground state
 * The CC energy E_CC = <0| exp(-T) H exp(T) |0> and the projected amplitude equations
 * <mu| exp(-T) H exp(T) |0> = 0 for all singles and doubles mu (Methods: the CC ground
 * state whose H-bar the EOM step uses).  With such T, the EOM-CCSD sigma of build_df is
 * the H-bar block minus E_CC, and for two electrons (o = 1) CCSD and EOM-CCSD are exact. */
typedef struct {
  int max_iter;     /* Jacobi/DIIS steps at most (ENOTCONV when reached) */
  double tol_e;     /* |E_CC change| of the last step (Eh) */
  double tol_r;     /* largest |Omega| over singles and doubles (Eh) */
  int diis_size;    /* (amplitude, step) pairs kept for Pulay's DIIS; <= 1: plain Jacobi steps */
  int precision;    /* contraction precision of the build_df done at the final amplitudes */
  /* Ground-state PNO-CCSD simulation (Methods: the modified Jacobi update) when gs_tcut_pno >= 0:
   * PNOs / OSVs of the pair densities of the first-order amplitudes, kept when |occupation| >=
   * gs_tcut_pno (pairs) or gs_tcut_osv (diagonal pairs; < 0 selects gs_tcut_pno / 10), made
   * semicanonical in the Fock matrix; the start is projected onto that space, every residual is
   * transformed into the OSV / PNO basis, divided there by f_ii (+ f_jj) - fbar_a (- fbar_b),
   * extrapolated by DIIS and transformed back, and tol_r bounds that transformed residual
   * (off-diagonal pair blocks weighted by sqrt 2).  gs_tcut_pno = 0 keeps every PNO. */
  double gs_tcut_pno;
  double gs_tcut_osv;
} pnoeom_ccsd_opts;

/* Fill opts with the defaults (max_iter 100, tol_e 1e-10, tol_r 1e-8, diis_size 8, FP64,
 * canonical: gs_tcut_pno = gs_tcut_osv = -1). */
void pnoeom_ccsd_defaults(pnoeom_ccsd_opts* opts);

/* CCSD residual Omega_mu = <mu| exp(-T) H exp(T) |0> and correlation energy of given
 * amplitudes (all device pointers; B, eps as for build_df; t2 must satisfy
 * t2[j][i][b][a] = t2[i][j][a][b]).
 *   r1_out : device [o][v];  r2_out : device [o][o][v][v];  e_corr_out : host, E_CC - E_ref
 * Rebuilds the context's intermediates for its own use and leaves none behind: call
 * build_df again before apply_sigma / davidson.  Errors: EINVAL, ENOMEM, EHIP. */
int pnoeom_ccsd_residual(pnoeom_ctx* ctx, const double* B, const double* eps, const double* t1,
                         const double* t2, double* r1_out, double* r2_out, double* e_corr_out);

/* Solve the CCSD equations by Jacobi steps (denominators e_i - e_a, e_i + e_j - e_a - e_b)
 * with Pulay's DIIS, from T1 = 0 and the first-order T2 (start = 0) or from the given
 * t1, t2 (start = 1).
 *   t1, t2 : device [o][v], [o][o][v][v]; the converged (or last) amplitudes on return
 *   e_corr_out : host, E_CC - E_ref;  resmax_out : host, largest |Omega|, or NULL
 *   iters_out  : host, steps taken, or NULL
 * On return the context holds the intermediates of build_df at those amplitudes in
 * opts->precision (ready for apply_sigma / davidson); earlier SA-PNOs are discarded.
 * opts NULL selects the defaults.  Device memory: 2 (diis_size + 2) vectors of o v + o^2 v^2
 * doubles besides the intermediates.
 * Errors: EINVAL, ENOMEM, EHIP, ENOTCONV (max_iter reached or the iteration diverged; the
 * last amplitudes are returned; after a divergence to non-finite values the context holds
 * no intermediates, and apply_sigma / davidson return ESTATE until the next build_df). */
int pnoeom_ccsd(pnoeom_ctx* ctx, const double* B, const double* eps, double* t1, double* t2, int start,
                const pnoeom_ccsd_opts* opts, double* e_corr_out, double* resmax_out, int* iters_out);

/* Convergence history of the last pnoeom_ccsd on ctx: E_CC - E_ref and the largest |Omega|
 * of every amplitude set it evaluated (the start, then one per step).
 *   energies, resmax : host [cap] (may be NULL when cap = 0);  n_out : host, number of entries
 *                      (entries past cap are not copied).  Errors: EINVAL. */
int pnoeom_ccsd_history(const pnoeom_ctx* ctx, int cap, double* energies, double* resmax, int* n_out);

/* PNO and OSV counts of the ground-state PNOs of the last pnoeom_ccsd with gs_tcut_pno >= 0.
 *   npno_out : host [o(o+1)/2] (pairs i <= j, row-major) or NULL;  nosv_out : host [o] or NULL
 * Errors: ESTATE (no ground-state PNOs on ctx: none built, or a canonical pnoeom_ccsd ran
 * since), EINVAL. */
int pnoeom_ccsd_gs_counts(const pnoeom_ctx* ctx, int* npno_out, int* nosv_out);

/* Eigenvalues and right eigenvectors of a small dense real matrix on the host
 * (Householder reduction to Hessenberg form, shifted QR iteration, inverse
 * iteration for the vectors).  Used for the Davidson subspace matrix.
 *   a  : host [n][n] row-major (not modified)
 *   wr, wi : host [n] real / imaginary parts, sorted by real part
 *   vr : host [n][n] or NULL; column k is the real part of the eigenvector of
 *        eigenvalue k, unit 2-norm.
 * Errors: EINVAL (n < 1 or null), ENOTCONV (QR iteration failed). */
int pnoeom_host_eig(int n, const double* a, double* wr, double* wi, double* vr);

/* Graph mode: sigma blocks applied by pnoeom_davidson and pnoeom_apply_sigma are
 * captured once per (number of vectors, precision, space) into a HIP graph and
 * replayed afterwards (launch-bound small systems gain most).  The first call of a
 * shape runs eagerly on a second stream of the context and its calls are captured;
 * replays read and write fixed staging buffers (copied from / to the caller's vectors
 * on the context stream) and are re-captured whenever a workspace the graph refers to
 * has moved.  build_df and build_sapno discard the graphs.  While a graph replays, the
 * ladder / region timings of pnoeom_last_timing cover only the eager calls.
 * pnoeom_graph_stats reports captures, replays and cached graphs.
 * Errors: EINVAL (null ctx), EHIP. */
int pnoeom_set_graph_mode(pnoeom_ctx* ctx, int enable);
int pnoeom_graph_stats(const pnoeom_ctx* ctx, int* captures, int* launches, int* cached);

/* Measured ceilings of the device, for roofline reports next to the published
 * figures: dense MFMA TFLOP/s (FP64 16x16x4, FP32 16x16x4, BF16 16x16x32 with FP32
 * accumulation) from register-only loops on every CU, and HBM GB/s of a plain
 * device copy of 1 GiB (read + write bytes).  Any output pointer may be NULL.
 * Allocates 2 GiB of device memory for the duration of the call.
 * Errors: EHIP, ENOMEM. */
int pnoeom_probe_peaks(pnoeom_ctx* ctx, double* fp64_tflops, double* fp32_tflops, double* bf16_tflops,
                       double* copy_gbs);

/* GEMM tile tuning (process-wide).  Every contraction of the library goes through one
 * MFMA GEMM whose tile shape (128x128, 64x64, 32x128, 128x32) and split of the K loop
 * (automatic when the output has fewer tiles than CUs, none, or wider) can be chosen
 * per shape.  A shape key is 8 integers {element size 8|4, ta, tb, reduce (batched
 * products summed), M, N, K, batch}; a variant is 3 * tile kind + split mode.
 *   pnoeom_gemm_record(1) starts collecting the keys launched (clearing earlier ones),
 *     (0) stops;  pnoeom_gemm_recorded copies up to cap keys into keys[8*i..] (host)
 *     and returns their number.
 *   pnoeom_gemm_time runs a variant reps times on scratch operands of the key's shape
 *     (allocated and freed by the call; shapes above 8 GiB of operands are not run and
 *     give *ms = -1) and returns the mean milliseconds on hip_stream (NULL = default).
 *   pnoeom_gemm_set_table replaces the table: shapes listed use their variant, the
 *     others the built-in rule.  The tuner that writes the table is
 *     paper_1802_06738_amd/autotune.py.
 * Errors: EINVAL (bad key, variant or count), EHIP, ENOMEM. */
int pnoeom_gemm_record(int enable);
int pnoeom_gemm_recorded(long long* keys, int cap);
int pnoeom_gemm_time(void* hip_stream, const long long* key, int variant, int reps, double* ms);
int pnoeom_gemm_set_table(int n, const long long* keys, const int* variants);

/* bfloat16 GEMM with FP32 accumulation, the kernel of every BF16 contraction (ladder, W
 * slab builds, ring products): C = alpha A B^T + beta C with A [M][lda] and B [N][ldb]
 * device bfloat16 bit patterns (K contiguous; K, lda, ldb multiples of 64 with the
 * padding columns zero; 16-byte aligned), C [M][ldc] device FP32, ldc >= N.  variant:
 * 0 = chosen by shape, 1 = 128 x 128 tiles (16x16x32 MFMA), 2 = 256 x 256 tiles
 * (32x32x16 MFMA, direct-to-LDS loads; needs M, N >= 160), 3 = as 2 with the k-steps
 * rotated across the K-tile barrier, 4 / 5 = as 3 with the tiles taken M-fastest / in
 * groups of 8 tile columns (3 chooses between M-fastest and groups of 4 by shape).  Variants
 * 0 and 3 split K (partials in a library workspace, summed in a fixed order) when the
 * tiles fill the 256 compute units poorly and K is long.
 * Stream-ordered on hip_stream (NULL = default).
 * pnoeom_gemm_bf16_time times a variant on scratch operands of shape M x N x K that it
 * allocates (reps launches; *ms = mean milliseconds, -1 above 16 GiB of operands).
 * Errors: EINVAL (shape, padding, alignment, variant), EHIP, ENOMEM. */
int pnoeom_gemm_bf16(void* hip_stream, long long M, long long N, long long K, float alpha, const void* A,
                     long long lda, const void* B, long long ldb, float beta, float* C, long long ldc, int variant);
int pnoeom_gemm_bf16_time(void* hip_stream, long long M, long long N, long long K, int variant, int reps,
                          double* ms);

/* Host symmetric eigensolver used by pnoeom_build_sapno for pair-density and
 * semicanonical blocks larger than the GPU Jacobi kernel handles well (Methods: the
 * per-pair diagonalisation of the state-averaged densities), exposed for CPU tests.
 * Householder tridiagonalisation + implicit QR with Wilkinson shifts.
 *   a : host [n][n] row-major symmetric (not modified)
 *   w : host [n] eigenvalues (unordered);  v : host [n][n], column k = unit
 *       eigenvector of w[k].
 * Errors: EINVAL (n < 1 or null), ENOTCONV. */
int pnoeom_host_syev(int n, const double* a, double* w, double* v);

/* Device memory of sigma evaluations (pnoeom_apply_sigma, the Davidson): the bytes one trial
 * vector of a chunk needs for (space, precision) -- the work arrays of the non-ladder terms,
 * the ladder's packed operands and results, and in the PNO space the canonical expansion of
 * the vector and of its sigma --, the bytes available to a chunk now (free device memory plus
 * what the sigma workspaces hold, less a headroom of max(2 GiB, 3% of the device) left to
 * the caller), and the vectors per chunk that gives (at least 1; a call on more vectors runs
 * in chunks of that many).  Any output may be NULL.  Errors: EINVAL (null ctx, bad space or
 * precision), ESTATE (before pnoeom_build_df; PNO space before pnoeom_build_sapno). */
int pnoeom_sigma_memory(pnoeom_ctx* ctx, int space, int precision, long long* per_vector, long long* avail,
                        int* chunk);

/* Where pnoeom_build_sapno (and pnoeom_syev_batched) solve symmetric eigenproblems larger
 * than 128 (Methods: the per-pair diagonalisation of the state-averaged densities, whose
 * kept eigenvectors are the PNOs, and the semicanonical rotation of each kept space):
 *   backend 0 (default): on the GPU up to n = 1024 -- Householder reduction to tridiagonal
 *             form, all eigenvalues by Sturm bisection, and only the eigenvectors that the
 *             truncation keeps by inverse iteration (reorthogonalised inside clusters of
 *             close eigenvalues), back-transformed by the reflectors; larger n on the host;
 *   backend 1: on host threads (pnoeom_host_syev's algorithm), all eigenvectors.
 * Matrices up to 128 always use the GPU Jacobi kernel.  Errors: EINVAL (null ctx, bad mode). */
int pnoeom_set_eig_backend(pnoeom_ctx* ctx, int backend);

/* The batched symmetric eigensolver of pnoeom_build_sapno on caller data, on the context's
 * stream (synchronised on return).
 *   a   : device [nmat][n][n] row-major symmetric matrices, overwritten (workspace)
 *   cut : eigenvectors are required only for eigenvalues with |lambda| >= cut (0: all)
 *   ev  : device [nmat][n] eigenvalues (ascending for n > 128 on the GPU backend, unordered
 *         otherwise)
 *   vt  : device [nmat][n][n]; row k of matrix m is the unit eigenvector of ev[m][k] for
 *         every k with |ev[m][k]| >= cut (rows of the other eigenvalues may be zero)
 * n above 1024 goes to the host solver.  Caller owns all buffers.  Errors: EINVAL (null ctx
 * or pointers, nmat < 0, n < 1), ENOTCONV (host solver). */
int pnoeom_syev_batched(pnoeom_ctx* ctx, int nmat, int n, double* a, double cut, double* ev, double* vt);

/* Time spent in the last pnoeom_davidson / pnoeom_apply_sigma call, measured with
 * HIP events on the context's stream: total milliseconds; milliseconds inside the
 * particle-ladder contractions and the number of ladder GEMM launches (two per
 * sigma block: the + and - halves of the packed form); the algorithmic flop count
 * of those contractions
 * (2 * nvec * P_o * (v+^2 + v-^2), P_o = o(o+1)/2, v+- = v(v+-1)/2).  Any output
 * pointer may be NULL. */
int pnoeom_last_timing(const pnoeom_ctx* ctx, double* total_ms, double* ladder_ms, int* ladder_launches,
                       double* ladder_flops);

/* The ladder part of pnoeom_last_timing restricted to the launches of one
 * contraction precision (PNOEOM_FP64, PNOEOM_FP32 or PNOEOM_BF16): a mixed-precision
 * Davidson with FP64 refinement runs ladder launches of both kinds.
 * Errors: EINVAL (null ctx, bad precision). */
int pnoeom_last_ladder_timing(const pnoeom_ctx* ctx, int precision, double* ladder_ms, int* ladder_launches,
                              double* ladder_flops);

/* Further timed regions of the last pnoeom_davidson / pnoeom_apply_sigma /
 * pnoeom_ladder_apply call, for
 * the roofline of the bandwidth-side kernels:
 *   region 0: the Davidson inner products (Gram-Schmidt, subspace matrix, residual
 *             norms); bytes = 8 (n_a + n_b) N per sweep over n_a x n_b products of
 *             length-N vectors, flops = 2 n_a n_b N;
 *   region 1: the PNO back-transform and projection (Methods, PNO simulation):
 *             per vector and direction, bytes = 8 (ov + o^2 v^2 + len + |U|) (canonical
 *             vector, compressed vector and bases each moved once), flops =
 *             sum over pairs of (2 n_p v^2 + 2 n_p^2 v) plus 2 n_i v per occupied i;
 *   region 2: the W slab builds of the streamed ladder (factor GEMM and pack of W+/-
 *             rows); flops = 2 (na v)(nb v) naux per slab of na rows a and nb columns
 *             b >= a0, bytes = the slab block written and read (3 passes) plus the
 *             packed rows written.  The contraction with the slab rows counts as ladder
 *             time in pnoeom_last_timing / pnoeom_last_ladder_timing;
 *   region 3: the ring (particle-hole) products of sigma2, three GEMMs per sigma
 *             block of nb vectors (R^s [Dr | Xr], E_X [T_ia | T^s_ia], R DX2 with
 *             M = nb o v rows); flops = 10 nb (ov)^3, bytes = the operands and the
 *             output moved once;
 *   region 4: the PNO-space ladder of the native pairs (pnoeom_set_pno_ladder), two
 *             grouped GEMMs per vector; flops = sum over those pairs of 4 n_p^3 naux.
 * ms are HIP-event times on the context stream.  Errors: EINVAL (null ctx, bad region). */
int pnoeom_last_region_timing(const pnoeom_ctx* ctx, int region, double* ms, int* launches, double* flops,
                              double* bytes);

#ifdef __cplusplus
}
#endif
#endif /* PNOEOM_H */
