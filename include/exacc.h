/*
 * exacc.h -- C ABI of the MI355X complex spin-orbital CCSD amplitude iteration.
 *
 * The problem is the one the paper hands to its coupled-cluster module
 * (section "Molecular spinors: interface to DIRAC and ReSpect" and eq.
 * Hamiltonian): an active space of nocc occupied and nvir virtual spinors,
 * spinor energies eps (Fock matrix f = diag(eps)) and the antisymmetrised
 * two-electron integrals <pq||rs> = (pr|qs) - (ps|qr), here given in
 * density-fitted form (pq|rs) = sum_P B[P][p][q] B[P][r][s].
 *
 * One handle = one CCSD solve resident on one GPU.  Each iteration evaluates
 * the residual of Appendix A (eq. CC_general), takes the denominator
 * (Jacobi) step and a Pulay DIIS extrapolation (section "Coupled cluster
 * implementation"), all on the device.  <ab||cd> is formed tile by tile from
 * B every iteration and never stored.
 *
 * Conventions for every function:
 *   - complex numbers are interleaved (re, im) pairs of double;
 *   - spinor index p in [0, nocc+nvir): occupied first, then virtual;
 *   - the return value is a status: 0 = EXACC_OK, > 0 informational, < 0 error;
 *   - a pointer argument flagged "device" must be a HIP device address that is
 *     valid for the handle's stream; otherwise it is host memory;
 *   - calls on one handle must be serialised by the caller; distinct handles
 *     may be driven concurrently from different host threads.
 */
#ifndef EXACC_H
#define EXACC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct exacc_ccsd_s* exacc_ccsd_t;   /* opaque; owns all device memory of one solve */

enum {
  EXACC_OK = 0,
  EXACC_NOT_CONVERGED = 1,      /* iterate: max_steps reached before tol; results readable */
  EXACC_ERR_INVALID_ARG = -1,   /* bad sizes, null pointer, non-finite input, non-Hermitian B, no gap */
  EXACC_ERR_NOMEM = -2,         /* memory plan exceeds hbm_budget_bytes or a device allocation failed */
  EXACC_ERR_DEVICE = -3,        /* a HIP runtime error (text via exacc_last_error) */
  EXACC_ERR_DIVERGED = -4,      /* energy or step norm non-finite or grew 1e6-fold; handle stays readable */
  EXACC_ERR_UNSUPPORTED = -5    /* option value not implemented by this library */
};

enum { EXACC_FP64 = 0, EXACC_MIXED_FP32 = 1, EXACC_MIXED_BF16X3 = 2 };

/* Options; the keywords are the paper's input keywords (Supporting
 * Information, table of ExaCorr keywords) where one exists. */
typedef struct {
  int    precision;          /* EXACC_FP64 (default); EXACC_MIXED_FP32: FP32 contractions, then FP64;
                                EXACC_MIXED_BF16X3: as MIXED_FP32 but the particle ladder's tile
                                build and contraction, the o^3 v^3 ring contractions, the
                                density-fitted terms of the ring intermediate and the vovv.tau
                                product use split-BF16 (hi*hi + hi*lo + lo*hi) products with FP32
                                accumulation */
  int    diis_size;          /* Pulay subspace size, default 8; 0 = plain Jacobi steps */
  int    max_iter;           /* .NCYCLES, default 30 */
  double tol;                /* .TCONVERG, default 1e-9, on ||Delta||_2 over the unique amplitudes */
  double level_shift;        /* .LSHIFT, default 0: added to every virtual energy in the denominators */
  int    fp64_final_iters;   /* mixed precision: at least this many FP64 iterations at the end (default 3) */
  double mixed_switch_tol;   /* mixed precision: FP64 contractions once ||Delta|| < this (default 1e-5),
                                or once 4 low-precision iterations in a row bring no new lowest
                                ||Delta|| (the low-precision rounding floor); the DIIS subspace
                                restarts at the switch.  Converged requires FP64 iterations */
  int    inputs_on_device;   /* 0: eps and B passed to create are host pointers; 1: device pointers */
  void*  stream;             /* hipStream_t to enqueue on; NULL: the handle creates its own */
  size_t hbm_budget_bytes;   /* 0 = unlimited; create fails with EXACC_ERR_NOMEM above it */
  long   ladder_chunk_pairs; /* a<b pairs per ladder chunk (scratch size); 0 = automatic */
  int    timing;             /* 1: record per-stage HIP-event times (exacc_ccsd_stage_times) */
  int    doubles_only;       /* .CCDOUBLES: 1 = CCD (T1 held at zero, no T1 equation and no
                                t1-dependent contractions; exacc_ccsd_residual returns S1 = 0);
                                default 0 = CCSD */
  int    cc2;                /* .CC2: 1 = CC2 (T1 equation unchanged; doubles from the T1-dressed
                                <ab||ij> plus the diagonal Fock term); exclusive with doubles_only */
  int    triples_occ_block;  /* perturbative triples: occupied block size n_red of the three nested
                                block loops (<ab||ie> tiles of three blocks resident); 0 = the
                                largest that fits in free device memory (all of nocc if possible) */
  int    ladder_defect_correction; /* mixed precision, default 1: after the switch to FP64, one
                                FP64 iteration stores the particle-ladder product L(tau_ref) of its
                                amplitudes (and, where the reference arrays fit in the budget and
                                in device memory, its ring product H_ref Tq_ref and H_ref); the
                                iterations that follow form every other term in FP64 and take the
                                ladder as L(tau_ref) + L_low(tau - tau_ref), the ring as
                                H_ref Tq_ref + [H_ref dTq + dH Tq]_low and (with the ring part) the
                                vovv.tau product of C^{kb}_{ij} likewise, the bracketed products in
                                the low precision of the mode on differences formed in FP64 (their
                                rounding is relative to the differences), until ||Delta|| <= tol
                                or 4 of them bring no new lowest ||Delta||; then at least
                                fp64_final_iters full FP64 iterations.  0: full FP64 iterations
                                from the switch on */
  int    graph_residual;     /* 1: the residual computation of each iteration kind (low precision,
                                FP64, FP64 with corrected products) is recorded into a HIP graph
                                on its first iteration and replayed by one launch afterwards
                                (results bitwise those of direct launches; for small problems,
                                whose iterations are bound by per-kernel launch cost).  Ignored
                                when timing is set.  Default 0 */
  int    ladder_group_nvir;  /* nvir up to which the particle ladder forms the integral tiles of
                                all virtual rows in one product (3 kernel launches per
                                iteration instead of about 2 nvir; v^4 naux complex
                                multiply-adds instead of about v^4 naux / 4, and v^4 complex
                                elements of scratch); requires the whole pair range in one
                                ladder chunk (ladder_chunk_pairs 0 or >= P_v).  Default 64;
                                0: per-row tiles at every size */
} exacc_ccsd_opts;

/* Fill *o with the defaults listed above. */
void exacc_ccsd_default_opts(exacc_ccsd_opts* o);

/* Device bytes create() will allocate for this problem (the a-priori memory
 * footprint the paper reports in "Coupled cluster implementation").
 * opts may be NULL (defaults).  Returns 0 for invalid sizes.  In the mixed
 * modes the estimate includes the reference arrays of the ring correction
 * (ladder_defect_correction) when they fit in hbm_budget_bytes (or no budget is
 * set); create drops them when the plan with them exceeds the device memory, and
 * the estimate then overstates the footprint by that part. */
size_t exacc_ccsd_memory_estimate(int nocc, int nvir, int naux, const exacc_ccsd_opts* opts);

/* Validate the inputs, copy them to the device, build the stored integral
 * classes (oooo, ooov, oovv, vovo and vovv packed over c<d) and set the
 * amplitudes to zero, so that the first iterate() step gives the MP2
 * amplitudes.
 *   eps : [nocc+nvir] doubles, occupied first (host or device, see opts)
 *   B   : [naux][n][n] complex, B[P][p][q] = conj(B[P][q][p]), n = nocc+nvir
 * Both are copied; the caller may free them on return.  On any error *out is
 * NULL and nothing stays allocated.  Errors: INVALID_ARG (nocc, nvir or naux
 * < 1, null pointers, non-finite entries, |B - B^H| > 1e-12 max|B|,
 * min(eps_vir) - max(eps_occ) <= 1e-8), NOMEM, DEVICE, UNSUPPORTED. */
int exacc_ccsd_create(exacc_ccsd_t* out, int nocc, int nvir, int naux,
                      const double* eps, const double* B, const exacc_ccsd_opts* opts);

/* Run up to max_steps iterations (eq. CC_general residual, Jacobi step, DIIS);
 * stop early once ||Delta||_2 <= tol.  Outputs (any may be NULL): steps done,
 * ||Delta||_2 of the last step, converged flag.  Returns OK when converged,
 * NOT_CONVERGED when max_steps ran out, DIVERGED, DEVICE. */
int exacc_ccsd_iterate(exacc_ccsd_t h, int max_steps, int* steps_done,
                       double* residual, int* converged);

/* FP64 correlation energy of the current amplitudes,
 * E = sum f_ia t_i^a + 1/4 sum <ij||ab> tau_ij^ab (complex). */
int exacc_ccsd_energy(exacc_ccsd_t h, double* e_re, double* e_im);

/* Copy the current amplitudes out: t1 [nocc][nvir] complex; t2
 * [nocc][nocc][nvir][nvir] complex, full antisymmetric.  Either may be NULL.
 * ptr_on_device selects device (1) or host (0) destinations. */
int exacc_ccsd_get_amplitudes(exacc_ccsd_t h, double* t1, double* t2, int ptr_on_device);

/* Replace the amplitudes (same layouts as get_amplitudes; t2 must be
 * antisymmetric: only the i<j, a<b entries are read).  Clears the DIIS
 * history.  Used for warm restarts and to evaluate the residual at given
 * amplitudes. */
int exacc_ccsd_set_amplitudes(exacc_ccsd_t h, const double* t1, const double* t2, int ptr_on_device);

/* The residual of eq. CC_general at the current amplitudes, without updating
 * them: s1 [nocc][nvir], s2 [nocc][nocc][nvir][nvir] (full, antisymmetric),
 * both including the diagonal Fock part.  Either may be NULL.  Contractions
 * run in the precision of the current phase (see exacc_ccsd_phase); the sum
 * with the inhomogeneous term <ab||ij> and the diagonal part is formed in
 * FP64. */
int exacc_ccsd_residual(exacc_ccsd_t h, double* s1, double* s2, int ptr_on_device);

/* Perturbative triples corrections at the current amplitudes (App. C, working
 * equations for perturbative triples; the paper's NOTRIPLES keyword turns
 * them off, here they are computed only on request).  *e_plus_t = E(+T), the
 * fourth-order term; *e_paren_t = E((T)) = E(+T) plus the singles-triples
 * term; *e_minus_t = E(-T) = E(+T) plus the Y-intermediate term (any pointer
 * may be NULL).  Complex spinors: W is formed with the excitation elements
 * <ab||ie>, <am||ij> (the complex conjugates of the printed ones) and the
 * singles-triples term of E((T)) has the standard CCSD(T) sign.
 * FP64; needs the FP64 phase (INVALID_ARG while a mixed-precision handle is
 * still in its low-precision phase).  The occupied space is split into blocks
 * of n_red = opts.triples_occ_block spinors (section "Coupled cluster
 * implementation": three nested loops over occupied subspaces, unique block
 * triples only); the <ab||ie> tiles of the three current blocks (3 n_red nvir^3
 * complex values, nocc nvir^3 when one block holds all) and at least one W row
 * (nvir^3) are allocated and freed inside the call (NOMEM if that does not
 * fit).  Zero for nocc < 3 or nvir < 3.  The amplitudes and the iteration
 * state are not changed. */
int exacc_ccsd_triples(exacc_ccsd_t h, double* e_plus_t, double* e_paren_t, double* e_minus_t);

/* Lambda (left-hand) equations of CCSD at the current amplitudes (App. D,
 * working equations for the CCSD lambda equations), FP64: lambda solves
 * dL/dt = 0 for the Lagrangian L = <0|(1 + Lambda) e^-T H e^T|0>.  Runs up to
 * max_steps Jacobi + DIIS steps on lambda (the amplitude denominators and DIIS
 * size; lambda starts at zero on the handle's first Lambda call); reports as
 * exacc_ccsd_iterate, converged when ||Delta lambda||_2 <= opts.tol.  The
 * amplitudes should be converged first; they are not changed.  The Lambda
 * iteration and the amplitude iteration share the DIIS storage: switching
 * from one to the other starts a fresh DIIS history.  Needs the FP64 phase and
 * a CCSD handle (INVALID_ARG for CCD or CC2 handles, or while a mixed handle is
 * in its low-precision phase).  The first call allocates the Lambda buffers
 * (about 2 nocc^2 nvir^2 + nvir^2 naux + 3 nocc^3 nvir complex values; NOMEM if
 * they do not fit); they stay with the handle until destroy. */
int exacc_ccsd_lambda_iterate(exacc_ccsd_t h, int max_steps, int* steps_done,
                              double* residual, int* converged);

/* The Lambda residual at the current lambda, without updating it: r1
 * [nocc][nvir], r2 [nocc][nocc][nvir][nvir] (full, antisymmetric), including
 * the diagonal Fock part (r = D lambda + ..., D as for the amplitudes).
 * Either may be NULL.  Same conditions as exacc_ccsd_lambda_iterate. */
int exacc_ccsd_lambda_residual(exacc_ccsd_t h, double* r1, double* r2, int ptr_on_device);

/* Copy lambda out / replace it, layouts as for the amplitudes: l1[i][a] =
 * lambda_a^i, l2[i][j][a][b] = lambda_ab^ij (antisymmetric; set reads only the
 * i<j, a<b entries; a NULL argument to set means zero).  Setting clears the
 * Lambda DIIS history. */
int exacc_ccsd_get_lambda(exacc_ccsd_t h, double* l1, double* l2, int ptr_on_device);
int exacc_ccsd_set_lambda(exacc_ccsd_t h, const double* l1, const double* l2, int ptr_on_device);

/* Correlation part of the one-body density of the CC Lagrangian at the
 * current t and lambda (App. E, working equations for the Lagrange one-body
 * density matrix): gamma [n][n] complex, gamma[p][q] =
 * <0|(1 + Lambda) e^-T {q+ p} e^T|0>, blocks [i][j], [i][a] = lambda_a^i,
 * [a][i], [a][b] with occupied spinors first.  The printed occupied block is
 * the transpose of this element; the matrix is not symmetrised (its Hermitian
 * part is the density used for properties).  Adding the identity on the
 * occupied block gives the full density (trace = nocc).  Same conditions as
 * exacc_ccsd_lambda_iterate. */
int exacc_ccsd_density(exacc_ccsd_t h, double* gamma, int ptr_on_device);

/* Density-fitting factors from AO three-index integrals (the step before the
 * CC iteration; the paper's Introduction names density fitting for the
 * integral tensor, its Performance section the cost of the AO->MO
 * transformation): with (mu nu|Q) = J[Q][mu][nu] (complex [naux][nao][nao]),
 * the fitting metric V[Q][R] = (Q|R) (real symmetric positive definite
 * [naux][naux]) and spinor coefficients C[mu][p] (complex [nao][nspinor]),
 *   B[P][p][q] = sum_Q [V^-1/2]_PQ sum_{mu nu} conj(C[mu][p]) J[Q][mu][nu] C[nu][q]
 * (complex [naux][nspinor][nspinor]; Hermitian in pq when J is Hermitian in
 * mu nu), so that sum_P B[P][p][q] B[P][r][s] is the fitted (pq|rs): the input
 * of exacc_ccsd_create.  V^-1/2 comes from the coupled Newton-Schulz iteration
 * (matrix products only) on V scaled by its largest absolute row sum;
 * *ns_iterations (may be NULL) receives its step count.  Pointers are device
 * pointers (ptrs_on_device = 1) or host pointers (0); the caller owns them.
 * stream: hipStream_t or NULL (the call then uses a stream of its own).
 * Temporary device memory of 6 naux^2 + naux nspinor (nao + nspinor) complex
 * values (plus copies of the inputs for host pointers) is allocated and freed
 * inside the call (NOMEM if it does not fit).  INVALID_ARG for sizes outside
 * 1 <= nspinor <= nao, naux >= 1, null pointers, or a metric on which the
 * iteration does not converge (not positive definite, or condition number
 * beyond about 1e14). */
int exacc_df_factors(int nao, int nspinor, int naux, const double* C, const double* J,
                     const double* V, double* B, int ptrs_on_device, void* stream,
                     int* ns_iterations);

/* Bytes of the static device array that holds the temporaries of
 * exacc_df_factors_noalloc: one such array per GPU the library runs on, held
 * from library load to process end. */
#define EXACC_DF_SCRATCH_BYTES ((size_t)256 << 20)

/* exacc_df_factors without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, serving loops that must not call
 * hipMalloc, harnesses that forbid it.  Same operation, result and errors as
 * exacc_df_factors with ptrs_on_device = 1: C, J, V and B are device pointers
 * on the calling thread's current device, owned by the caller.  stream:
 * hipStream_t, or NULL for the null stream.  Every temporary lives in the
 * library's static array of EXACC_DF_SCRATCH_BYTES on that device; the call
 * makes no device allocation and frees nothing.  Limit: the six naux x naux
 * Newton-Schulz matrices plus one spinor row of the transform intermediates,
 * 16 (6 naux^2 + naux (nao + nspinor)) bytes plus about 64 KiB, must fit in
 * the array (naux up to about 1670); larger sizes return EXACC_ERR_NOMEM
 * before any device work.  The transform runs over slices of spinor rows as
 * wide as the array allows.  Calls on one GPU share the array and it keeps the
 * last call's contents (nothing in it needs to start at zero): calls that
 * overlap in time on one GPU, from different threads or streams, race and
 * must be serialised by the caller. */
int exacc_df_factors_noalloc(int nao, int nspinor, int naux, const double* C, const double* J,
                             const double* V, double* B, void* stream, int* ns_iterations);

/* Accumulated device time in ms of each stage since create (or the last
 * reset), measured with HIP events on the handle's stream; requires
 * opts.timing = 1.  names[k] (static strings) and ms[k] for k < *count.
 * Pass reset = 1 to zero the counters after reading. */
int exacc_ccsd_stage_times(exacc_ccsd_t h, const char** names, double* ms, int* count, int reset);

/* Precision of the contractions the next iterate() step will use: 1 = low
 * precision (the FP32 / BF16x3 phase of a mixed mode), 2 = FP64 with the
 * defect-corrected low-precision particle ladder (see
 * ladder_defect_correction), 0 = FP64.  *fp64_iters (may be NULL) receives the
 * number of full FP64 iterations since the last phase change. */
int exacc_ccsd_phase(exacc_ccsd_t h, int* fp32, int* fp64_iters);

/* Algorithmic flop count (real flops, 8 per complex multiply-add) of one
 * iteration's particle-particle ladder: the tile build of the blocks of
 * <ab||cd> on and above the diagonal of the Hermitian pair matrix (for each
 * virtual a, (ac|bd) over c, d >= a and b > a: naux * sum_{m=1}^{nvir}
 * m^2 (m - 1) complex multiply-adds, about naux nvir^4 / 4) plus the
 * contraction P_o*P_v^2 complex multiply-adds, P_o = nocc(nocc-1)/2,
 * P_v = nvir(nvir-1)/2. */
double exacc_ladder_flops(int nocc, int nvir, int naux);

/* Release every device buffer of the handle.  NULL-safe. */
int exacc_ccsd_destroy(exacc_ccsd_t h);

/* Text for a status code. */
const char* exacc_status_string(int status);

/* Text of the last error raised on the calling thread (empty if none). */
const char* exacc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* EXACC_H */
