/*
 * libmlcc -- multilevel CC2 / CCSD (MLCC2, MLCCSD with CCS/CCSD levels) on
 * Cholesky-decomposed electron-repulsion integrals, for AMD MI355X (gfx950).
 *
 * Method: Folkestad, Kjonstad, Goletto, Koch, "Multilevel CC2 and CCSD in
 * reduced orbital spaces" (arXiv 2006.05226).  Section numbers below refer to
 * that paper: Sec. 2.1 (the MLCC2 and MLCCSD models, their ground-state
 * equations and Jacobians) and Appendix A (the equations in terms of the
 * Cholesky vectors: X1 basis, Fock matrix, energy, Omega vectors, Jacobian
 * transformations).
 *
 * ---------------------------------------------------------------------------
 * Conventions shared by every call
 * ---------------------------------------------------------------------------
 * Orbitals.  n = n_occ + n_vir molecular orbitals, occupied first.  Inside each
 *   block the active orbitals come first: active occupied 0..n_occ_act-1,
 *   active virtual n_occ..n_occ+n_vir_act-1.  The active-active Fock blocks are
 *   diagonal (semicanonical basis, Sec. 2.1); the library takes the MO Fock
 *   matrix F to be diag(eps), or the matrix given in mlcc_problem_desc.fock,
 *   and the one-electron integrals to be h = F - G(D_HF), so that the
 *   reference is the Hartree-Fock state of the Hamiltonian defined by (h, L).
 * Cholesky vectors.  L[J][p][q], row major, J < n_chol, L[J][p][q] == L[J][q][p],
 *   g_pqrs = sum_J L[J][p][q] L[J][r][s] (Appendix A).
 * Singles.  t1 / omega1 / c1 / sigma1 are [n_vir][n_occ] (all orbitals).
 * Doubles.  Active space only, M = n_occ_act * n_vir_act pairs with pair index
 *   ai = a * n_occ_act + i.  A doubles array is the full symmetric M x M matrix
 *   x[ai][bj] == x[bj][ai] with X2 = 1/2 sum x_aibj E_ai E_bj, projected with
 *   the biorthonormal basis <mu_aibj|E_ck E_dl|HF> = d(ai,ck)d(bj,dl) +
 *   d(ai,dl)d(bj,ck).
 * Excitation vectors.  dim = n_vir*n_occ (+ M*M for MLCC2/MLCCSD in the full
 *   space): singles block followed by the doubles block.  Several vectors are
 *   stored back to back, [n_vec][dim].
 * Pointers.  Every array argument may be host memory or device memory on the
 *   context's GPU; the library tells them apart with hipPointerGetAttributes
 *   (with MLCC_INPUT_ON_DEVICE a problem descriptor's inputs must be device
 *   memory).
 *   The caller owns every pointer it passes; inputs are copied before a call
 *   returns, outputs are written only into the caller's buffers and only when
 *   the call returns MLCC_OK (MLCC_E_NOCONV also fills best-so-far values).
 * Streams.  All device work of a context is ordered on the stream given at
 *   context creation; every call except mlcc_submit/mlcc_poll has completed
 *   its device work when it returns.  Device memory passed in must be ready
 *   when the call is made: work that produces it on another stream (a
 *   library's own stream is non-blocking) must have completed, or been made
 *   to precede the call, by the caller.
 * Threading.  One host thread at a time per context (and its problems);
 *   mlcc_submit / mlcc_poll are thread safe.
 * Units.  Hartree.
 * Errors.  No exception or abort crosses this interface; a negative status is
 *   returned and mlcc_last_error() describes it.
 */
#ifndef MLCC_H
#define MLCC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mlcc_status;
#define MLCC_OK 0
#define MLCC_PENDING 1       /* mlcc_poll: request not finished yet */
#define MLCC_E_ARG (-1)      /* invalid argument (dimensions, NULL, flags) */
#define MLCC_E_OOM (-2)      /* device memory or the HBM budget exhausted */
#define MLCC_E_NOCONV (-3)   /* iteration limit reached */
#define MLCC_E_NUMERIC (-4)  /* NaN/Inf in inputs or iterates */
#define MLCC_E_DEVICE (-5)   /* HIP runtime error */
#define MLCC_E_BUSY (-6)     /* server queue full */
#define MLCC_E_STATE (-7)    /* call out of order (e.g. no amplitudes yet) */

/* Models (Sec. 2.1). */
#define MLCC_CCS 0     /* X = X1 */
#define MLCC_MLCC2 1   /* X = X1 + S2, S2 in the active space, perturbative */
#define MLCC_MLCCSD 2  /* CCS/CCSD: X = X1 + T2, T2 in the active space */
/* CCS/CC2/CCSD: X = X1 + S2 + T2 with S2 in the active space and T2 in the
 * CCSD space (n_occ_ccsd, n_vir_ccsd prefixes of the active space), Sec. 2.1.
 * The paper gives the cluster operator but no equations for this model; the
 * library's reading: the doubles x = S2 + T2 span the active space; the
 * singles and the doubles projections with all four indices in the CCSD
 * space are those of exp(-X) H exp(X) (CCSD level, coupled to every
 * amplitude of the active space), the other doubles projections keep the
 * CC2 form g~_aibj + eps_aibj x_aibj.  Doubles arrays, excitation vectors
 * and the ground-state and Davidson drivers are those of MLCC_MLCCSD over
 * the active space.  n_occ_ccsd = n_occ_act and n_vir_ccsd = n_vir_act give
 * MLCC_MLCCSD; an empty CCSD space gives MLCC2 with iterated doubles. */
#define MLCC_MLCCSD3 3

/* Arithmetic of the Cholesky-index contractions (the MFMA GEMMs).  Amplitude
 * and denominator updates, DIIS, Davidson and energies are FP64 always. */
#define MLCC_FP64 0
#define MLCC_FP32 1
/* FP32 storage; the Cholesky-index contractions whose operands are
 * contiguous along the reduction index run on the BF16 matrix cores as
 * hi*hi + hi*lo + lo*hi (x = hi + lo, hi = bf16(x), lo = bf16(x - hi); FP32
 * accumulation), the others on FP32 MFMA; FP64 elsewhere as for MLCC_FP32. */
#define MLCC_BF16X3 2
/* As MLCC_BF16X3, except that the contractions named in the context's BF16
 * map (mlcc_bf16_map, include/mlcc_engine.h) run one BF16 product of
 * operands rounded to BF16 (FP32 accumulation) instead of three.  The
 * built-in map holds the contractions whose plain BF16 products keep the
 * energies within 1e-6 Eh and the excitation energies within 1e-5 eV of FP64
 * on the 40/400/1200 MLCC2 and 60/600/2000 MLCCSD workloads. */
#define MLCC_BF16 3

typedef struct mlcc_context mlcc_context;
typedef struct mlcc_problem mlcc_problem;
typedef struct mlcc_server mlcc_server;

typedef struct {
  int32_t n_occ, n_vir, n_chol;   /* N_o, N_v, N_J */
  int32_t n_occ_act, n_vir_act;   /* active prefixes (ignored for MLCC_CCS) */
  int32_t model;                  /* MLCC_CCS | MLCC_MLCC2 | MLCC_MLCCSD | MLCC_MLCCSD3 */
  int32_t precision;              /* MLCC_FP64 | MLCC_FP32 | MLCC_BF16X3 | MLCC_BF16 */
  const double *L;                /* [n_chol][n][n], symmetric in the last two */
  const double *eps;              /* [n] orbital energies in the order above */
  uint32_t flags;                 /* MLCC_SYNTH_L | MLCC_INPUT_ON_DEVICE |
                                     MLCC_DETERMINISTIC, or 0 */
  uint64_t seed;                  /* seed of MLCC_SYNTH_L */
  const double *fock;             /* [n][n] symmetric Fock matrix (host or device), or
                                     NULL for diag(eps).  For a semicanonical basis
                                     (Sec. 2.2: the Fock matrix diagonal within the
                                     active and within the inactive orbitals, as
                                     mlcc_cnto returns it); eps must be its diagonal,
                                     which the denominators use.  The occupied-virtual
                                     block must vanish (a Hartree-Fock reference). */
  int32_t n_occ_ccsd, n_vir_ccsd; /* MLCC_MLCCSD3: the CCSD space, prefixes of the
                                     active space (0 <= n_occ_ccsd <= n_occ_act,
                                     0 <= n_vir_ccsd <= n_vir_act); ignored by the
                                     other models */
} mlcc_problem_desc;

/* flags: L is not read; the library draws synthetic Cholesky vectors on the
 * device from seed: L[J][p][q] = L[J][q][p] = sigma exp(-J/10) z, sigma =
 * 0.5 / sqrt(n_occ n_vir), z standard normal from the Philox4x32-10
 * counter-based generator (Salmon et al., SC'11) with key (seed lo, seed hi)
 * and counter (p*n + q, J, 0, 0), Box-Muller on its first two words.  For
 * benchmark and serving workloads too large to stage from the host; eps is
 * still read. */
#define MLCC_SYNTH_L 1u
/* flags: the caller states that L (unless MLCC_SYNTH_L), eps and fock (when
 * not NULL) are device memory; the library checks each pointer and fails with
 * MLCC_E_ARG for one that is not.  Without the flag each of them may be host
 * or device memory (the library classifies them itself).  The server copies
 * a submitted request's inputs in either case. */
#define MLCC_INPUT_ON_DEVICE 2u
/* flags: bitwise-reproducible results.  Residuals, transformations, ground
 * states, Davidson roots and served results of a problem run on this
 * library's kernels only, and every reduction among them has a fixed order
 * (split-K partial sums are added by a separate pass in split order; no
 * floating-point atomics), so for equal inputs, model, precision, context
 * settings and device the results are bitwise equal, with or without this
 * flag; it is accepted so that a caller can state the requirement.  Not
 * covered: mlcc_cnto's eigenvectors, computed by rocSOLVER. */
#define MLCC_DETERMINISTIC 4u

typedef struct {
  double tol;             /* ground state: ||Omega||_2; Davidson: residual norm */
  int32_t max_iter;       /* iteration limit */
  int32_t diis_dim;       /* DIIS history length (ground state), 0 -> 8 */
  int32_t max_subspace;   /* Davidson subspace before collapse, 0 -> 20*n_roots */
  int32_t n_guess;        /* Davidson start vectors, 0 -> n_roots + 2 */
  int32_t effective;      /* MLCC2 Davidson on the singles space with the
                             omega-dependent effective Jacobian (Sec. 2.1: the
                             doubles-doubles block is diagonal) */
} mlcc_solver_opts;

typedef struct {
  int32_t iterations;
  int32_t converged;      /* 1 if every quantity met opts.tol */
  double residual;        /* final ||Omega|| or max root residual */
  double energy;          /* correlation energy at the final amplitudes */
  int32_t complex_roots;  /* number of returned roots that had a complex pair */
  int32_t transforms;     /* Jacobian transformations performed */
} mlcc_info;

/* ---- context -------------------------------------------------------------
 * device: HIP ordinal.  hip_stream: a hipStream_t of that device (NULL = the
 * library creates its own).  hbm_budget: bytes the context may allocate on
 * the device (0 = no limit beyond the device's free memory). */
mlcc_status mlcc_context_create(int device, void *hip_stream, uint64_t hbm_budget,
                                mlcc_context **ctx);
/* Drops the caller's handle.  Problems and servers created on the context
 * keep it alive: its device memory, stream and pinned buffers are freed when
 * the last of them is destroyed, so the handles may be destroyed in any
 * order; no call may be made on ctx itself after this one. */
mlcc_status mlcc_context_destroy(mlcc_context *ctx);
/* Message of the last error on this context (or of the last failed create when
 * ctx is NULL).  Valid until the next call on the context. */
const char *mlcc_last_error(mlcc_context *ctx);
/* Device bytes currently allocated by the context. */
uint64_t mlcc_context_bytes(mlcc_context *ctx);

/* ---- problems --------------------------------------------------------------
 * Copies L and eps to the device, forms h (see Conventions) and prepares the
 * packed blocks of L the model needs.  Errors: MLCC_E_ARG (dimensions < 1,
 * active > total, NULL pointers), MLCC_E_NUMERIC (NaN/Inf in eps),
 * MLCC_E_OOM. */
mlcc_status mlcc_problem_create(mlcc_context *ctx, const mlcc_problem_desc *desc,
                                mlcc_problem **prob);
mlcc_status mlcc_problem_destroy(mlcc_problem *prob);
/* dims[0..7] = n_occ, n_vir, n_chol, n_occ_act, n_vir_act, M, singles dim,
 * full-space excitation dim. */
mlcc_status mlcc_problem_dims(const mlcc_problem *prob, int64_t dims[8]);

/* Set the amplitudes at which mlcc_residual / mlcc_jacobian_transform are
 * evaluated.  t1 [n_vir][n_occ]; x2 [M][M] symmetric: the MLCCSD t2, or an
 * independent MLCC2 s2 (NULL for MLCC2 = use the analytic s2 of t1). */
mlcc_status mlcc_set_amplitudes(mlcc_problem *prob, const double *t1, const double *x2);

/* Omega vector (Sec. 2.1 eqs. mlcc2_1/2, mlccsd_1/2; Appendix A.1) at the
 * current amplitudes.  omega1 [n_vir][n_occ]; omega2 [M][M] or NULL; x2_out
 * [M][M] or NULL receives the doubles used (analytic s2 for MLCC2 when no s2
 * was set); e_corr (or NULL) receives the correlation energy (Appendix A.1).
 * MLCC_E_STATE if no amplitudes were set. */
mlcc_status mlcc_residual(mlcc_problem *prob, double *omega1, double *omega2,
                          double *x2_out, double *e_corr);

/* Ground state: DIIS-accelerated quasi-Newton on Omega = 0 (Sec. 2.1); MLCC2
 * re-solves s2 analytically each iteration.  Starts from the current t1 (zero
 * if none was set) and leaves the converged amplitudes set.  t1_out may be
 * NULL.  MLCC_E_NOCONV after opts.max_iter iterations (outputs filled). */
mlcc_status mlcc_ground_state(mlcc_problem *prob, const mlcc_solver_opts *opts,
                              double *t1_out, double *e_corr, mlcc_info *info);

/* sigma = A c for n_vec vectors [n_vec][dim] (full space, Appendix A.2) at the
 * current amplitudes.  The transformation is the derivative of the Omega
 * vector; for MLCC2 the doubles-doubles block is eps_aibj (Sec. 2.1).  The
 * doubles block of each c must be symmetric (the doubles convention above);
 * the result for a nonsymmetric block is unspecified. */
mlcc_status mlcc_jacobian_transform(mlcc_problem *prob, int32_t n_vec, const double *c,
                                    double *sigma);

/* MLCC2 effective singles transformation at frequency omega:
 * s1 = A11 c1 + A12 (omega - eps)^-1 A21 c1   (A22 is diagonal, Sec. 2.1).
 * c1, s1: [n_vec][n_vir*n_occ]. */
mlcc_status mlcc_jacobian_transform_eff(mlcc_problem *prob, double omega, int32_t n_vec,
                                        const double *c1, double *s1);

/* Lowest n_roots excitation energies (eigenvalues of the Jacobian, Sec. 2.1)
 * by a nonsymmetric Davidson method at the current amplitudes.  omega
 * [n_roots]; r1 [n_roots][n_vir*n_occ] (singles part of the unit-norm right
 * eigenvectors) or NULL. */
mlcc_status mlcc_davidson_solve(mlcc_problem *prob, int32_t n_roots,
                                const mlcc_solver_opts *opts, double *omega, double *r1,
                                mlcc_info *info);

/* ---- serving: continuous batching of excitation solves ---------------------
 * A server owns a scheduler thread on the context's device.  Requests are
 * admitted when their estimated HBM footprint fits in the budget left and a
 * slot is free; admitted requests advance together, one solver step each per
 * scheduler round, so the work of requests of different sizes overlaps on the
 * GPU.  Each request runs ground state then Davidson. */
typedef struct {
  int32_t max_slots;        /* requests on the device at once (0 -> 8) */
  int32_t max_queue;        /* waiting requests before MLCC_E_BUSY (0 -> 1024) */
  uint64_t hbm_budget;      /* bytes for admitted requests (0 -> the context's
                               budget, else 90% of the device memory that is
                               free or held idle by the context) */
  uint64_t host_budget;     /* host bytes that the input copies of waiting (and
                               admitted, until staged on the device) requests may
                               hold (0 -> a quarter of the host's physical memory) */
} mlcc_server_opts;

typedef struct {
  mlcc_status status;       /* MLCC_OK, MLCC_E_NOCONV, ... of the finished solve */
  int32_t n_roots;
  double omega[16];         /* first min(n_roots, 16) excitation energies */
  double e_corr;
  double t_submit, t_admit, t_done;  /* seconds on the server's clock */
  int32_t gs_iterations, es_iterations;
} mlcc_result;

mlcc_status mlcc_server_create(mlcc_context *ctx, const mlcc_server_opts *opts,
                               mlcc_server **srv);
/* Drains admitted work, cancels waiting requests, joins the thread. */
mlcc_status mlcc_server_destroy(mlcc_server *srv);
/* Copies the request's inputs (host or device) and queues it.  MLCC_E_BUSY if
 * the queue is full or its input copies would pass the host budget (try
 * again later); MLCC_E_OOM if its footprint exceeds the server's HBM budget
 * or its inputs alone the host budget (it could never be admitted);
 * MLCC_E_ARG for invalid descriptors.  The host copy of the Cholesky vectors
 * is dropped as soon as the admitted request has staged them on the device;
 * requests with MLCC_SYNTH_L hold none.  A request whose lane finds device
 * memory exhausted first frees the idle and cached blocks of every lane of
 * the server, then waits up to about a minute for other requests to return
 * memory; only then does its result carry MLCC_E_OOM. */
mlcc_status mlcc_submit(mlcc_server *srv, const mlcc_problem_desc *desc, int32_t n_roots,
                        const mlcc_solver_opts *gs_opts, const mlcc_solver_opts *es_opts,
                        uint64_t *ticket);
/* MLCC_PENDING until the request is done, then MLCC_OK and *out filled (the
 * ticket is released).  MLCC_E_ARG for an unknown ticket. */
mlcc_status mlcc_poll(mlcc_server *srv, uint64_t ticket, mlcc_result *out);
/* Estimated device bytes of one request (admission uses this). */
uint64_t mlcc_request_footprint(const mlcc_problem_desc *desc, int32_t n_roots,
                                const mlcc_solver_opts *es_opts);

/* ---- orbital selection ------------------------------------------------------
 * Correlated natural transition orbitals from CCS excitation vectors (Sec. 2.2:
 * eqs. M, N, approx_double_1, approx_double_2, select_CNTOs).  prob: a problem
 * in the canonical (or semicanonical) basis of the full space; its L, Fock
 * matrix and precision are used, whatever its model.  R [n_states][n_vir][n_occ]
 * and omega [n_states]: excitation vectors and energies (for instance the r1 and
 * omega of mlcc_davidson_solve on an MLCC_CCS problem); host or device.
 * For each state the approximate doubles R_aibj = -gbar_aibj / ((1 +
 * d_ai,bj)(e_a + e_b - e_i - e_j - omega)) are built over the full space;
 * M (n_occ x n_occ) and N (n_vir x n_vir) of eqs. M and N are summed over the
 * states.  The eigenvectors of the n_occ_act largest eigenvalues of M span the
 * active occupied space, those of the n_vir_act largest of N the active
 * virtual space (eq. select_CNTOs gives n_vir_act = n_vir n_occ_act / n_occ when
 * the caller wants the paper's rule).  The active and inactive blocks are
 * then made semicanonical: the Fock matrix diagonal within each, energies
 * ascending.
 * Outputs, each optional (NULL to skip):
 *   m_eig [n_occ], n_eig [n_vir]: eigenvalues of M and N, descending (host);
 *   C [n][n]: the rotation (row major; column p is new orbital p in the order
 *     active occupied, inactive occupied, active virtual, inactive virtual;
 *     block diagonal; in each column the entry of largest magnitude, the first
 *     of equals, is positive) (host);
 *   eps_out [n] and fock_out [n][n]: the Fock matrix in the new basis (host);
 *   L_out [n_chol][n][n]: C^T L C in FP64 (host or device).
 * (L_out, eps_out, fock_out) are the inputs of a multilevel problem on the new
 * orbitals with n_occ_act / n_vir_act active (mlcc_problem_desc.fock).
 * Device scratch: (n_vir n_occ)^2 elements of the problem's operand type, plus
 * 3 n_chol n_vir n_occ, plus 2 n_chol n^2 when L_out is requested.
 * MLCC_E_ARG for bad sizes or NULL R / omega; MLCC_E_OOM if the scratch does
 * not fit; MLCC_E_NUMERIC if an eigensolver fails. */
mlcc_status mlcc_cnto(mlcc_problem *prob, int32_t n_states, const double *R, const double *omega,
                      int32_t n_occ_act, int32_t n_vir_act, double *m_eig, double *n_eig,
                      double *C, double *eps_out, double *fock_out, double *L_out);

/* ---- Cholesky vectors in the MO basis (Sec. 2.4) -----------------------------
 * The two-step Cholesky decomposition of AO electron-repulsion integrals,
 * which builds the MO Cholesky vectors without storing AO ones.  The
 * integrals are a matrix over packed AO pairs: G[ab][cd] = (ab|cd) for a >= b,
 * c >= d, pair index a (a + 1) / 2 + b, npair = n_ao (n_ao + 1) / 2, row
 * major, symmetric positive semidefinite (host or device memory; it stands in
 * for an AO integral engine, which this library does not include).
 *
 * First step, the Cholesky basis: pivoted Cholesky decomposition of G.  The
 * updated diagonal D_ab = (ab|ab) - sum_J (L^J_ab)^2 is screened as
 * D~_ab = nu_a D_ab nu_b (eq. cd_screening) with nu [n_ao] (host or device;
 * e.g. nu_a = max_p (C^a_ap)^2 over the active MOs, eq. mo_screening), or not
 * screened when nu is NULL.  The pair with the largest D~ (the lowest pair
 * index among equals) is the next pivot; the decomposition stops when
 * max D~ < tau or after max_vectors pivots.
 * Outputs: pivots [max_vectors] (host; pair indices in selection order),
 * *n_vectors, and QinvT (host or device, NULL to skip): its first n_vectors^2
 * entries, row stride n_vectors, hold Q^-T with S = Q Q^T the Cholesky
 * factorization of S_KL = (K|L) over the pivots in selection order.
 * MLCC_E_ARG for bad sizes or a non-positive tau; MLCC_E_NUMERIC for a
 * non-finite diagonal, a matrix that is not positive semidefinite, or a
 * singular S. */
mlcc_status mlcc_cholesky_basis(mlcc_context *ctx, int32_t n_ao, const double *G, const double *nu,
                                double tau, int32_t max_vectors, int32_t *pivots,
                                int32_t *n_vectors, double *QinvT);

/* Second step, Algorithm 1 (Sec. 2.4): the MO Cholesky vectors
 *   L^J_pq = sum_K X_pqK [Q^-T]_KJ,  X_pqK = sum_ab C_ap C_bq (ab|K),
 * built for batches of p_batch MO indices p at a time (0: as many as 2 GB of
 * scratch allows), the integrals (ab|K) taken again from G at the pivots for
 * each batch.  G as for mlcc_cholesky_basis; pivots [n_vec] (host) and QinvT
 * [n_vec][n_vec] (host or device) as it returns them; C [n_ao][n_mo] MO
 * coefficients (host or device).  L_out [n_vec][n_mo][n_mo] FP64 (host or
 * device): the n_chol x n x n input of mlcc_problem_desc.  precision: the
 * arithmetic of the three contractions (MLCC_FP64, MLCC_FP32, MLCC_BF16X3).
 * MLCC_E_ARG for bad sizes, NULL pointers or pivots outside the pair range. */
mlcc_status mlcc_mo_cholesky(mlcc_context *ctx, int32_t precision, int32_t n_ao, int32_t n_mo,
                             const double *G, int32_t n_vec, const int32_t *pivots,
                             const double *QinvT, const double *C, int32_t p_batch,
                             double *L_out);

#ifdef __cplusplus
}
#endif

#endif /* MLCC_H */
