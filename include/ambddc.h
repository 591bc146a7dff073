/*
 * ambddc.h -- C ABI of the MI355X Adaptive-Multilevel BDDC library.
 *
 * Adaptive-Multilevel BDDC (Sousedik, Sistek, Mandel) for symmetric positive
 * definite Q1 finite-element systems (3D Poisson, 1 DOF per node; linear
 * elasticity, 3 DOF per node).  The library computes, on one GPU:
 *   - per-subdomain interior factorisations and interface Schur complements
 *     (Section 2: S = K_GG - K_GI K_II^{-1} K_IG);
 *   - the adaptive set-up of Alg. 3: per level, BDDC structures with the
 *     initial constraints (corners + edge averages, Section 7), the pair
 *     generalized eigenproblems of eq. eig-matrix solved by LOBPCG with the
 *     BDDC pair preconditioner of eq. bddc_pair (Section 5), selection of
 *     eigenvalues above tau (Alg. 2), face constraint rows from eq. d-def
 *     (Prop. 1; edge entries dropped and rows orthonormalised, Section 7),
 *     enriched BDDC structures, and recursion to the next level (Section 3);
 *   - PCG preconditioned by Multilevel BDDC (Alg. 1) with a Lanczos
 *     condition estimate (Section 8);
 *   - the element gradient -lambda^T (dK/dtheta_e) x of a misfit with
 *     respect to element log10-coefficients.
 *
 * Conventions for every call:
 *   - Status codes are returned; ambddc_last_error() gives a message for the
 *     calling thread, valid until that thread's next call.
 *   - Indices are 0-based int32.  Matrices are column-major.
 *   - Free-DOF numbering: node-major, component-minor (DOF id = node*d + c),
 *     Dirichlet DOFs removed, remaining DOFs keep their order.
 *   - Element local node order is lexicographic: local index a + 2b + 4c is
 *     the node at offset (a, b, c) from the element's lowest corner.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are GPU
 *     memory on the handle's device (e.g. torch tensor data_ptr()).
 *   - The caller owns every buffer it passes; the library copies what it
 *     keeps and owns all memory inside the handle.  One handle must not be
 *     used by two threads at the same time.
 */
#ifndef AMBDDC_H
#define AMBDDC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AMBDDC_OK = 0,
  AMBDDC_E_INVALID_ARG = 1,   /* bad pointer, size or option */
  AMBDDC_E_NOT_SPD = 2,       /* a Cholesky pivot was not positive (message names the matrix) */
  AMBDDC_E_ASSUMPTION = 3,    /* Assumption 1 fails on a pair (message names the pair) */
  AMBDDC_E_NO_CONVERGENCE = 4,/* PCG hit maxit; x holds the last iterate */
  AMBDDC_E_OOM = 5,           /* device allocation failed */
  AMBDDC_E_DEVICE = 6,        /* HIP runtime error */
  AMBDDC_E_STATE = 7          /* call out of order (e.g. solve before setup) */
} ambddc_status;

typedef struct ambddc_ctx* ambddc_handle;

enum { AMBDDC_INIT_CE = 0, AMBDDC_INIT_CEF = 1, AMBDDC_INIT_C = 2 };

/* Conforming hexahedral mesh (Section 2).  All pointers are host. */
typedef struct {
  int32_t n_nodes;
  int32_t n_elems;
  int32_t dof_per_node;        /* 1 = Poisson, 3 = elasticity */
  const double* coords;        /* [n_nodes*3] x,y,z per node */
  const int32_t* elem_nodes;   /* [n_elems*8] lexicographic local order */
  const uint8_t* dirichlet;    /* [n_nodes*dof_per_node] 1 = DOF fixed to zero */
} ambddc_mesh;

/* Decomposition into subdomains (unions of elements) and agglomerated
 * higher levels (Section 3).  All pointers are host. */
typedef struct {
  int32_t levels;                  /* L >= 2: levels 1..L-1 are substructured, level L solved directly */
  const int32_t* elem_to_sub;      /* [n_elems] level-1 subdomain of each element */
  const int32_t* const* parents;   /* [levels-2] arrays: level-i subdomain -> level-(i+1) subdomain */
} ambddc_decomp;

typedef struct {
  double tau;                  /* adaptive threshold (Alg. 2); <= 0 or inf disables adaptivity */
  int32_t nev_max;             /* cap on adaptive constraints per face (10 in Section 8) */
  int32_t lobpcg_maxit;        /* LOBPCG iteration cap (e.g. 100) */
  int32_t lobpcg_block;        /* LOBPCG block size m >= nev_max+1 (e.g. 16) */
  double lobpcg_tol;           /* relative residual tolerance (e.g. 1e-8) */
  int32_t precision;           /* 0 = FP64 everywhere.
                                  1 = the dense subdomain operators of the PCG
                                  preconditioner (Alg. 1 on every substructured
                                  level) stored in FP32 and widened to FP64 on load;
                                  PCG iterates on FP64 residuals, so it reaches the
                                  same FP64 accuracy (iterative refinement around
                                  the rounded preconditioner).
                                  2 = precision 1, and the pair LOBPCG starts with
                                  its operator products (S^s, and the Neumann
                                  inverse and coarse basis of the pair
                                  preconditioner) on FP32 copies with FP32 MFMA
                                  accumulation; each pair moves to FP64 products
                                  once its residual reaches 1e-5 or stops halving
                                  over three iterations, and converges to
                                  lobpcg_tol in FP64, so eigenvalues, the tau
                                  decision and the constraints are those of FP64.
                                  Gram matrices, Rayleigh-Ritz, orthogonalisation,
                                  Schur complements and the coarsest problem stay
                                  FP64 in every mode. */
  int32_t initial_constraints; /* initial coarse DOFs (Section 7; the variants of
                                  Section 8.2's tables): AMBDDC_INIT_CE (0) corners and
                                  one arithmetic average per edge and displacement
                                  component; AMBDDC_INIT_CEF (1) also face averages;
                                  AMBDDC_INIT_C (2) corners only */
  int32_t keep_edges;          /* 0: adaptive constraint rows keep only their entries on
                                  the face (the entries on shared edges and corners are
                                  set to zero, Section 7); 1: rows keep their entries on
                                  all DOFs the two subdomains share (the rows of
                                  eq. d-def as they are, which keep the bound
                                  omega <= tau); the row is a coarse DOF of the pair's
                                  two subdomains only */
  int32_t fixed_per_face;      /* 0: Alg. 2 (eigenvalues above tau, at most nev_max);
                                  k > 0: every face gets the constraints of its k
                                  largest eigenvectors whatever tau ("3eigv" in
                                  Section 8.2 is k = 3 with AMBDDC_INIT_CE) */
  uint64_t seed;               /* LOBPCG start vectors */
  void* stream;                /* hipStream_t for all work (NULL = default stream) */
} ambddc_options;

/* Fill *opt with defaults: tau 10, nev_max 10, maxit 100, block 16, tol 1e-7, FP64. */
void ambddc_default_options(ambddc_options* opt);

/* Level-1 structure counts (the columns n, n_Gamma, n_f of Section 8's
 * tables) computed on the host only; touches no GPU. */
typedef struct {
  int32_t n_free;              /* unknowns after Dirichlet removal */
  int32_t n_sub;
  int32_t n_interface;         /* free DOFs on the interface Gamma */
  int32_t n_faces, n_edges, n_corners;   /* globs with at least one free DOF */
  int32_t n_coarse_initial;    /* initial constraints of the chosen set (AMBDDC_INIT_*) */
  int32_t n_pairs;             /* adjacent pairs = faces */
} ambddc_analysis;

/* sub_sizes_host may be NULL, else [2*n_sub]: (n_I, n_Gamma) per subdomain.
 * Pass n_sub_cap = its capacity in subdomains; E_INVALID_ARG if too small. */
ambddc_status ambddc_analyze(const ambddc_mesh* mesh, const ambddc_decomp* decomp,
                             int32_t initial_constraints, ambddc_analysis* out,
                             int32_t* sub_sizes_host, int32_t n_sub_cap);

/* Analyse the mesh and decomposition: level-1 DOF numbering, interface and
 * glob classification (faces, edges, corners; Section 2), initial
 * constraints, pair lists, device index maps.  Copies everything it needs;
 * the inputs may be freed afterwards.  Errors: E_INVALID_ARG for
 * inconsistent sizes or ids, E_OOM, E_DEVICE. */
ambddc_status ambddc_create(const ambddc_mesh* mesh, const ambddc_decomp* decomp,
                            const ambddc_options* opt, ambddc_handle* out);

/* Numeric set-up (Alg. 3) for element coefficients resident on the device:
 * coeff[n_elems] = kappa (Poisson) or Young's modulus E (elasticity),
 * nu[n_elems] = Poisson ratio (elasticity; NULL for Poisson).  May be called
 * again with new coefficients; the previous hierarchy is replaced.  The
 * first set-up on a handle also chooses, by timing both, the tile shape of
 * the grouped pair-eigenproblem products on every level (64 x 64 or
 * 128 x 32; both give identical results) and keeps the choice for later
 * set-ups.
 * Errors: E_INVALID_ARG (also for a coefficient that is not a finite number,
 * naming the element, or a Poisson ratio outside (-1, 1/2)), E_NOT_SPD (a
 * subdomain or coarse factorisation meets a non-positive pivot, e.g. for a
 * negative coefficient), E_ASSUMPTION (a pair coarse matrix has null vectors
 * beyond the rigid modes both subdomains share: Assumption 1 of Section 4
 * fails; the message names the pair), E_OOM, E_DEVICE.  LOBPCG that reaches
 * lobpcg_maxit is not an error: the unconverged pairs are counted in the
 * statistics (n_unconverged) and their current Ritz values are used. */
ambddc_status ambddc_setup(ambddc_handle h, const double* coeff_dev, const double* nu_dev);

/* PCG with the Multilevel BDDC preconditioner (Alg. 1), stopping when
 * ||f - K x||_2 / ||f||_2 <= rtol per column (FP64 residual).  x0 is the
 * level-1 interior solution [K_II^-1 f_I; 0], so every residual is zero on
 * the level-1 interiors and the iterates stay in the discrete harmonic
 * space of Section 2: PCG on the interface problem of the Schur complement,
 * the problem BDDC preconditions (Section 5).  Alg. 1's level-1 interior
 * pre-correction is then zero and skipped.  The
 * iteration updates the residual recursively; when that meets rtol, the true
 * residual f - K x is recomputed, and a column stops only if it meets rtol
 * too; otherwise it restarts from the true residual (residual replacement),
 * unless the true residual fell by less than half since the column's
 * previous check: then rtol lies below what FP64 attains on this system
 * (the rounding floor of f - K x) and the column stops, counted in
 * ambddc_stats.pcg_stalled, with E_NO_CONVERGENCE.
 * rhs_dev, x_dev: device [n_free*nrhs] column-major (ld = n_free).
 * iterations_host[nrhs], cond_host[nrhs] (Lanczos estimate of the
 * preconditioned condition number) may be NULL.  The columns are
 * independent recurrences advanced in lockstep.  Errors: E_STATE before
 * setup, E_NO_CONVERGENCE (maxit reached or a stalled column; x holds the
 * last iterate and ambddc_last_residual its true residuals), E_DEVICE. */
ambddc_status ambddc_solve(ambddc_handle h, const double* rhs_dev, int32_t nrhs, double rtol,
                           int32_t maxit, double* x_dev, int32_t* iterations_host,
                           double* cond_host);

/* ambddc_solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same PCG and preconditioner, with every scratch buffer of the solve
 * (the PCG columns, dot products, coefficient histories, column flags) in
 * one fixed device array of 64 MiB per GPU, held until the process ends; it
 * calls no device allocator.  Arguments, results and errors as ambddc_solve,
 * and the results are identical to it.  Limits, rejected with
 * E_INVALID_ARG: nrhs in 1..3, no more than the preconditioner's workspace
 * of the handle holds (1 after set-up; an ambddc_solve with more columns
 * prepares more), and (4 n_free + 2 maxit + 270) nrhs doubles must fit in
 * the array (n_free nrhs up to about two million).  Every call on a GPU
 * shares that GPU's array: calls that overlap in time on one GPU (from two
 * threads or two streams) race and must not be issued; each call
 * initialises what it reads. */
ambddc_status ambddc_solve_noalloc(ambddc_handle h, const double* rhs_dev, int32_t nrhs,
                                   double rtol, int32_t maxit, double* x_dev,
                                   int32_t* iterations_host, double* cond_host);

/* True relative residuals ||f_k - K x_k||_2 / ||f_k||_2 of the last
 * ambddc_solve (recomputed with one product by K after the iteration, which
 * itself tracks only the recursively updated residual): res_host[nrhs], host.
 * Errors: E_STATE if nrhs differs from the last solve's. */
ambddc_status ambddc_last_residual(ambddc_handle h, int32_t nrhs, double* res_host);

/* Numeric set-up from element log10-coefficients: coeff_e = 10^theta_e is
 * computed on the device, then as ambddc_setup.  theta_dev: device
 * [n_elems]; nu_dev as in ambddc_setup.  Same errors as ambddc_setup. */
ambddc_status ambddc_setup_log10(ambddc_handle h, const double* theta_dev, const double* nu_dev);

/* Least-squares misfit of solutions against observations:
 * R = X - X_obs (device [n_free*nrhs], may alias neither input) and, if
 * J_host is not NULL, J = 1/2 ||R||_F^2 (host).  R is the right-hand side of
 * the adjoint solve K Lam = R.  nrhs in 1..16.  Errors: E_INVALID_ARG. */
ambddc_status ambddc_misfit(ambddc_handle h, const double* X_dev, const double* Xobs_dev,
                            int32_t nrhs, double* R_dev, double* J_host);

/* Element gradient of a misfit w.r.t. element log10-coefficients theta_e,
 * K = sum_e 10^theta_e Khat_e:  grad[e] = -ln(10) sum_k lam_k,e^T K_e x_k,e
 * with the element matrices of the last setup.  X_dev, Lam_dev: device
 * [n_free*nrhs] column-major; grad_dev: device [n_elems]. */
ambddc_status ambddc_element_gradient(ambddc_handle h, const double* X_dev, const double* Lam_dev,
                                      int32_t nrhs, double* grad_dev);

/* Set-up statistics, per level i < 8 (paper's reported quantities). */
typedef struct {
  int32_t levels;                /* substructured levels (L-1) */
  int32_t n_free;                /* level-1 unknowns */
  int32_t n_sub[8];
  int32_t n_pairs[8];            /* faces = adjacent pairs */
  int32_t n_coarse[8];           /* coarse DOFs after enrichment */
  int32_t n_adaptive[8];         /* adaptive constraints added */
  int32_t lobpcg_iters[8];       /* LOBPCG iterations run (lockstep) */
  int32_t lobpcg_iters_fp32[8];  /* of those, iterations in which some pair ran FP32
                                    products (precision 2) */
  int32_t n_unconverged[8];      /* pairs not converged at lobpcg_maxit */
  double omega_tilde[8];         /* max over pairs of the first unselected eigenvalue */
  double t_phase[16];            /* seconds: 0 assembly+Schur, 1 BDDC init, 2 LOBPCG,
                                    3 selection, 4 enriched BDDC, 5 coarse, 6 total setup,
                                    7 last solve */
  int32_t pcg_replacements;      /* residual replacements in the last solve: columns whose
                                    recursive residual met rtol while the recomputed
                                    f - K x did not, and which went on from the latter */
  int32_t pcg_stalled;           /* columns of the last solve stopped because their true
                                    residual no longer fell above rtol (E_NO_CONVERGENCE) */
} ambddc_stats;

ambddc_status ambddc_get_stats(ambddc_handle h, ambddc_stats* out);

/* ---- introspection (copies to host; for parity checks and tooling) ---- */

/* Sizes of substructured level `level` (0-based). Any out pointer may be NULL. */
ambddc_status ambddc_level_info(ambddc_handle h, int32_t level, int32_t* n_dof, int32_t* n_sub,
                                int32_t* n_pairs, int32_t* n_coarse);

/* Level DOF ids of subdomain `sub`, interior first then interface, each
 * group ascending.  dofs_host may be NULL to query n_I, n_G only. */
ambddc_status ambddc_sub_dofs(ambddc_handle h, int32_t level, int32_t sub, int32_t* dofs_host,
                              int32_t* n_I, int32_t* n_G);

/* Interface Schur complement S of `sub`, n_G x n_G column-major, host. */
ambddc_status ambddc_get_schur(ambddc_handle h, int32_t level, int32_t sub, double* S_host);

/* Subdomains of pair `pair` (one pair per face glob); n_face = number of
 * DOFs its constraint rows are supported on (see ambddc_get_face_constraints). */
ambddc_status ambddc_pair_info(ambddc_handle h, int32_t level, int32_t pair, int32_t* s, int32_t* t,
                               int32_t* n_face);

/* Result of the pair eigenproblem: *block = the LOBPCG block size m of the
 * level (max(lobpcg_block, constraints per face + 1)); lam_host[m]
 * (descending) and resid_host[m], relative residuals
 * |A x - lam B x| / (|A x| + max(|lam|, 1e-6 lam_1) |B x|), written when
 * cap >= m (cap = entries the two arrays hold; E_INVALID_ARG otherwise, so
 * query m first with both NULL); number of selected constraints k (after the
 * QR rank test), the first unselected eigenvalue, LOBPCG iterations and a
 * converged flag.  Any output pointer may be NULL. */
ambddc_status ambddc_get_pair_result(ambddc_handle h, int32_t level, int32_t pair, int32_t cap,
                                     int32_t* block, double* lam_host, double* resid_host,
                                     int32_t* k, double* lam_next, int32_t* iters,
                                     int32_t* converged);

/* Adaptive constraint rows of the face of `pair`: rows_host[k*n_face],
 * row-major (row l = l-th orthonormal row), and the level DOF ids they are
 * supported on, face_dofs_host[n_face], ascending: the face DOFs, or with
 * keep_edges every DOF the two subdomains share.  Either pointer may be
 * NULL. */
ambddc_status ambddc_get_face_constraints(ambddc_handle h, int32_t level, int32_t pair,
                                          double* rows_host, int32_t* face_dofs_host);

/* Coarse element matrix K_c^s = Psi^T S Psi of `sub` (n_c x n_c, column-major,
 * rows in ascending coarse id, Section 5), host.  n_c from *nc (may be
 * queried with Kc_host = NULL). */
ambddc_status ambddc_get_coarse_element(ambddc_handle h, int32_t level, int32_t sub,
                                        double* Kc_host, int32_t* nc);

/* Assembled coarse matrix of the top level (n_coarse x n_coarse of the last
 * substructured level), host, column-major. */
ambddc_status ambddc_get_top_coarse(ambddc_handle h, double* Kc_host, int32_t* n);

/* ---- kernel timing (measurement) ----
 * ambddc_timing_enable selects classes of kernel launches (comma-separated
 * names; NULL or "" switches timing off) and clears their counters.  Each
 * launch of a selected class is then bracketed by two HIP events recorded on
 * the handle's stream, and the library adds to the class the algorithmic
 * work of that launch (the count the roofline is taken against):
 *   "pair_rr"      batched Rayleigh-Ritz of the pair LOBPCG (one workgroup
 *                  per active pair, order nb = 3m): flops 9 nb^3 + 4/3 nb^3
 *                  + 2 nb^2 m per pair (reduction to a standard problem and a
 *                  symmetric eigendecomposition with vectors, LAPACK-style
 *                  counts), bytes 8 (2 nb^2 + 2 nb m) per pair;
 *   "pair_apply"   grouped S^s products of the pair LOBPCG: per subdomain
 *                  with an active pair, 2 nG^2 c flops and 8 (nG^2 + 2 nG c)
 *                  bytes, c = columns of the slots of its active pairs (tiles
 *                  whose slots all belong to converged pairs are skipped);
 *   "pair_gram"    Gram matrices V^T (A V), V^T (B V): 2 n nb^2 flops and
 *                  8 (2 n nb + nb^2) bytes per active pair and matrix;
 *   "schur"        batched interior factorisations and Schur complements
 *                  (partial Cholesky on level 1 with the triangular solve
 *                  for K_GI K_II^-1, augmented partial LDL^T deeper): per
 *                  subdomain nI^3/3 + nI^2 nG + nI nG^2 flops (level 1 also
 *                  nG nI^2 for the solve) and 8 (nI + nG)^2 bytes;
 *   "bddc_apply"   one application of the multilevel preconditioner
 *                  (Alg. 1, all levels) to harmonic residuals: the dense
 *                  operators it reads, per subdomain nI nG + nG^2 + 2 nG nc
 *                  entries (deeper levels also nI^2 + nI nG), plus the
 *                  n_top^2 coarsest inverse; flops 2 x entries x nrhs;
 *                  bytes 8 x entries (4 x the deeper levels' and the Z, Psi
 *                  entries with precision 1; nG (nG + 1) / 2 for Z in FP64
 *                  with up to 3 right-hand sides, which read its lower
 *                  tiles) + 8 x 6 vector entries per DOF and right-hand
 *                  side.
 * ambddc_timing_read returns, for one class, the launches, the summed event
 * time in milliseconds and the summed algorithmic flops and bytes since the
 * last enable (any pointer may be NULL; it waits for the recorded events).
 * Errors: E_INVALID_ARG for an unknown class name. */
ambddc_status ambddc_timing_enable(ambddc_handle h, const char* classes);
ambddc_status ambddc_timing_read(ambddc_handle h, const char* cls, int32_t* launches,
                                 double* total_ms, double* flops, double* bytes);

/* ---- PCG iteration graphs ----
 * flags & 1: ambddc_solve with up to 3 right-hand sides and kernel-class
 * timing off runs each PCG iteration from its second on as two HIP graphs
 * (the mat-vec through the convergence flags, then the preconditioner),
 * captured on a private stream of the library and launched on the handle's
 * stream; they are captured again after a set-up and for new solve
 * arguments.  Results are identical to the launch-by-launch iteration.  Off
 * by default (flags 0): on MI355X a replayed node costs about as much as the
 * launch it replaces, and every set-up forces a new capture.
 * Errors: E_INVALID_ARG for a null handle or unknown flag bits. */
ambddc_status ambddc_set_graphs(ambddc_handle h, int32_t flags);

const char* ambddc_last_error(void);
void ambddc_destroy(ambddc_handle h);

#ifdef __cplusplus
}
#endif
#endif /* AMBDDC_H */
