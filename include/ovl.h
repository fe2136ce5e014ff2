/*
 * ovl.h -- C ABI of the MI355X (gfx950) overlap-operator library.
 *
 * Method: N. Cundy, W. Lee, "The eigSUMR inverter for overlap fermions"
 * (arXiv:1501.01855).  The library applies the overlap operator
 *     D[mu] = (1 + mu + (1 - mu) gamma_5 sign(K)) / 2          (Sec. 1, eq. 1)
 * with the Wilson kernel K = gamma_5 D_W(-rho)                  (Sec. 1, eq. 2)
 * and solves D[mu] x = b with GMRESR(relSUMR)                   (Secs. 2-3, Algs. 1-3)
 * with eigSUMR deflation                                        (Secs. 4-5, Algs. 5-6),
 * or with GMRESR(relCG) and the spectral preconditioner          (Sec. 4, its CGNE).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Status:   every function returns an ovl_status; 0 = OVL_OK.  On error a
 *           message is available from ovl_last_error() (per thread).  No C++
 *           exception crosses the ABI.
 * Memory:   field buffers are caller-owned DEVICE memory unless the argument
 *           name ends in _host.  The library never frees them.  Handles own
 *           their internal (packed) copies and workspace, released by the
 *           matching destroy call.
 * Layout:   canonical complex128, real and imaginary parts interleaved:
 *             spinor  psi[site][spin][colour]        (12 complex per site)
 *             gauge   U[site][mu][a][b]              (36 complex per site)
 *           site = x + Lx*(y + Ly*(z + Lz*t)), mu = 0..3 = x, y, z, t,
 *           periodic boundaries.  nrhs right-hand sides are contiguous
 *           fields (rhs-major).
 * Gammas:   chiral basis, gamma_k = [[0, -i s_k], [i s_k, 0]] (s_k Pauli),
 *           gamma_4 = [[0, 1], [1, 0]], gamma_5 = diag(1, 1, -1, -1).
 * Kernel:   K = gamma_5 [(4 - rho) - H/2],
 *           H psi(x) = sum_mu (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                     + (1 + gamma_mu) U_mu(x-mu)^dagger psi(x-mu),
 *           i.e. the paper's kernel times (8 - 2 rho)/2 (kappa = 1/(8 - 2 rho));
 *           sign(K) is unchanged by that positive factor.
 * Streams:  all device work of a context runs on the HIP stream given at
 *           creation (0 = the null stream).  Operator calls are asynchronous;
 *           solver calls and calls that return host data block until done.
 * Precision: OVL_F64 (FP64 storage and arithmetic), OVL_F32 (FP32 storage and
 *           arithmetic, FP64 reductions and scalars), OVL_HALF (FP16 links,
 *           FP16 spinors with one FP32 scale per site, FP32 arithmetic).
 */
#ifndef OVL_H
#define OVL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    OVL_OK = 0,
    OVL_ERR_ARG = -1,           /* invalid argument (null pointer, size, range) */
    OVL_ERR_HIP = -2,           /* a HIP runtime call failed                   */
    OVL_ERR_NOMEM = -3,         /* device allocation failed                    */
    OVL_ERR_NOT_CONVERGED = -4, /* iteration limit reached; best iterate written */
    OVL_ERR_BREAKDOWN = -5,     /* NaN / Inf or a breakdown of a recurrence    */
    OVL_ERR_UNSUPPORTED = -6,   /* valid request the library does not provide  */
    OVL_ERR_STATE = -7          /* missing set-up (no gauge field loaded, ...) */
} ovl_status;

typedef enum { OVL_F64 = 0, OVL_F32 = 1, OVL_HALF = 2 } ovl_prec;

typedef enum { OVL_SRC_POINT = 0, OVL_SRC_GAUSS = 1, OVL_SRC_Z2 = 2 } ovl_source_kind;

#define OVL_MAX_NZ 64

/* Zolotarev optimal rational approximation (Sec. 3, eq. 7):
 *   eps(x) = x sum_{l<n_z} omega[l] / (x^2 + sigma[l]),  |eps| in [1-delta, 1+delta]
 *   for a <= |x| <= b. */
typedef struct {
    int32_t n_z;
    double a, b, delta;
    double omega[OVL_MAX_NZ];
    double sigma[OVL_MAX_NZ];
} ovl_zolo;

/* Counters of one call (or, for the solver, one right-hand side).
 * dslash_calls[p] counts hopping-term applications in precision p (the paper
 * counts a double-precision Wilson call as two units, single as one, Sec. 6). */
typedef struct {
    int64_t dslash_calls[3];
    int64_t sign_calls[3];
    int64_t mscg_iters;
    int64_t sumr_iters;       /* middle-solve iterations (SUMR or CG)            */
    int64_t gmresr_steps;
    int64_t restarts;
    double computed_relres;     /* solver: final recurrence residual / ||b|| */
    double seconds;             /* wall time of the call                     */
} ovl_stats;

/* Parameters of ovl_sumr_gmresr_solve (defaults from ovl_solver_defaults). */
typedef struct {
    double rho;            /* kernel mass parameter, K = gamma_5 D_W(-rho)          */
    double mu;             /* overlap mass parameter, 0 <= mu < 1                   */
    double tol;            /* outer target ||b - D x|| <= tol ||b|| (Alg. 3 eps)    */
    double eta_tilde;      /* middle-solve relative accuracy (Alg. 3 eta~)          */
    double relax_floor;    /* worst sign accuracy allowed in the middle solve (Sec. 3: 1e-2) */
    double f32_threshold;  /* sign accuracies >= this use OVL_F32 (Sec. 3: ~1e-7, larger) */
    double half_threshold; /* sign accuracies >= this use OVL_HALF; > 1 disables    */
    double norm_restart;   /* SUMR restart when | ||q|| - 1 | exceeds this (Sec. 6: 0.1) */
    int32_t max_outer;     /* GMRESR steps                                          */
    int32_t max_middle;    /* SUMR or CG iterations per middle solve                */
    int32_t max_mscg;      /* multi-shift CG iterations per sign call               */
    int32_t use_deflation; /* 1: start middle solves from the eigenspace projection (Sec. 4) */
    int32_t eig_calc;      /* 1: collect eigenvectors during this solve: eigSUMR
                              (Alg. 5) or, with middle_cg, eigCG (Sec. 5); the solve
                              ends with the three-set re-diagonalisation of Sec. 5
                              (its eigenvectors and those kept at the end of the
                              previous two calculating solves)                    */
    int32_t n_eig;         /* eigSUMR: eigenvectors kept (n)                         */
    int32_t m_eig;         /* eigSUMR: basis size at which Alg. 6 runs (m > n)       */
    int32_t k_recalc;      /* eigSUMR: recompute v^D = D v every k diagonalisations   */
    int32_t verbose;
    double eig_eps;        /* eigSUMR: target eigenvector accuracy (Sec. 6: 1e-4)    */
    double delta_split;    /* eigSUMR: pair splitting in M (Sec. 5), 0 < delta < 1/2 */
    int32_t middle_cg;     /* 0: relSUMR middle solve (Algs. 1, 2); 1: relCG, the
                              preconditioned CGNE of Sec. 4 on H^2 = D^+ D for
                              H u = gamma_5 r, relaxed as in Sec. 3 for CG; with
                              use_deflation the spectral preconditioner of Sec. 4 is
                              built from the held eigenspace (Rayleigh-Ritz vectors
                              of H^2 in its span, c = sqrt(3)/2).  Its sign calls
                              use FP32 at most (FP16 rounding swamps the lowest
                              eigenvalues of H^2, ~mu^2).  With eig_calc (eigCG,
                              Sec. 5) each CG iteration adds its direction
                              w = Hhat^{-1} p and H w, unit-normed, with images
                              gamma_5 H w and gamma_5 H H w, to the eigenspace; Alg. 6
                              diagonalises at m and after each middle solve, the
                              Sec. 5.1 bound caps the sign accuracy, and each middle
                              solve keeps the preconditioner it started with. */
    int32_t eig_block;     /* with eig_calc (relSUMR middle solve): the nrhs
                              right-hand sides are solved together and every
                              field's Krylov vectors (q, U q) enter the one
                              eigenspace (block eigSUMR); Alg. 6 then
                              orthonormalises the basis canonically
                              (eigenvectors of V^H V, directions below 1e-10 of
                              the largest dropped) since Krylov sequences of
                              related sources are nearly dependent.  0: calculating
                              solves run one right-hand side after another. */
} ovl_solver_params;

typedef struct ovl_context ovl_context;

/* ---- context ----------------------------------------------------------- */

/* Create a context for one lattice of extents dims[4] (x, y, z, t, each >= 2)
 * on the current HIP device, issuing work on hip_stream (a hipStream_t; 0 =
 * null stream).  Allocates the context's workspace. */
ovl_status ovl_create(const int32_t dims[4], void *hip_stream, ovl_context **out);
ovl_status ovl_destroy(ovl_context *ctx);
const char *ovl_last_error(void);
void ovl_solver_defaults(ovl_solver_params *p);
/* Device bytes currently held by the context (workspace + packed fields). */
int64_t ovl_device_bytes(const ovl_context *ctx);

/* ---- set-up: gauge field, sources (not part of the method; Sec. 6 inputs) -- */

/* Load a gauge field from canonical complex128 device memory U_dev[V*36*2]
 * and pack it into the internal layouts of every precision. */
ovl_status ovl_gauge_load(ovl_context *ctx, const double *U_dev);

/* Generate U_mu(x) = exp(i eps sum_a g_a T^a), g_a ~ N(0,1) from the seeded
 * Philox4x32-10 stream, on the GPU, and load it; if U_out_dev is not null the
 * canonical field is also written there.  Bit-identical to the reference
 * generator of the test suite. */
ovl_status ovl_gauge_generate(ovl_context *ctx, uint64_t seed, double eps, double *U_out_dev);

/* Write one source field (canonical, device): point source at
 * (site, spin, colour); complex Gaussian (Re, Im ~ N(0,1)); or Z2 noise (each
 * real component +-1, Sec. 6). */
ovl_status ovl_source_generate(ovl_context *ctx, int kind, uint64_t seed, int64_t site,
                               int32_t spin, int32_t colour, double *out_dev);

/* ---- operators (Sec. 1, eqs. 1-2; Sec. 3, eq. 7) ------------------------- */

/* out = H in (the hopping term, 8-point stencil), nrhs fields. */
ovl_status ovl_wilson_dslash(ovl_context *ctx, const double *in_dev, double *out_dev,
                             int32_t nrhs, int32_t prec);

/* out = K in = gamma_5 [(4 - rho) in - H in / 2], nrhs fields. */
ovl_status ovl_kernel_K_apply(ovl_context *ctx, double rho, const double *in_dev,
                              double *out_dev, int32_t nrhs, int32_t prec);

/* Zolotarev coefficients for n_z poles on [a, b] (host, FP64; Sec. 3, eq. 7).
 * 1 <= n_z <= OVL_MAX_NZ, 0 < a < b. */
ovl_status ovl_zolotarev_coeffs(int32_t n_z, double a, double b, ovl_zolo *out_host);

/* Kernel low modes (Sec. 1 after eq. 4; Sec. 3): compute the n_low eigenpairs
 * of K with the smallest |lambda| (FP64, on the GPU) and keep them in the
 * context; the sign function then treats them exactly.  evals_host (may be
 * null) receives the n_low eigenvalues, ordered by |lambda|; lmax_host (may
 * be null) receives an upper bound for |lambda| (largest Ritz value of K^2,
 * square-rooted, times 1.01).  tol is the eigen-residual target
 * ||K v - lambda v|| <= tol. */
ovl_status ovl_lowmodes_compute(ovl_context *ctx, double rho, int32_t n_low, double tol,
                                double *evals_host, double *lmax_host);
/* Spectral interval of K for the Zolotarev approximation when no kernel
 * modes are treated exactly (Sec. 3: a^2 and b^2 are the smallest and largest
 * eigenvalues of K^2): Lanczos on K^2 in FP64 from a fixed Gaussian start,
 * at most max_iter steps (2 .. 2000), stopping once the smallest Ritz value
 * has moved by less than 1e-10 (relative) over two checks ten steps apart.
 * lmin_host: square root of the smallest Ritz value of K^2, which lies above
 * min |lambda|^2 (Ritz values of a Hermitian matrix lie inside its spectrum),
 * so callers take a margin below it; lmin_err_host (may be null): the Lanczos
 * residual bound |beta_k y_k| of that Ritz value of K^2 (some eigenvalue of
 * K^2 is within it); lmax_host (may be null): square root of the largest Ritz
 * value (a lower estimate of max |lambda|; 8 - rho bounds it from above). */
ovl_status ovl_kernel_interval(ovl_context *ctx, double rho, int32_t max_iter, double *lmin_host,
                               double *lmin_err_host, double *lmax_host);
/* Install caller-provided low modes instead (n vectors, canonical, device;
 * orthonormal).  n = 0 removes them. */
ovl_status ovl_lowmodes_set(ovl_context *ctx, int32_t n, const double *evals_host,
                            const double *evecs_dev);
/* Copy the context's low modes out (canonical, device, n_low fields). */
ovl_status ovl_lowmodes_get(ovl_context *ctx, double *evecs_dev);

/* out = sign(K) in: the context's low modes exactly, eps(K) on the rest,
 * eps(K) by multi-shift CG on (K^2 + sigma_l) to sign accuracy eta
 * (||error|| <= eta ||in|| in exact arithmetic, plus zolo->delta). */
ovl_status ovl_sign_zolotarev_mscg(ovl_context *ctx, double rho, const ovl_zolo *zolo,
                                   const double *in_dev, double *out_dev, int32_t nrhs,
                                   double eta, int32_t prec, ovl_stats *stats_host);

/* out = sign(K) in by the two-pass Lanczos method (the Lanczos approach to
 * the sign function cited in Sec. 1 after eq. 4), FP64: the context's low
 * modes exactly; on the rest, Lanczos on K^2 keeps only its tridiagonal
 * matrix T in a first pass, stopping once lambda_max ||y_k - y_{k-10}|| <=
 * eta ||in|| for y_k = ||in_perp|| T_k^{-1/2} e_1 (checked every ten steps),
 * and a second pass regenerates the Lanczos vectors from the stored
 * coefficients and sums them with weights y; the result is K times that sum.
 * No rational approximation error: zolo is used for its interval only
 * (zolo->a <= |lambda| <= zolo->b off the low modes; 0 < a < b).  stats_host
 * (may be null): mscg_iters = Lanczos steps of the first pass, summed over
 * the nrhs fields.  OVL_ERR_NOT_CONVERGED after 20000 steps. */
ovl_status ovl_sign_lanczos(ovl_context *ctx, double rho, const ovl_zolo *zolo, const double *in_dev,
                            double *out_dev, int32_t nrhs, double eta, ovl_stats *stats_host);

/* out = D[mu] in (Sec. 1, eq. 1) with the sign function as above. */
ovl_status ovl_overlap_apply(ovl_context *ctx, double rho, double mu, const ovl_zolo *zolo,
                             const double *in_dev, double *out_dev, int32_t nrhs, double eta,
                             int32_t prec, ovl_stats *stats_host);

/* Derivatives of S = sum_f Re(chi_f^H D[mu] psi_f) over nrhs field pairs, for
 * D[mu] (Sec. 1, eq. 1) with the rational sign function
 * eps(K) = K sum_l omega_l (K^2 + sigma_l)^{-1} (Sec. 1, eq. 4; Sec. 3, eq. 7).
 * Gradients are d/dRe + i d/dIm, every link entry an independent complex
 * variable (U in the forward hop, U^dagger in the backward one).
 *   dS_dpsi_dev (may be null): D^dagger chi_f = gamma_5 D gamma_5 chi_f per
 *     field, canonical [nrhs][V][4][3] complex128.
 *   dS_dU_dev (may be null): the link gradient summed over the nrhs pairs,
 *     canonical [V][4][3][3] complex128 (same layout as the gauge field);
 *     overwritten.  Needs psi_dev.
 * At least one output must be given.  Each shifted inversion runs to
 * |zeta_l| ||r|| <= eta ||source||; prec OVL_F64 or OVL_F32 (FP32 storage
 * and arithmetic for the inversions, FP64 link accumulation).  The exactly
 * treated low modes are not differentiated: with low modes in the context this
 * returns OVL_ERR_UNSUPPORTED.  stats_host (may be null): one record. */
ovl_status ovl_overlap_adjoint(ovl_context *ctx, double rho, double mu, const ovl_zolo *zolo,
                               const double *psi_dev, const double *chi_dev, int32_t nrhs, double eta,
                               int32_t prec, double *dS_dpsi_dev, double *dS_dU_dev,
                               ovl_stats *stats_host);

/* ---- solver (Algs. 1-3, Sec. 3 relaxation, Secs. 4-5 deflation) ---------- */

/* Solve D[mu] x = b for nrhs right-hand sides (one after another) with
 * GMRESR(relSUMR).  b_dev, x_dev canonical; x is overwritten.  stats_host
 * (may be null) has nrhs entries.  Returns OVL_ERR_NOT_CONVERGED with the best
 * iterate in x when an iteration limit is hit. */
ovl_status ovl_sumr_gmresr_solve(ovl_context *ctx, const ovl_zolo *zolo,
                                 const ovl_solver_params *params, const double *b_dev,
                                 double *x_dev, int32_t nrhs, ovl_stats *stats_host);

/* Several independent solves at once: lattice instances of any sizes, each
 * with its own context (and so its own stream, gauge field, low modes and
 * workspace).  A pool of at most 32 host threads takes the instances in
 * index order, one solve per thread at a time, so the GPU runs up to 32
 * instances' kernels side by side (small lattices alone cannot fill it).
 * Contexts must be distinct, and their streams should be distinct for the
 * work to overlap.  params apply to every instance.  inst[i].status receives
 * each solve's status and inst[i].message its error text (empty on success);
 * the return value is the first failure in index order (OVL_OK if none), and
 * ovl_last_error() then names that instance.  Blocks until every solve has
 * finished. */
typedef struct {
    ovl_context *ctx;
    const ovl_zolo *zolo;
    const double *b_dev;   /* canonical, nrhs fields */
    double *x_dev;         /* canonical, overwritten */
    int32_t nrhs;
    ovl_stats *stats;      /* nrhs entries, may be null */
    int32_t status;        /* out */
    char message[160];     /* out: error text of this instance's solve */
} ovl_instance;
ovl_status ovl_sumr_gmresr_solve_many(ovl_instance *inst, int32_t n, const ovl_solver_params *params);

/* ---- eigenspace (eigSUMR basis; Secs. 4-5) ------------------------------ */

/* Number of vectors held (n after a diagonalisation), their Ritz values
 * (v, gamma_5 v^D) and residuals ||gamma_5 v^D - h v|| (host arrays of
 * capacity cap, may be null), and the number of diagonalisations so far. */
ovl_status ovl_eigspace_info(ovl_context *ctx, int32_t *n_held, int32_t cap, double *ritz_host,
                             double *resid_host, int32_t *n_diag);
/* Copy the held vectors v and v^D out (canonical, device, n_held fields each). */
ovl_status ovl_eigspace_get(ovl_context *ctx, double *v_dev, double *vD_dev);
/* Install k vectors v and their images v^D = D v (canonical, device) as the
 * eigSUMR basis for n wanted eigenvectors and mass mu (k <= m); clears the
 * diagonalisation history.  k = 0 empties the space. */
ovl_status ovl_eigspace_set(ovl_context *ctx, int32_t n, int32_t m, double mu, double delta, int32_t k,
                            const double *v_dev, const double *vD_dev);
/* Checkpoint of the eigenspace (the eigSUMR basis and its images, Secs. 4-5):
 * ovl_eigspace_save writes its configuration (n, m, mu, delta, eps, k_recalc),
 * the diagonalisation count, the recent max|UV| values of the Sec. 5.1
 * bound, the Ritz values and residuals, and the held vectors v and v^D (FP64,
 * canonical layout) to the file path_host, with the lattice extents;
 * ovl_eigspace_load reads such a file into a context of the same extents,
 * replacing its eigenspace (the sets kept for the three-set
 * re-diagonalisation are not saved: the next calculating solve starts them
 * again).  Deflation and further calculating solves continue from the loaded
 * state as from the saved one.  Errors: OVL_ERR_ARG for an unreadable,
 * truncated or foreign file or other extents, OVL_ERR_STATE when saving an
 * unconfigured eigenspace.  Both block until done. */
ovl_status ovl_eigspace_save(ovl_context *ctx, const char *path_host);
ovl_status ovl_eigspace_load(ovl_context *ctx, const char *path_host);
/* Run Alg. 6 on the held vectors now. */
ovl_status ovl_eigspace_diagonalise(ovl_context *ctx);
/* Recompute v^D = D v for the held vectors with FP64 sign accuracy eta. */
ovl_status ovl_eigspace_recompute(ovl_context *ctx, double rho, const ovl_zolo *zolo, double eta);
/* The standalone eigSUMR eigensolver (Sec. 6, eigenvector calculation; Algs.
 * 1, 5, 6, the Sec. 5.1 relaxation, the three-set re-diagonalisation of Sec. 5)
 * for the n_eig lowest eigenvectors of gamma_5 D[mu] (lowest in
 * D^+ D + 2 mu delta gamma_5 D), from the start vector q0_dev (canonical
 * complex128 [V][4][3], device, one field, not modified).  Used from params:
 * rho, mu, n_eig (3 n_eig <= 512), m_eig (> n_eig), eig_eps (target residual),
 * delta_split, norm_restart, k_recalc (in the Sec. 5.1 bound), relax_floor,
 * f32_threshold / half_threshold (the
 * precision of each sign call), max_mscg, verbose (one line per run).
 * Runs: each generates the Alg. 1 basis of U = gamma_5 sign(K) from its start
 * vector, collecting every (q, U q); it ends after diag_per_run
 * diagonalisations, when | ||q|| - 1 | > norm_restart or |gamma| >= 1, or when
 * every residual is at most the run's target; then Alg. 6, v^D recomputed to
 * 1e-12, and one Rayleigh-Ritz over the eigenvectors and those kept at the
 * previous two runs (canonically orthonormalised, directions below 1e-10 of
 * the largest Gram eigenvalue dropped).  The next run starts from the last q
 * orthogonalised against the eigenvectors, with the target max(eig_eps, 0.1 x
 * the largest residual).  Sign accuracy per application: the Sec. 5.1 bound,
 * never looser than relax_floor, when eta_fixed <= 0; else eta_fixed.  The eigenvectors are left in the
 * context's eigenspace (ovl_eigspace_info / _get; usable for deflation).
 * Host outputs (each may be null): runs_out; applies_hist[max_runs] and
 * maxres_hist[max_runs], the U applications so far and the largest residual
 * after each run; stats (one entry; sumr_iters = U applications).  Returns
 * OVL_OK when every residual reached eig_eps, OVL_ERR_NOT_CONVERGED after
 * max_runs runs, OVL_ERR_BREAKDOWN on a non-finite basis vector or when a run
 * ends before the first diagonalisation (fewer than n_eig + 1 vectors before
 * the norm test: lower n_eig).  Collection continues from the vectors the
 * eigenspace holds when n_eig, m_eig and mu match its configuration, else it
 * starts from an empty space. */
ovl_status ovl_eigsumr_eigensolve(ovl_context *ctx, const ovl_zolo *zolo, const ovl_solver_params *params,
                                  const double *q0_dev, int32_t max_runs, int32_t diag_per_run, double eta_fixed,
                                  int32_t *runs_out, int64_t *applies_hist, double *maxres_hist,
                                  ovl_stats *stats);
/* Sec. 4 deflated start: x0 = sum_j alpha_j psi'_j and D x0 = sum_j alpha_j D psi'_j,
 * alpha_j = (D psi'_j, b)/(D psi'_j, D psi'_j), over the held vectors rotated
 * so that (psi'_i, gamma_5 D psi'_j) is diagonal; nrhs fields (canonical). */
ovl_status ovl_deflate_project(ovl_context *ctx, const double *b_dev, double *x0_dev, double *Dx0_dev,
                               int32_t nrhs);

/* Per-kernel timing of the context for roofline reporting: while enabled,
 * each launch of the two hot kernels carries a pair of HIP events attached to
 * its dispatch packet (hipExtLaunchKernelGGL), which time the kernel's own
 * execution on the context's stream.  kernel: 0 = hopping stencil (all K /
 * Dslash launches), 1 = multi-shift update; prec selects the storage
 * precision.  bytes: the algorithmic HBM bytes of the timed launches.
 * Enabling (or disabling) resets the counts. */
ovl_status ovl_profile_enable(ovl_context *ctx, int32_t on);
ovl_status ovl_profile_read(ovl_context *ctx, int32_t kernel, int32_t prec, int64_t *launches,
                            double *milliseconds, double *bytes);

/* Streaming ceiling of the GPU's memory system for rooflines (not part of
 * the method): kind 0 copies bytes from src_dev to dst_dev, kind 1 reads
 * src_dev (dst_dev receives one 4-byte word per block: give it >= 64 KiB),
 * with 16-byte loads and stores over a grid of 16 blocks of 256 threads per
 * compute unit; bytes a multiple of 16, at least 16 MiB; buffers 16-byte
 * aligned, caller-owned device memory.  One untimed launch, then reps
 * launches on the context's stream timed by events: *ms_host = average
 * milliseconds per launch. */
ovl_status ovl_stream_bench(ovl_context *ctx, int32_t kind, const void *src_dev, void *dst_dev, int64_t bytes,
                            int32_t reps, double *ms_host);

/* Execution options of a context (value 0 = off, 1 = on):
 *   OVL_OPT_GRAPHS   (default off) the multi-shift CG replays a graph of four
 *                    iterations per chunk after the first chunk (off: every
 *                    kernel is launched on its own); results are identical.
 *                    Off by default: on MI355X the replays were slower than
 *                    direct launches for the 16^3x32 solve.
 *   OVL_OPT_AUTOTUNE (default on) time the stencil launch variants on first
 *                    use (off: a fixed variant).
 *   OVL_OPT_ADAPTIVE_NZ (default off) inside the solvers, each sign-function
 *                    call at accuracy eta uses the fewest Zolotarev poles n <= n_z
 *                    whose approximation error Delta(n) on the same interval
 *                    [a, b] is at most eta / 4, and gives the multi-shift CG the
 *                    rest, eta - Delta(n) (the error of a sign call is bounded by
 *                    the larger of Delta and the inversion error, Sec. 3).  Relaxed
 *                    calls then run fewer shifted systems with a larger smallest
 *                    shift; calls at tight accuracy keep all n_z poles.  Direct
 *                    calls of the sign function and the overlap operator through
 *                    this ABI always use the coefficients passed.
 *   OVL_OPT_BOUND_PRINTED (default off) the Sec. 5.1 eq. (bound) with chi
 *                    on the square root only, chi sqrt(eps^2 + r0^2) - r0, as the
 *                    equation is printed; off: chi (sqrt(eps^2 + r0^2) - r0), the
 *                    bound scaled by chi as the text describes.  For comparing
 *                    the two readings; the eigenvector relaxation only.
 *   OVL_OPT_TWO_ROW_LINKS (default on) the FP32 and FP16 stencils read 12 of
 *                    the 18 reals of each link and rebuild the third row as
 *                    the conjugate cross product of the first two, when every
 *                    loaded link passes the SU(3) test of ovl_gauge_info
 *                    (otherwise, or with the option off, the full links).
 *   OVL_OPT_OUTER_PRINTED (default off) the GMRESR outer product c = D u
 *                    (Alg. 3) to the accuracy the algorithm prints,
 *                    ||D u - c|| < eps ||b|| ||u|| / ||r||: the sign function
 *                    to 2 eps ||b|| / ((1 - mu) ||r||), looser as the outer
 *                    residual r falls; off: ||D u - c|| <= eps ||b|| / 4 at
 *                    every outer step. */
enum { OVL_OPT_GRAPHS = 1, OVL_OPT_AUTOTUNE = 2, OVL_OPT_ADAPTIVE_NZ = 3, OVL_OPT_BOUND_PRINTED = 4,
       OVL_OPT_TWO_ROW_LINKS = 5, OVL_OPT_OUTER_PRINTED = 6 };
ovl_status ovl_set_option(ovl_context *ctx, int32_t option, int32_t value);

/* The loaded links (Sec. 1, eq. 2: U_mu(x) in SU(3)).  *su3_deviation
 * receives the largest |U_2b - conj(U_0 x U_1)_b| over all links and entries,
 * computed in FP64 when the links were loaded; *two_row is 1 when the FP32
 * and FP16 stencils use the two-row form (deviation at most 2^-23 and
 * OVL_OPT_TWO_ROW_LINKS on), else 0.  Either pointer may be null.
 * OVL_ERR_STATE without links. */
ovl_status ovl_gauge_info(ovl_context *ctx, double *su3_deviation, int32_t *two_row);

/* Stencil launch shapes.  The first launch of each (precision, epilogue,
 * field count) times the launch variants on the context's lattice and keeps
 * the fastest (variant 0/1: one lane per site, lexicographic tiles in plain
 * or XCD-contiguous order; 2/3: two lanes per site, likewise; 4/5: one / two
 * lanes per site, each XCD walking one of eight xyz columns through t, when
 * the x, y, z extents split into 8 columns; 6/7: one / two lanes per xyz site,
 * each lane walking Lt/8 consecutive time slices with the time hops kept in
 * registers, one t chunk per XCD, when Lt is a multiple of 8; 8 .. 11: one
 * lane per site of a 256-site spatial tile whose spinors are shared through
 * LDS, each block walking T = 1, 2, 4, 8 time slices (FP32 and FP16 storage,
 * Lt a multiple of T); 12 .. 15: one / two lanes per site with each XCD
 * owning a contiguous eighth of the tiles, walked in groups of 32 (12, 13) or
 * 64 (14, 15) tiles with every field of the launch back to back inside a
 * group, so that a group's links are reused from that XCD's L2; 16 .. 19: as
 * 8 .. 11 with the tile's forward x, y, z links also staged in LDS; 20, FP16
 * storage only: one lane per site walking a group of four fields with the
 * site's eight links held in registers, links read once per tile and group;
 * 21, FP16 storage only: as 20 in the XCD column order of 4/5, the groups one
 * after another, when the x, y, z extents split into 8 columns).
 * A key is (precision * 8 + epilogue) * 64 + min(field count, 63), the
 * epilogue 0 for the plain hopping term; variants run 0 .. OVL_STENCIL_VARIANTS - 1.
 * ovl_tuning_get copies up to cap (key, variant) pairs and sets *n to the
 * number held; ovl_tuning_set installs pairs (a variant out of range or not
 * admissible on the context's lattice and precision is an argument error),
 * so a run can reuse another run's choices. */
enum { OVL_STENCIL_VARIANTS = 22 };
ovl_status ovl_tuning_get(ovl_context *ctx, int32_t *keys, int32_t *variants, int32_t cap, int32_t *n);
ovl_status ovl_tuning_set(ovl_context *ctx, const int32_t *keys, const int32_t *variants, int32_t n);

/* ---- allocation-free variant --------------------------------------------- */

/* Bytes of the library's fixed device scratch array: one per GPU, held from
 * the first ovl_create on that GPU until the process ends. */
#define OVL_NOALLOC_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same
 * operation as ovl_wilson_dslash (out = H in, nrhs canonical fields, device
 * in/out owned by the caller), with no hipMalloc, hipFree or other allocating
 * call.  The packed copies of in and out (and, for OVL_F32 / OVL_HALF, an FP64
 * staging field) live in the fixed scratch array, so
 *   2 * round256(S_prec * V * nrhs) + (prec != OVL_F64 ? round256(192 * V * nrhs) : 0)
 * must not exceed OVL_NOALLOC_SCRATCH_BYTES (S_prec = 192, 96, 52 bytes per
 * site for OVL_F64, OVL_F32, OVL_HALF), else OVL_ERR_ARG and no work.  The
 * context must hold a gauge field (ovl_gauge_load / _generate, which do
 * allocate, at set-up).  A stencil launch shape not yet timed by the context
 * is not timed here: the fixed shape is used (same values).  The array is
 * shared by every call on the GPU and keeps the last call's contents; calls
 * that overlap in time on one GPU race.  Asynchronous on the context's stream. */
ovl_status ovl_wilson_dslash_noalloc(ovl_context *ctx, const double *in_dev, double *out_dev, int32_t nrhs,
                                     int32_t prec);

#ifdef __cplusplus
}
#endif
#endif
