// Host drivers of the method's steps (each in its own .hip file).
#pragma once
#include "context.h"

namespace ovl {

// sign(K) in -> out, packed fields of precision prec (mscg.hip).
void sign_mscg(Context &c, double rho, const ovl_zolo &z, const void *in, void *out, int nf,
               double eta, int prec, int maxiter, ovl_stats *st);
// per-field accuracies eta[f]; eta[f] <= 0 skips field f (its output is unspecified)
void sign_mscg(Context &c, double rho, const ovl_zolo &z, const void *in, void *out, int nf,
               const double *eta, int prec, int maxiter, ovl_stats *st);

// Every shifted solution xs[l][f] = (K^2 + sigma_l)^{-1} in_f (shift-major,
// nf fields per shift), each to |zeta_l| ||r|| <= eta_f ||in_f||; FP64 or FP32.
void shifts_mscg(Context &c, double rho, const ovl_zolo &z, const void *in, void *xs, int nf, const double *eta,
                 int prec, int maxiter, ovl_stats *st);

// Derivatives of S = sum_f Re(chi_f^H D[mu] psi_f): dpsi = D^dagger chi (packed
// FP64, nullable) and the link gradient summed over fields into dU (canonical
// [V][4][3][3] complex, device, nullable) (adjoint.hip).
void overlap_adjoint(Context &c, double rho, double mu, const ovl_zolo &z, const double2 *psi, const double2 *chi,
                     double2 *dpsi, double2 *dU, int nf, double eta, int prec, int maxiter, ovl_stats *st);

// out = D[mu] in, packed FP64 in/out; the sign function in precision prec
// (conversions at its boundary) (solver.hip).
void overlap_f64(Context &c, double rho, double mu, const ovl_zolo &z, const double2 *in,
                 double2 *out, int nf, double eta, int prec, int maxiter, ovl_stats *st);

// sign(K) in -> out (packed FP64, nf fields) by the two-pass Lanczos method;
// z gives the interval [a, b] of |K| off the low modes (lanczos.hip).
void sign_lanczos(Context &c, double rho, const ovl_zolo &z, const double2 *in, double2 *out, int nf, double eta,
                  int maxiter, ovl_stats *st);

// Zolotarev coefficients (zolo.cpp).
void zolotarev(int nz, double a, double b, ovl_zolo &out);

// out = D[mu] in with per-field accuracies (eta[f] <= 0 skips field f).
void overlap_f64(Context &c, double rho, double mu, const ovl_zolo &z, const double2 *in, double2 *out,
                 int nf, const double *eta, int prec, int maxiter, ovl_stats *st);

// GMRESR(relSUMR) for nf right-hand sides solved together, packed FP64 b and
// x (nf contiguous fields); st has nf entries (solver.hip).
ovl_status solve_batch(Context &c, const ovl_zolo &z, const ovl_solver_params &p, const double2 *b,
                       double2 *x, int nf, ovl_stats *st);

// Kernel low modes (lowmodes.hip).
void lowmodes_compute(Context &c, double rho, int n_low, double tol, double *evals, double *lmax);
// Ends of the K^2 spectrum by Lanczos: sqrt of the smallest / largest Ritz
// values and the residual bound of the smallest (lowmodes.hip).
void kernel_interval(Context &c, double rho, int max_iter, double *lmin, double *lmin_err, double *lmax);

// eigSUMR and deflation (eigspace.hip).
void eig_configure(Context &c, int n, int m, double mu, double delta, double eps, int krecalc);
void eig_collect(Context &c, const double2 *q, const double2 *u);
void eig_collect_cg(Context &c, const double2 *w, const double2 *hw, const double2 *hhw);
void eig_diagonalise(Context &c);
void eig_rediagonalise_sets(Context &c);
ovl_status eig_eigensolve(Context &c, const ovl_zolo &z, const ovl_solver_params &prm, const double2 *q0,
                          int max_runs, int diag_per_run, double eta_fixed, int *runs_out, int64_t *applies_hist,
                          double *maxres_hist, ovl_stats *st);
double eig_sign_accuracy(const Context &c);
void eig_recompute(Context &c, double rho, const ovl_zolo &z, double eta, ovl_stats *st);
void eig_project(Context &c, const double2 *b, double2 *x0, double2 *Dx0);
// the spectral preconditioner of Sec. 4 from the held eigenspace
bool spectral_available(const Context &c);
void spectral_apply(Context &c, const double2 *v, double2 *out, int nf);

// Streaming ceiling of the memory system (stream.hip): average ms per launch
// of a 16-byte-word copy (kind 0) or read (kind 1) over bytes.
double stream_bench(Context &c, int kind, const void *src, void *dst, int64_t bytes, int reps);

// Generators (gen.hip).
void gauge_generate(Context &c, uint64_t seed, double eps, double *canon_out);
void source_generate(Context &c, int kind, uint64_t seed, int64_t site, int spin, int colour,
                     double *canon_out);

}  // namespace ovl
