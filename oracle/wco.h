/*
 * wco.h -- plain FP64 CPU oracle for the Wilson-Clover operator and its
 * solvers (test infrastructure only).
 *
 * This library is the checker of the HIP path, not part of it.  It shares no
 * code, header, table or helper with the GPU library; only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark load it.  Every
 * routine is a direct transcription of a textbook definition (cited per
 * function in wco.c) in double precision, with no blocking, fusion or
 * reordering beyond what the definition states.
 *
 * The paper (Boku et al., "A performance evaluation of CCS QCD Benchmark on
 * the COMA system", LATTICE2016) names the operator (Sec. 1 and Sec. 2:
 * even/odd preconditioned Wilson-Clover matrix), the solvers (Sec. 2: FP64
 * flexible BiCGStab, FP32 BiCGStab preconditioner with even/odd and
 * overlapped Restricted Additive Schwarz) but prints none of the formulas;
 * the readings used here are listed in the design notes of the repository.
 *
 * Conventions
 *   dims[4] = {Lx, Ly, Lz, Lt}, all even; site n = x + Lx*(y + Ly*(z + Lz*t)).
 *   Gauge field  U  : complex double [V][4][3][3] (row-major 3x3 per link).
 *   Spinor field    : complex double [V][4][3]    ([spin][colour]).
 *   Complex numbers are passed as interleaved (re, im) double pairs.
 *   tbc = +1 periodic, -1 antiperiodic in t for the fermion hops.
 *
 * Even/odd vectors are full-lattice vectors whose other-parity entries are
 * zero; parity(n) = (x+y+z+t) mod 2, "even" = 0.
 */
#ifndef WCO_H
#define WCO_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wco_ctx wco_ctx;

/* Copies U, builds the field strength F and the per-site inverse of T.
 * Returns NULL on bad arguments or when a site's T is singular. */
wco_ctx *wco_create(const int dims[4], int tbc, double kappa, double csw,
                    const double *U);
void wco_destroy(wco_ctx *c);
long wco_volume(const wco_ctx *c);
int  wco_set_threads(int n);   /* OpenMP threads for the site loops (0 = default) */

/* Elementary operators on full-lattice spinors. */
void wco_hop(const wco_ctx *c, const double *in, double *out);        /* H psi        */
void wco_clover(const wco_ctx *c, const double *in, double *out);     /* T psi        */
void wco_clover_inv(const wco_ctx *c, const double *in, double *out); /* T^-1 psi     */
void wco_clover_C(const wco_ctx *c, const double *in, double *out);   /* sum sigma(x)F */
void wco_D(const wco_ctx *c, const double *in, double *out, int dagger); /* D or D^dag */
void wco_field_strength(const wco_ctx *c, double *F);  /* F[V][6][3][3], planes 01,02,03,12,13,23 */
void wco_clover_matrix(const wco_ctx *c, double *T);   /* T[V][12][12], index s*3+c */
void wco_clover_inv_matrix(const wco_ctx *c, double *Ti);

/* Even/odd Schur complement (left T_ee^-1 form). */
void wco_schur(const wco_ctx *c, const double *xe, double *out);
void wco_schur_rhs(const wco_ctx *c, const double *b, double *bhat);
void wco_reconstruct(const wco_ctx *c, const double *b, const double *xe, double *x);

/* Overlapped restricted additive Schwarz (one application) on even vectors.
 * solver 0: minimal residual steps from z = 0; solver 1: the linear block
 * Jacobi (Richardson) steps z <- z + (r_B - Dhat_B z) from z = 0; solver 2:
 * `iters` BiCGStab iterations (two block applications each) from z = 0. */
int wco_ras(const wco_ctx *c, const int block[4], int overlap, int iters, int solver,
            const double *in, double *out);
/* Multiplicative Schwarz on even vectors: the 16 block colours (parities of
 * the block coordinates) in turn, each on the residual v - Dhat z left by the
 * previous colours, same block solver and restriction as wco_ras. */
int wco_sap(const wco_ctx *c, const int block[4], int overlap, int iters, int solver,
            const double *in, double *out);

/* Solvers; return 0 on convergence, 1 if max iterations hit, 2 on breakdown.
 * iters_out / relres_out receive the iteration count and the final true
 * relative residual ||b - D x|| / ||b|| of the full system. */
int wco_bicgstab_full(const wco_ctx *c, const double *b, double *x, double tol,
                      int maxiter, int *iters_out, double *relres_out);
int wco_bicgstab_eo(const wco_ctx *c, const double *b, double *x, double tol,
                    int maxiter, int *iters_out, double *relres_out);
/* Right-preconditioned BiCGStab on the Schur operator (the inner solver),
 * preconditioner = RAS when use_ras, relative-residual stop at stol. */
int wco_inner_bicgstab(const wco_ctx *c, const double *rhs, double *xe, double stol,
                       int maxiter, int use_ras, const int block[4], int overlap,
                       int ras_iters, int *iters_out);
/* Flexible BiCGStab (outer) with the inner solve as preconditioner. */
int wco_fbicgstab(const wco_ctx *c, const double *b, double *x, double tol,
                  int max_outer, double inner_tol, int max_inner, int use_ras,
                  const int block[4], int overlap, int ras_iters,
                  int *outer_out, int *inner_total_out, double *relres_out);

/* Gradient of L = Re<eta, D^-1 b> given x = D^-1 b and y = D^-dag eta:
 * gU[V][4][3][3] (complex, PyTorch convention 2 dL/d conj(U)), *gkappa. */
void wco_grad(const wco_ctx *c, const double *x, const double *y,
              double *gU, double *gkappa);

#ifdef __cplusplus
}
#endif
#endif
