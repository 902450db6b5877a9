/*
 * wco.c -- plain FP64 CPU oracle for the Wilson-Clover operator (test
 * infrastructure: only the tests, the smoke check and the benchmark's CPU
 * baseline use it; the HIP library never links or calls it).
 *
 * The paper names the operator and the solver structure (Sec. 1: Wilson-Clover
 * quark propagator, single-precision BiCGStab preconditioner with overlapped
 * RAS; Sec. 2: even/odd site preconditioned Wilson-Clover matrix, FP64
 * flexible BiCGStab outer, FP32 BiCGStab inner with even/odd and RAS
 * preconditioning) without printing the formulas.  The definitions below are
 * the textbook ones; every convention the paper leaves open is a stated
 * reading (gamma basis, hop projector signs, clover normalisation, Schur form,
 * Schwarz block solver), recorded in the repository's design notes.
 *
 * Style: whole 4x4 spin matrices and whole 3x3 colour matrices, one site at a
 * time, no half-spinor projection, no packing, no fusion.
 */
#include "wco.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double _Complex cplx;

struct wco_ctx {
    int L[4];
    long V;
    int tbc;
    double kappa, csw;
    cplx *U;   /* [V][4][3][3] */
    cplx *F;   /* [V][6][3][3] */
    cplx *Ti;  /* [V][12][12]  */
};

/* ---------------------------------------------------------------------------
 * Dirac matrices, chiral basis (the paper does not state its basis).
 * gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] for k = x, y, z and
 * gamma_t = [[0, 1], [1, 0]]; written out entry by entry.
 * ------------------------------------------------------------------------- */
static cplx GAM[4][4][4];
static cplx GAM5[4][4];
static cplx SIG[6][4][4];                 /* sigma_{mu nu} = (i/2)[g_mu, g_nu] */
static const int PMU[6] = {0, 0, 0, 1, 1, 2};
static const int PNU[6] = {1, 2, 3, 2, 3, 3};
static int gamma_ready = 0;

static void init_gamma(void)
{
    if (gamma_ready) return;
    const cplx J = _Complex_I;
    memset(GAM, 0, sizeof(GAM));
    /* gamma_x */
    GAM[0][0][3] = -J; GAM[0][1][2] = -J; GAM[0][2][1] = J;  GAM[0][3][0] = J;
    /* gamma_y */
    GAM[1][0][3] = -1; GAM[1][1][2] = 1;  GAM[1][2][1] = 1;  GAM[1][3][0] = -1;
    /* gamma_z */
    GAM[2][0][2] = -J; GAM[2][1][3] = J;  GAM[2][2][0] = J;  GAM[2][3][1] = -J;
    /* gamma_t */
    GAM[3][0][2] = 1;  GAM[3][1][3] = 1;  GAM[3][2][0] = 1;  GAM[3][3][1] = 1;

    /* gamma_5 = gamma_x gamma_y gamma_z gamma_t */
    cplx a[4][4], b[4][4];
    memcpy(a, GAM[0], sizeof(a));
    for (int m = 1; m < 4; m++) {
        for (int i = 0; i < 4; i++)
            for (int j = 0; j < 4; j++) {
                cplx s = 0;
                for (int k = 0; k < 4; k++) s += a[i][k] * GAM[m][k][j];
                b[i][j] = s;
            }
        memcpy(a, b, sizeof(a));
    }
    memcpy(GAM5, a, sizeof(a));

    for (int p = 0; p < 6; p++) {
        const int mu = PMU[p], nu = PNU[p];
        for (int i = 0; i < 4; i++)
            for (int j = 0; j < 4; j++) {
                cplx s = 0;
                for (int k = 0; k < 4; k++)
                    s += GAM[mu][i][k] * GAM[nu][k][j] - GAM[nu][i][k] * GAM[mu][k][j];
                SIG[p][i][j] = 0.5 * J * s;
            }
    }
    gamma_ready = 1;
}

/* ---------------------------------------------------------------------------
 * Lattice geometry: lexicographic site index, periodic wrap, and the fermion
 * boundary sign (tbc on the hop that crosses t = Lt-1 <-> 0).
 * ------------------------------------------------------------------------- */
static void coords(const wco_ctx *c, long n, int x[4])
{
    for (int mu = 0; mu < 4; mu++) {
        x[mu] = (int)(n % c->L[mu]);
        n /= c->L[mu];
    }
}

static long index_of(const wco_ctx *c, const int x[4])
{
    return x[0] + (long)c->L[0] * (x[1] + (long)c->L[1] * (x[2] + (long)c->L[2] * x[3]));
}

static long nb(const wco_ctx *c, long n, int mu, int dir)
{
    int x[4];
    coords(c, n, x);
    x[mu] = (x[mu] + dir + c->L[mu]) % c->L[mu];
    return index_of(c, x);
}

static double bc_sign(const wco_ctx *c, long n, int mu, int dir)
{
    if (mu != 3 || c->tbc == 1) return 1.0;
    int x[4];
    coords(c, n, x);
    if (dir > 0 && x[3] == c->L[3] - 1) return (double)c->tbc;
    if (dir < 0 && x[3] == 0) return (double)c->tbc;
    return 1.0;
}

static int parity(const wco_ctx *c, long n)
{
    int x[4];
    coords(c, n, x);
    return (x[0] + x[1] + x[2] + x[3]) & 1;
}

static const cplx *link(const wco_ctx *c, long n, int mu) { return c->U + (n * 4 + mu) * 9; }

/* 3x3 complex helpers (row-major). */
static void m3_mul(const cplx *A, const cplx *B, cplx *C)
{
    cplx t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            cplx s = 0;
            for (int k = 0; k < 3; k++) s += A[i * 3 + k] * B[k * 3 + j];
            t[i * 3 + j] = s;
        }
    memcpy(C, t, sizeof(t));
}

static void m3_dag(const cplx *A, cplx *C)
{
    cplx t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) t[i * 3 + j] = conj(A[j * 3 + i]);
    memcpy(C, t, sizeof(t));
}

/* ---------------------------------------------------------------------------
 * Wilson hopping term, r = 1:
 *   (H psi)(x) = sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                       + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]
 * with the t-boundary sign on hops that cross the t boundary.
 * ------------------------------------------------------------------------- */
static void hop_site(const wco_ctx *c, const cplx *in, long n, cplx *out)
{
    for (int i = 0; i < 12; i++) out[i] = 0;
    for (int mu = 0; mu < 4; mu++) {
        for (int dir = +1; dir >= -1; dir -= 2) {
            const long m = nb(c, n, mu, dir);
            const double s = bc_sign(c, n, mu, dir);
            cplx t[4][3];
            if (dir > 0) {
                const cplx *u = link(c, n, mu);
                for (int sp = 0; sp < 4; sp++)
                    for (int a = 0; a < 3; a++) {
                        cplx acc = 0;
                        for (int b = 0; b < 3; b++) acc += u[a * 3 + b] * in[m * 12 + sp * 3 + b];
                        t[sp][a] = acc;
                    }
            } else {
                const cplx *u = link(c, m, mu);
                for (int sp = 0; sp < 4; sp++)
                    for (int a = 0; a < 3; a++) {
                        cplx acc = 0;
                        for (int b = 0; b < 3; b++) acc += conj(u[b * 3 + a]) * in[m * 12 + sp * 3 + b];
                        t[sp][a] = acc;
                    }
            }
            /* projector 1 - gamma (forward) or 1 + gamma (backward) */
            const double pg = -(double)dir;
            for (int sp = 0; sp < 4; sp++)
                for (int a = 0; a < 3; a++) {
                    cplx acc = 0;
                    for (int q = 0; q < 4; q++)
                        acc += ((sp == q ? 1.0 : 0.0) + pg * GAM[mu][sp][q]) * t[q][a];
                    out[sp * 3 + a] += s * acc;
                }
        }
    }
}

static void hop_all(const wco_ctx *c, const cplx *in, cplx *out)
{
#pragma omp parallel for schedule(static)
    for (long n = 0; n < c->V; n++) hop_site(c, in, n, out + n * 12);
}

void wco_hop(const wco_ctx *c, const double *in, double *out)
{
    hop_all(c, (const cplx *)in, (cplx *)out);
}

/* ---------------------------------------------------------------------------
 * Clover term (Sheikholeslami-Wohlert).
 *   Q_{mu nu}(x): sum of the four plaquette leaves around x,
 *   F_{mu nu} = (Q - Q^dag) / (8i), made traceless,
 *   T = 1 - c_sw kappa sum_{mu<nu} sigma_{mu nu} (x) F_{mu nu}.
 * The leaves use the links as given (no boundary sign).
 * ------------------------------------------------------------------------- */
static void leaf_product(const cplx *A, int da, const cplx *B, int db, const cplx *C, int dc,
                         const cplx *D, int dd, cplx *out)
{
    cplx a[9], b[9], cc[9], d[9];
    if (da) m3_dag(A, a); else memcpy(a, A, sizeof(a));
    if (db) m3_dag(B, b); else memcpy(b, B, sizeof(b));
    if (dc) m3_dag(C, cc); else memcpy(cc, C, sizeof(cc));
    if (dd) m3_dag(D, d); else memcpy(d, D, sizeof(d));
    m3_mul(a, b, out);
    m3_mul(out, cc, out);
    m3_mul(out, d, out);
}

/* The four leaves of the clover at x in plane (mu, nu), each as an ordered
 * product of four links: site index and dagger flag per factor. */
static void leaves(const wco_ctx *c, long x, int mu, int nu, long site[4][4], int dag[4][4],
                   int dirn[4][4])
{
    const long xpm = nb(c, x, mu, +1), xpn = nb(c, x, nu, +1);
    const long xmm = nb(c, x, mu, -1), xmn = nb(c, x, nu, -1);
    const long xmm_pn = nb(c, xmm, nu, +1), xmm_mn = nb(c, xmm, nu, -1);
    const long xpm_mn = nb(c, xpm, nu, -1);
    /* leaf 1: U_mu(x) U_nu(x+mu) U_mu(x+nu)^dag U_nu(x)^dag */
    long s1[4] = {x, xpm, xpn, x};         int d1[4] = {0, 0, 1, 1}; int m1[4] = {mu, nu, mu, nu};
    /* leaf 2: U_nu(x) U_mu(x-mu+nu)^dag U_nu(x-mu)^dag U_mu(x-mu) */
    long s2[4] = {x, xmm_pn, xmm, xmm};    int d2[4] = {0, 1, 1, 0}; int m2[4] = {nu, mu, nu, mu};
    /* leaf 3: U_mu(x-mu)^dag U_nu(x-mu-nu)^dag U_mu(x-mu-nu) U_nu(x-nu) */
    long s3[4] = {xmm, xmm_mn, xmm_mn, xmn}; int d3[4] = {1, 1, 0, 0}; int m3[4] = {mu, nu, mu, nu};
    /* leaf 4: U_nu(x-nu)^dag U_mu(x-nu) U_nu(x+mu-nu) U_mu(x)^dag */
    long s4[4] = {xmn, xmn, xpm_mn, x};    int d4[4] = {1, 0, 0, 1}; int m4[4] = {nu, mu, nu, mu};
    for (int k = 0; k < 4; k++) {
        site[0][k] = s1[k]; dag[0][k] = d1[k]; dirn[0][k] = m1[k];
        site[1][k] = s2[k]; dag[1][k] = d2[k]; dirn[1][k] = m2[k];
        site[2][k] = s3[k]; dag[2][k] = d3[k]; dirn[2][k] = m3[k];
        site[3][k] = s4[k]; dag[3][k] = d4[k]; dirn[3][k] = m4[k];
    }
}

static void field_strength_site(const wco_ctx *c, long x, cplx *F /* [6][9] */)
{
    const cplx J = _Complex_I;
    for (int p = 0; p < 6; p++) {
        long site[4][4];
        int dag[4][4], dirn[4][4];
        leaves(c, x, PMU[p], PNU[p], site, dag, dirn);
        cplx Q[9] = {0};
        for (int l = 0; l < 4; l++) {
            cplx P[9];
            leaf_product(link(c, site[l][0], dirn[l][0]), dag[l][0],
                         link(c, site[l][1], dirn[l][1]), dag[l][1],
                         link(c, site[l][2], dirn[l][2]), dag[l][2],
                         link(c, site[l][3], dirn[l][3]), dag[l][3], P);
            for (int k = 0; k < 9; k++) Q[k] += P[k];
        }
        cplx *f = F + p * 9;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) f[a * 3 + b] = (Q[a * 3 + b] - conj(Q[b * 3 + a])) / (8.0 * J);
        const cplx tr = (f[0] + f[4] + f[8]) / 3.0;
        f[0] -= tr; f[4] -= tr; f[8] -= tr;
    }
}

/* out = sum_p (sigma_p (x) F_p) in   at one site */
static void sigmaF_site(const cplx *F, const cplx *in, cplx *out)
{
    for (int i = 0; i < 12; i++) out[i] = 0;
    for (int p = 0; p < 6; p++)
        for (int s = 0; s < 4; s++)
            for (int a = 0; a < 3; a++) {
                cplx acc = 0;
                for (int t = 0; t < 4; t++)
                    for (int b = 0; b < 3; b++) acc += SIG[p][s][t] * F[p * 9 + a * 3 + b] * in[t * 3 + b];
                out[s * 3 + a] += acc;
            }
}

static void clover_site(const wco_ctx *c, long n, const cplx *in, cplx *out)
{
    cplx t[12];
    sigmaF_site(c->F + n * 54, in, t);
    const double ck = c->csw * c->kappa;
    for (int i = 0; i < 12; i++) out[i] = in[i] - ck * t[i];
}

void wco_clover(const wco_ctx *c, const double *in, double *out)
{
    const cplx *ci = (const cplx *)in;
    cplx *co = (cplx *)out;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < c->V; n++) clover_site(c, n, ci + n * 12, co + n * 12);
}

void wco_clover_C(const wco_ctx *c, const double *in, double *out)
{
    const cplx *ci = (const cplx *)in;
    cplx *co = (cplx *)out;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < c->V; n++) sigmaF_site(c->F + n * 54, ci + n * 12, co + n * 12);
}

static void clover_matrix_site(const wco_ctx *c, long n, cplx *T /* [12][12] */)
{
    const double ck = c->csw * c->kappa;
    const cplx *F = c->F + n * 54;
    for (int s = 0; s < 4; s++)
        for (int a = 0; a < 3; a++)
            for (int t = 0; t < 4; t++)
                for (int b = 0; b < 3; b++) {
                    cplx acc = 0;
                    for (int p = 0; p < 6; p++) acc += SIG[p][s][t] * F[p * 9 + a * 3 + b];
                    T[(s * 3 + a) * 12 + t * 3 + b] = ((s == t && a == b) ? 1.0 : 0.0) - ck * acc;
                }
}

/* Gauss-Jordan elimination with partial pivoting; returns 0 if singular. */
static int invert12(const cplx *A, cplx *Ainv)
{
    cplx M[12][24];
    for (int i = 0; i < 12; i++)
        for (int j = 0; j < 12; j++) {
            M[i][j] = A[i * 12 + j];
            M[i][12 + j] = (i == j) ? 1.0 : 0.0;
        }
    for (int col = 0; col < 12; col++) {
        int piv = col;
        double best = cabs(M[col][col]);
        for (int r = col + 1; r < 12; r++)
            if (cabs(M[r][col]) > best) { best = cabs(M[r][col]); piv = r; }
        if (best == 0.0) return 0;
        if (piv != col)
            for (int j = 0; j < 24; j++) { cplx t = M[col][j]; M[col][j] = M[piv][j]; M[piv][j] = t; }
        const cplx d = M[col][col];
        for (int j = 0; j < 24; j++) M[col][j] /= d;
        for (int r = 0; r < 12; r++) {
            if (r == col) continue;
            const cplx f = M[r][col];
            if (f == 0) continue;
            for (int j = 0; j < 24; j++) M[r][j] -= f * M[col][j];
        }
    }
    for (int i = 0; i < 12; i++)
        for (int j = 0; j < 12; j++) Ainv[i * 12 + j] = M[i][12 + j];
    return 1;
}

static void mat12_site(const cplx *M, const cplx *in, cplx *out)
{
    for (int i = 0; i < 12; i++) {
        cplx acc = 0;
        for (int j = 0; j < 12; j++) acc += M[i * 12 + j] * in[j];
        out[i] = acc;
    }
}

void wco_clover_inv(const wco_ctx *c, const double *in, double *out)
{
    const cplx *ci = (const cplx *)in;
    cplx *co = (cplx *)out;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < c->V; n++) mat12_site(c->Ti + n * 144, ci + n * 12, co + n * 12);
}

void wco_field_strength(const wco_ctx *c, double *F) { memcpy(F, c->F, sizeof(cplx) * 54 * c->V); }

void wco_clover_matrix(const wco_ctx *c, double *T)
{
    cplx *t = (cplx *)T;
    for (long n = 0; n < c->V; n++) clover_matrix_site(c, n, t + n * 144);
}

void wco_clover_inv_matrix(const wco_ctx *c, double *Ti) { memcpy(Ti, c->Ti, sizeof(cplx) * 144 * c->V); }

/* ---------------------------------------------------------------------------
 * Full operator D = T - kappa H;  D^dag = gamma5 D gamma5.
 * ------------------------------------------------------------------------- */
static void gamma5_apply(const wco_ctx *c, const cplx *in, cplx *out)
{
    for (long n = 0; n < c->V; n++)
        for (int s = 0; s < 4; s++)
            for (int a = 0; a < 3; a++) {
                cplx acc = 0;
                for (int t = 0; t < 4; t++) acc += GAM5[s][t] * in[n * 12 + t * 3 + a];
                out[n * 12 + s * 3 + a] = acc;
            }
}

static void D_plain(const wco_ctx *c, const cplx *in, cplx *out)
{
#pragma omp parallel for schedule(static)
    for (long n = 0; n < c->V; n++) {
        cplx h[12], t[12];
        hop_site(c, in, n, h);
        clover_site(c, n, in + n * 12, t);
        for (int i = 0; i < 12; i++) out[n * 12 + i] = t[i] - c->kappa * h[i];
    }
}

void wco_D(const wco_ctx *c, const double *in, double *out, int dagger)
{
    const cplx *ci = (const cplx *)in;
    cplx *co = (cplx *)out;
    if (!dagger) {
        D_plain(c, ci, co);
        return;
    }
    cplx *a = malloc(sizeof(cplx) * 12 * c->V), *b = malloc(sizeof(cplx) * 12 * c->V);
    gamma5_apply(c, ci, a);
    D_plain(c, a, b);
    gamma5_apply(c, b, co);
    free(a);
    free(b);
}

/* ---------------------------------------------------------------------------
 * Vector helpers (sequential, fixed order).
 * ------------------------------------------------------------------------- */
static cplx vdot(long N, const cplx *a, const cplx *b)
{
    cplx s = 0;
    for (long i = 0; i < N; i++) s += conj(a[i]) * b[i];
    return s;
}

static double vnorm(long N, const cplx *a) { return sqrt(creal(vdot(N, a, a))); }

static void mask_parity(const wco_ctx *c, cplx *v, int keep)
{
    for (long n = 0; n < c->V; n++)
        if (parity(c, n) != keep)
            for (int i = 0; i < 12; i++) v[n * 12 + i] = 0;
}

static cplx *vnew(const wco_ctx *c) { return calloc((size_t)c->V * 12, sizeof(cplx)); }

/* ---------------------------------------------------------------------------
 * Even/odd decomposition.
 *   D = [[T_ee, -k H_eo], [-k H_oe, T_oo]]
 *   Dhat = 1 - k^2 T_ee^-1 H_eo T_oo^-1 H_oe      (on even sites)
 *   bhat = T_ee^-1 (b_e + k H_eo T_oo^-1 b_o)
 *   x_o  = T_oo^-1 (b_o + k H_oe x_e)
 * ------------------------------------------------------------------------- */
static void schur_plain(const wco_ctx *c, const cplx *xe_in, cplx *out)
{
    cplx *xe = vnew(c), *t1 = vnew(c), *t2 = vnew(c);
    memcpy(xe, xe_in, sizeof(cplx) * 12 * c->V);
    mask_parity(c, xe, 0);
    hop_all(c, xe, t1);
    mask_parity(c, t1, 1);
    wco_clover_inv(c, (double *)t1, (double *)t2);
    mask_parity(c, t2, 1);
    hop_all(c, t2, t1);
    mask_parity(c, t1, 0);
    wco_clover_inv(c, (double *)t1, (double *)t2);
    const double k2 = c->kappa * c->kappa;
    for (long i = 0; i < 12 * c->V; i++) out[i] = xe[i] - k2 * t2[i];
    mask_parity(c, out, 0);
    free(xe); free(t1); free(t2);
}

void wco_schur(const wco_ctx *c, const double *xe, double *out)
{
    schur_plain(c, (const cplx *)xe, (cplx *)out);
}

void wco_schur_rhs(const wco_ctx *c, const double *b, double *bhat)
{
    cplx *bo = vnew(c), *t1 = vnew(c), *t2 = vnew(c);
    memcpy(bo, b, sizeof(cplx) * 12 * c->V);
    mask_parity(c, bo, 1);
    wco_clover_inv(c, (double *)bo, (double *)t1);
    mask_parity(c, t1, 1);
    hop_all(c, t1, t2);
    mask_parity(c, t2, 0);
    const cplx *cb = (const cplx *)b;
    for (long i = 0; i < 12 * c->V; i++) t1[i] = cb[i] + c->kappa * t2[i];
    mask_parity(c, t1, 0);
    wco_clover_inv(c, (double *)t1, bhat);
    mask_parity(c, (cplx *)bhat, 0);
    free(bo); free(t1); free(t2);
}

void wco_reconstruct(const wco_ctx *c, const double *b, const double *xe_in, double *x)
{
    cplx *xe = vnew(c), *t1 = vnew(c), *t2 = vnew(c);
    memcpy(xe, xe_in, sizeof(cplx) * 12 * c->V);
    mask_parity(c, xe, 0);
    hop_all(c, xe, t1);
    const cplx *cb = (const cplx *)b;
    for (long i = 0; i < 12 * c->V; i++) t2[i] = cb[i] + c->kappa * t1[i];
    mask_parity(c, t2, 1);
    wco_clover_inv(c, (double *)t2, (double *)t1);
    mask_parity(c, t1, 1);
    cplx *cx = (cplx *)x;
    for (long i = 0; i < 12 * c->V; i++) cx[i] = xe[i] + t1[i];
    free(xe); free(t1); free(t2);
}

/* ---------------------------------------------------------------------------
 * Context.
 * ------------------------------------------------------------------------- */
long wco_volume(const wco_ctx *c) { return c->V; }

int wco_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

wco_ctx *wco_create(const int dims[4], int tbc, double kappa, double csw, const double *U)
{
    init_gamma();
    if (!dims || !U || (tbc != 1 && tbc != -1)) return NULL;
    for (int mu = 0; mu < 4; mu++)
        if (dims[mu] < 2 || (dims[mu] & 1)) return NULL;
    wco_ctx *c = calloc(1, sizeof(*c));
    memcpy(c->L, dims, sizeof(c->L));
    c->V = (long)dims[0] * dims[1] * dims[2] * dims[3];
    c->tbc = tbc;
    c->kappa = kappa;
    c->csw = csw;
    c->U = malloc(sizeof(cplx) * 36 * c->V);
    c->F = malloc(sizeof(cplx) * 54 * c->V);
    c->Ti = malloc(sizeof(cplx) * 144 * c->V);
    if (!c->U || !c->F || !c->Ti) { wco_destroy(c); return NULL; }
    memcpy(c->U, U, sizeof(cplx) * 36 * c->V);
    int ok = 1;
#pragma omp parallel for schedule(static) reduction(&& : ok)
    for (long n = 0; n < c->V; n++) {
        field_strength_site(c, n, c->F + n * 54);
        cplx T[144];
        clover_matrix_site(c, n, T);
        ok = ok && invert12(T, c->Ti + n * 144);
    }
    if (!ok) { wco_destroy(c); return NULL; }
    return c;
}

void wco_destroy(wco_ctx *c)
{
    if (!c) return;
    free(c->U); free(c->F); free(c->Ti);
    free(c);
}

/* ---------------------------------------------------------------------------
 * Plain BiCGStab (van der Vorst 1992) on the full D, zero start, with
 * residual replacement by the true residual when the recursive one passes
 * the threshold.
 * ------------------------------------------------------------------------- */
typedef void (*op_fn)(const wco_ctx *, const cplx *, cplx *);

static void op_D(const wco_ctx *c, const cplx *in, cplx *out) { D_plain(c, in, out); }
static void op_schur(const wco_ctx *c, const cplx *in, cplx *out) { schur_plain(c, in, out); }

static int bicgstab(const wco_ctx *c, op_fn A, const cplx *b, cplx *x, double tol, int maxiter,
                    double (*true_res)(const wco_ctx *, const cplx *, const cplx *, cplx *),
                    const cplx *b_full, int *iters_out, double *relres_out)
{
    const long N = 12 * c->V;
    cplx *r = vnew(c), *rt = vnew(c), *p = vnew(c), *v = vnew(c), *s = vnew(c), *t = vnew(c);
    const double bn = vnorm(N, b);
    int status = 1, it = 0;
    double relres = 0.0;
    memset(x, 0, sizeof(cplx) * N);
    if (bn == 0.0) { status = 0; goto done; }
    memcpy(r, b, sizeof(cplx) * N);
    memcpy(rt, r, sizeof(cplx) * N);
    cplx rho = 1, alpha = 1, omega = 1;
    for (it = 1; it <= maxiter; it++) {
        const cplx rho1 = vdot(N, rt, r);
        if (cabs(rho1) == 0.0) { status = 2; break; }
        const cplx beta = (rho1 / rho) * (alpha / omega);
        for (long i = 0; i < N; i++) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        A(c, p, v);
        const cplx rtv = vdot(N, rt, v);
        if (cabs(rtv) == 0.0) { status = 2; break; }
        alpha = rho1 / rtv;
        for (long i = 0; i < N; i++) s[i] = r[i] - alpha * v[i];
        A(c, s, t);
        const double tt = creal(vdot(N, t, t));
        omega = (tt == 0.0) ? 0.0 : vdot(N, t, s) / tt;
        for (long i = 0; i < N; i++) x[i] += alpha * p[i] + omega * s[i];
        for (long i = 0; i < N; i++) r[i] = s[i] - omega * t[i];
        rho = rho1;
        if (vnorm(N, r) <= tol * bn) {
            /* the true residual decides; replace the recursive one if needed */
            relres = true_res(c, b_full, x, r);
            if (relres <= tol) { status = 0; break; }
            if (omega == 0.0) { status = 2; break; }
        }
    }
    if (it > maxiter) it = maxiter;
    if (status != 0) relres = true_res(c, b_full, x, r);
done:
    *iters_out = it;
    *relres_out = relres;
    free(r); free(rt); free(p); free(v); free(s); free(t);
    return status;
}

/* r = b - D x on the full lattice; returns ||r|| / ||b|| */
static double true_res_full(const wco_ctx *c, const cplx *b, const cplx *x, cplx *r)
{
    const long N = 12 * c->V;
    D_plain(c, x, r);
    for (long i = 0; i < N; i++) r[i] = b[i] - r[i];
    return vnorm(N, r) / vnorm(N, b);
}

int wco_bicgstab_full(const wco_ctx *c, const double *b, double *x, double tol, int maxiter,
                      int *iters_out, double *relres_out)
{
    return bicgstab(c, op_D, (const cplx *)b, (cplx *)x, tol, maxiter, true_res_full,
                    (const cplx *)b, iters_out, relres_out);
}

/* For the Schur system: the stopping test is on the full system, so the
 * residual replacement reconstructs x and measures b - D x, then hands back
 * the Schur residual bhat - Dhat x_e in r.  The caller's b is passed through
 * a static slot because the plain BiCGStab above sees only bhat. */
static const cplx *g_bhat;
static double true_res_schur(const wco_ctx *c, const cplx *b, const cplx *xe, cplx *r)
{
    const long N = 12 * c->V;
    cplx *x = vnew(c), *rf = vnew(c);
    wco_reconstruct(c, (const double *)b, (const double *)xe, (double *)x);
    const double rel = true_res_full(c, b, x, rf);
    schur_plain(c, xe, r);
    for (long i = 0; i < N; i++) r[i] = g_bhat[i] - r[i];
    free(x); free(rf);
    return rel;
}

int wco_bicgstab_eo(const wco_ctx *c, const double *b, double *x, double tol, int maxiter,
                    int *iters_out, double *relres_out)
{
    cplx *bh = vnew(c), *xe = vnew(c);
    wco_schur_rhs(c, b, (double *)bh);
    g_bhat = bh;
    const int st = bicgstab(c, op_schur, bh, xe, tol, maxiter, true_res_schur, (const cplx *)b,
                            iters_out, relres_out);
    g_bhat = NULL;
    wco_reconstruct(c, b, (const double *)xe, x);
    free(bh); free(xe);
    return st;
}

/* ---------------------------------------------------------------------------
 * Overlapped Restricted Additive Schwarz.  Cores: hypercubes of size
 * block[mu] with origins at multiples of block[mu]; each core is extended by
 * `overlap` sites on both sides.  The block operator is the Schur complement
 * of D restricted to the extended block with every hop leaving the block
 * dropped (Dirichlet cut); the block system is solved approximately by
 * `iters` minimal-residual steps from zero; the solution is kept on the even
 * sites of the core only.
 * ------------------------------------------------------------------------- */
typedef struct {
    int e[4];      /* extended extents */
    long Ne;       /* sites in the extended block */
    long *g;       /* local -> global site */
} blockmap;

static long lidx(const blockmap *B, const int a[4])
{
    return a[0] + (long)B->e[0] * (a[1] + (long)B->e[1] * (a[2] + (long)B->e[2] * a[3]));
}

static void lcoords(const blockmap *B, long l, int a[4])
{
    for (int mu = 0; mu < 4; mu++) { a[mu] = (int)(l % B->e[mu]); l /= B->e[mu]; }
}

/* Block hop: only neighbour pairs inside the extended block contribute. */
static void block_hop(const wco_ctx *c, const blockmap *B, const cplx *in, cplx *out)
{
    for (long l = 0; l < B->Ne; l++) {
        int a[4];
        lcoords(B, l, a);
        const long n = B->g[l];
        cplx *o = out + l * 12;
        for (int i = 0; i < 12; i++) o[i] = 0;
        for (int mu = 0; mu < 4; mu++)
            for (int dir = +1; dir >= -1; dir -= 2) {
                int b[4] = {a[0], a[1], a[2], a[3]};
                b[mu] += dir;
                if (b[mu] < 0 || b[mu] >= B->e[mu]) continue;
                const long lm = lidx(B, b);
                const long m = B->g[lm];
                const double s = bc_sign(c, n, mu, dir);
                const cplx *u = (dir > 0) ? link(c, n, mu) : link(c, m, mu);
                cplx t[4][3];
                for (int sp = 0; sp < 4; sp++)
                    for (int x = 0; x < 3; x++) {
                        cplx acc = 0;
                        for (int y = 0; y < 3; y++)
                            acc += (dir > 0 ? u[x * 3 + y] : conj(u[y * 3 + x])) * in[lm * 12 + sp * 3 + y];
                        t[sp][x] = acc;
                    }
                const double pg = -(double)dir;
                for (int sp = 0; sp < 4; sp++)
                    for (int x = 0; x < 3; x++) {
                        cplx acc = 0;
                        for (int q = 0; q < 4; q++)
                            acc += ((sp == q ? 1.0 : 0.0) + pg * GAM[mu][sp][q]) * t[q][x];
                        o[sp * 3 + x] += s * acc;
                    }
            }
    }
}

static void block_mask(const wco_ctx *c, const blockmap *B, cplx *v, int keep)
{
    for (long l = 0; l < B->Ne; l++)
        if (parity(c, B->g[l]) != keep)
            for (int i = 0; i < 12; i++) v[l * 12 + i] = 0;
}

static void block_clover_inv(const wco_ctx *c, const blockmap *B, const cplx *in, cplx *out)
{
    for (long l = 0; l < B->Ne; l++) mat12_site(c->Ti + B->g[l] * 144, in + l * 12, out + l * 12);
}

static void block_schur(const wco_ctx *c, const blockmap *B, const cplx *x, cplx *out, cplx *t1,
                        cplx *t2)
{
    const long N = B->Ne * 12;
    block_hop(c, B, x, t1);
    block_mask(c, B, t1, 1);
    block_clover_inv(c, B, t1, t2);
    block_hop(c, B, t2, t1);
    block_mask(c, B, t1, 0);
    block_clover_inv(c, B, t1, t2);
    const double k2 = c->kappa * c->kappa;
    for (long i = 0; i < N; i++) out[i] = x[i] - k2 * t2[i];
    block_mask(c, B, out, 0);
}

/* Block BiCGStab (van der Vorst 1992) on Dhat_B z = r_B from z = 0 with the
 * shadow residual rh = r_B, `iters` iterations of two block operator
 * applications each.  The block stops (z as it stands) when rho = <rh, r> or
 * <rh, v> is exactly zero; <t, t> = 0 means s = 0, and the step ends with
 * omega = 0.  On entry r = r_B; q, t1, t2 are scratch of the block's size. */
static void block_bicgstab(const wco_ctx *c, const blockmap *B, int iters, cplx *r, cplx *z, cplx *q,
                           cplx *t1, cplx *t2)
{
    const long N = B->Ne * 12;
    cplx *rh = calloc(N, sizeof(cplx)), *p = calloc(N, sizeof(cplx)), *v = calloc(N, sizeof(cplx));
    cplx *s = calloc(N, sizeof(cplx));
    memcpy(rh, r, sizeof(cplx) * N);
    cplx rho_old = 1.0, alpha = 1.0, omega = 1.0;
    for (int k = 0; k < iters; k++) {
        const cplx rho = vdot(N, rh, r);
        if (rho == 0.0) break;
        const cplx beta = (rho / rho_old) * (alpha / omega);
        for (long i = 0; i < N; i++) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        block_schur(c, B, p, v, t1, t2);
        const cplx rv = vdot(N, rh, v);
        if (rv == 0.0) break;
        alpha = rho / rv;
        for (long i = 0; i < N; i++) s[i] = r[i] - alpha * v[i];
        block_schur(c, B, s, q, t1, t2);   /* q = t = Dhat_B s */
        const double tt = creal(vdot(N, q, q));
        omega = tt == 0.0 ? 0.0 : vdot(N, q, s) / tt;
        for (long i = 0; i < N; i++) {
            z[i] += alpha * p[i] + omega * s[i];
            r[i] = s[i] - omega * q[i];
        }
        rho_old = rho;
        if (tt == 0.0) break;
    }
    free(rh); free(p); free(v); free(s);
}

/* The restricted block solves of one Schwarz application on the blocks of
 * one colour (colour < 0: every block).  Colour of a block = the parities of
 * its block coordinates, bit mu for direction mu (16 colours).  The restricted
 * result (even core sites) is added to out. */
static int ras_blocks(const wco_ctx *c, const int block[4], int overlap, int iters, int solver, int colour,
                      const cplx *vin, cplx *vout)
{
    int nb_[4];
    for (int mu = 0; mu < 4; mu++) nb_[mu] = c->L[mu] / block[mu];
    const long nblocks = (long)nb_[0] * nb_[1] * nb_[2] * nb_[3];

#pragma omp parallel for schedule(dynamic)
    for (long bi = 0; bi < nblocks; bi++) {
        blockmap B;
        int bo[4], col = 0;
        long rem = bi;
        for (int mu = 0; mu < 4; mu++) {
            const int bk = (int)(rem % nb_[mu]);
            bo[mu] = bk * block[mu];
            col |= (bk & 1) << mu;
            rem /= nb_[mu];
            B.e[mu] = block[mu] + 2 * overlap;
        }
        if (colour >= 0 && col != colour) continue;
        B.Ne = (long)B.e[0] * B.e[1] * B.e[2] * B.e[3];
        B.g = malloc(sizeof(long) * B.Ne);
        for (long l = 0; l < B.Ne; l++) {
            int a[4], x[4];
            lcoords(&B, l, a);
            for (int mu = 0; mu < 4; mu++) x[mu] = ((bo[mu] - overlap + a[mu]) % c->L[mu] + c->L[mu]) % c->L[mu];
            B.g[l] = index_of(c, x);
        }
        const long N = B.Ne * 12;
        cplx *r = calloc(N, sizeof(cplx)), *z = calloc(N, sizeof(cplx)), *q = calloc(N, sizeof(cplx));
        cplx *t1 = calloc(N, sizeof(cplx)), *t2 = calloc(N, sizeof(cplx));
        for (long l = 0; l < B.Ne; l++)
            for (int i = 0; i < 12; i++) r[l * 12 + i] = vin[B.g[l] * 12 + i];
        block_mask(c, &B, r, 0);
        if (solver == 2) {
            block_bicgstab(c, &B, iters, r, z, q, t1, t2);
        } else {
            /* from z = 0, r = r_B: minimal residual (alpha = <q, r> / <q, q>)
             * or block Jacobi (alpha = 1), with q = Dhat_B r */
            for (int k = 0; k < iters; k++) {
                block_schur(c, &B, r, q, t1, t2);
                cplx alpha = 1.0;
                if (solver == 0) {
                    const double qq = creal(vdot(N, q, q));
                    if (qq == 0.0) break;
                    alpha = vdot(N, q, r) / qq;
                }
                for (long i = 0; i < N; i++) { z[i] += alpha * r[i]; r[i] -= alpha * q[i]; }
            }
        }
        /* restriction: keep the even core sites (cores never overlap) */
        for (long l = 0; l < B.Ne; l++) {
            int a[4];
            lcoords(&B, l, a);
            int core = 1;
            for (int mu = 0; mu < 4; mu++)
                if (a[mu] < overlap || a[mu] >= overlap + block[mu]) core = 0;
            if (!core || parity(c, B.g[l]) != 0) continue;
            for (int i = 0; i < 12; i++) vout[B.g[l] * 12 + i] += z[l * 12 + i];
        }
        free(r); free(z); free(q); free(t1); free(t2); free(B.g);
    }
    return 0;
}

static int ras_args_ok(const wco_ctx *c, const int block[4], int overlap, int solver)
{
    if (solver < 0 || solver > 2) return 0;
    for (int mu = 0; mu < 4; mu++) {
        if (block[mu] < 2 || (block[mu] & 1) || c->L[mu] % block[mu]) return 0;
        if (c->L[mu] < block[mu] + 2 * overlap || overlap < 0) return 0;
    }
    return 1;
}

int wco_ras(const wco_ctx *c, const int block[4], int overlap, int iters, int solver,
            const double *in, double *out)
{
    if (!ras_args_ok(c, block, overlap, solver)) return -1;
    memset(out, 0, sizeof(cplx) * 12 * c->V);
    return ras_blocks(c, block, overlap, iters, solver, -1, (const cplx *)in, (cplx *)out);
}

/* Multiplicative Schwarz: the 16 block colours in turn, each solving on the
 * residual that the previous colours left:  z = 0;  for colour k:
 * r = v - Dhat z,  z += (restricted block solves of colour k on r). */
int wco_sap(const wco_ctx *c, const int block[4], int overlap, int iters, int solver,
            const double *in, double *out)
{
    if (!ras_args_ok(c, block, overlap, solver)) return -1;
    const long N = 12 * c->V;
    const cplx *v = (const cplx *)in;
    cplx *z = (cplx *)out, *r = vnew(c), *t = vnew(c);
    memset(z, 0, sizeof(cplx) * N);
    for (int k = 0; k < 16; k++) {
        if (k == 0) {
            memcpy(r, v, sizeof(cplx) * N);
        } else {
            schur_plain(c, z, t);
            for (long i = 0; i < N; i++) r[i] = v[i] - t[i];
        }
        mask_parity(c, r, 0);
        ras_blocks(c, block, overlap, iters, solver, k, r, z);
    }
    free(r); free(t);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Inner solver: BiCGStab on Dhat, right-preconditioned by RAS
 * (p^ = M^-1 p, v = Dhat p^, s^ = M^-1 s, t = Dhat s^, x += a p^ + w s^).
 * Stops when the recursive residual reaches stol * ||rhs||.
 * ------------------------------------------------------------------------- */
typedef struct {
    int use_ras, block[4], overlap, iters;
} precond;

static void apply_precond(const wco_ctx *c, const precond *P, const cplx *in, cplx *out)
{
    if (P->use_ras) wco_ras(c, P->block, P->overlap, P->iters, 0, (const double *)in, (double *)out);
    else memcpy(out, in, sizeof(cplx) * 12 * c->V);
}

static int inner_solve(const wco_ctx *c, const precond *P, const cplx *rhs, cplx *x, double stol,
                       int maxiter, int *iters_out)
{
    const long N = 12 * c->V;
    cplx *r = vnew(c), *rt = vnew(c), *p = vnew(c), *v = vnew(c), *s = vnew(c), *t = vnew(c);
    cplx *ph = vnew(c), *sh = vnew(c);
    memset(x, 0, sizeof(cplx) * N);
    const double bn = vnorm(N, rhs);
    int status = 1, it = 0;
    if (bn == 0.0) { status = 0; goto done; }
    memcpy(r, rhs, sizeof(cplx) * N);
    memcpy(rt, r, sizeof(cplx) * N);
    cplx rho = 1, alpha = 1, omega = 1;
    for (it = 1; it <= maxiter; it++) {
        const cplx rho1 = vdot(N, rt, r);
        if (cabs(rho1) == 0.0) { status = 2; break; }
        const cplx beta = (rho1 / rho) * (alpha / omega);
        for (long i = 0; i < N; i++) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        apply_precond(c, P, p, ph);
        schur_plain(c, ph, v);
        const cplx rtv = vdot(N, rt, v);
        if (cabs(rtv) == 0.0) { status = 2; break; }
        alpha = rho1 / rtv;
        for (long i = 0; i < N; i++) s[i] = r[i] - alpha * v[i];
        apply_precond(c, P, s, sh);
        schur_plain(c, sh, t);
        const double tt = creal(vdot(N, t, t));
        omega = (tt == 0.0) ? 0.0 : vdot(N, t, s) / tt;
        for (long i = 0; i < N; i++) x[i] += alpha * ph[i] + omega * sh[i];
        for (long i = 0; i < N; i++) r[i] = s[i] - omega * t[i];
        rho = rho1;
        if (vnorm(N, r) <= stol * bn) { status = 0; break; }
        if (omega == 0.0) { status = 2; break; }
    }
    if (it > maxiter) it = maxiter;
done:
    *iters_out = it;
    free(r); free(rt); free(p); free(v); free(s); free(t); free(ph); free(sh);
    return status;
}

int wco_inner_bicgstab(const wco_ctx *c, const double *rhs, double *xe, double stol, int maxiter,
                       int use_ras, const int block[4], int overlap, int ras_iters, int *iters_out)
{
    precond P = {use_ras, {2, 2, 2, 2}, overlap, ras_iters};
    if (block) memcpy(P.block, block, sizeof(P.block));
    return inner_solve(c, &P, (const cplx *)rhs, (cplx *)xe, stol, maxiter, iters_out);
}

/* ---------------------------------------------------------------------------
 * Outer flexible BiCGStab on the Schur system; the preconditioner K is the
 * inner solve applied to the normalised vector and scaled back.
 * ------------------------------------------------------------------------- */
static void inner_K(const wco_ctx *c, const precond *P, const cplx *in, cplx *out, double stol,
                    int maxiter, int *inner_total)
{
    const long N = 12 * c->V;
    const double nrm = vnorm(N, in);
    if (nrm == 0.0) { memset(out, 0, sizeof(cplx) * N); return; }
    cplx *u = vnew(c);
    for (long i = 0; i < N; i++) u[i] = in[i] / nrm;
    int it = 0;
    inner_solve(c, P, u, out, stol, maxiter, &it);
    *inner_total += it;
    for (long i = 0; i < N; i++) out[i] *= nrm;
    free(u);
}

int wco_fbicgstab(const wco_ctx *c, const double *b_in, double *x_out, double tol, int max_outer,
                  double inner_tol, int max_inner, int use_ras, const int block[4], int overlap,
                  int ras_iters, int *outer_out, int *inner_total_out, double *relres_out)
{
    precond P = {use_ras, {2, 2, 2, 2}, overlap, ras_iters};
    if (block) memcpy(P.block, block, sizeof(P.block));
    const long N = 12 * c->V;
    const cplx *b = (const cplx *)b_in;
    cplx *bh = vnew(c), *x = vnew(c), *r = vnew(c), *rt = vnew(c), *p = vnew(c), *v = vnew(c);
    cplx *s = vnew(c), *t = vnew(c), *ph = vnew(c), *sh = vnew(c), *xf = vnew(c), *rf = vnew(c);
    int inner_total = 0, status = 1, k = 0;
    double relres = 0.0;
    const double bn = vnorm(N, b);
    if (bn == 0.0) { memset(x_out, 0, sizeof(cplx) * N); status = 0; goto done; }
    wco_schur_rhs(c, b_in, (double *)bh);
    memcpy(r, bh, sizeof(cplx) * N);
    memcpy(rt, r, sizeof(cplx) * N);
    memcpy(p, r, sizeof(cplx) * N);
    cplx rho = vdot(N, rt, r);
    for (k = 1; k <= max_outer; k++) {
        inner_K(c, &P, p, ph, inner_tol, max_inner, &inner_total);
        schur_plain(c, ph, v);
        const cplx rtv = vdot(N, rt, v);
        if (cabs(rtv) == 0.0) { status = 2; break; }
        const cplx alpha = rho / rtv;
        for (long i = 0; i < N; i++) s[i] = r[i] - alpha * v[i];
        inner_K(c, &P, s, sh, inner_tol, max_inner, &inner_total);
        schur_plain(c, sh, t);
        const double tt = creal(vdot(N, t, t));
        const cplx omega = (tt == 0.0) ? 0.0 : vdot(N, t, s) / tt;
        for (long i = 0; i < N; i++) x[i] += alpha * ph[i] + omega * sh[i];
        for (long i = 0; i < N; i++) r[i] = s[i] - omega * t[i];
        if (vnorm(N, r) <= tol * bn) {
            wco_reconstruct(c, b_in, (const double *)x, (double *)xf);
            relres = true_res_full(c, b, xf, rf);
            if (relres <= tol) { status = 0; break; }
            /* residual replacement and restart of the recurrence */
            schur_plain(c, x, r);
            for (long i = 0; i < N; i++) r[i] = bh[i] - r[i];
            memcpy(p, r, sizeof(cplx) * N);
            rho = vdot(N, rt, r);
            continue;
        }
        if (omega == 0.0) { status = 2; break; }
        const cplx rho1 = vdot(N, rt, r);
        const cplx beta = (rho1 / rho) * (alpha / omega);
        for (long i = 0; i < N; i++) p[i] = r[i] + beta * (p[i] - omega * v[i]);
        rho = rho1;
    }
    if (k > max_outer) k = max_outer;
    wco_reconstruct(c, b_in, (const double *)x, x_out);
    if (status != 0) relres = true_res_full(c, b, (const cplx *)x_out, rf);
done:
    *outer_out = k;
    *inner_total_out = inner_total;
    *relres_out = relres;
    free(bh); free(x); free(r); free(rt); free(p); free(v);
    free(s); free(t); free(ph); free(sh); free(xf); free(rf);
    return status;
}

/* ---------------------------------------------------------------------------
 * Gradient of L = Re<eta, D^-1 b>.  With x = D^-1 b, y = D^-dag eta:
 *   dL = -Re<y, dD x>,  D = T - kappa H,  T = 1 - csw kappa sum sigma F.
 * Link gradient G (dL = Re sum conj(G_ab) dU_ab):
 *   hopping:  kappa s_mu(x) sum_spin { [(1-g_mu) y(x)] x(x+mu)^dag
 *                                     + x(x) [(1+g_mu) y(x+mu)]^dag }
 *   clover :  dL = sum_x sum_{mu<nu} Re[ z tr(dQ_{mu nu}(x) K_{mu nu}(x)) ],
 *             z = -i csw kappa / 8, K = M' + M'^dag, M' = M - tr(M)/3,
 *             M_ab = sum_{s,t} sigma_st x_t,a conj(y_s,b);
 *             each leaf is a product A B C D and the product rule gives,
 *             for a factor U at position j with X = (factors after j) K
 *             (factors before j): G += conj(z) X^dag; for a factor U^dag:
 *             G += z X.
 *   kappa  :  dL/dkappa = Re<y, H x> + csw Re<y, C x>,  C = sum sigma F.
 * ------------------------------------------------------------------------- */
void wco_grad(const wco_ctx *c, const double *xd, const double *yd, double *gUd, double *gkappa)
{
    const cplx *x = (const cplx *)xd, *y = (const cplx *)yd;
    cplx *G = (cplx *)gUd;
    memset(G, 0, sizeof(cplx) * 36 * c->V);

    /* hopping part */
#pragma omp parallel for schedule(static)
    for (long n = 0; n < c->V; n++)
        for (int mu = 0; mu < 4; mu++) {
            const long f = nb(c, n, mu, +1);
            const double s = bc_sign(c, n, mu, +1);
            cplx w[4][3], v[4][3];
            for (int sp = 0; sp < 4; sp++)
                for (int a = 0; a < 3; a++) {
                    cplx aw = 0, av = 0;
                    for (int q = 0; q < 4; q++) {
                        const cplx g = GAM[mu][sp][q];
                        aw += ((sp == q ? 1.0 : 0.0) - g) * y[n * 12 + q * 3 + a];
                        av += ((sp == q ? 1.0 : 0.0) + g) * y[f * 12 + q * 3 + a];
                    }
                    w[sp][a] = aw;
                    v[sp][a] = av;
                }
            cplx *g = G + (n * 4 + mu) * 9;
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++) {
                    cplx acc = 0;
                    for (int sp = 0; sp < 4; sp++)
                        acc += w[sp][a] * conj(x[f * 12 + sp * 3 + b]) +
                               x[n * 12 + sp * 3 + a] * conj(v[sp][b]);
                    g[a * 3 + b] += c->kappa * s * acc;
                }
        }

    /* clover part (serial: contributions land on links of other sites) */
    const cplx z = -_Complex_I * c->csw * c->kappa / 8.0;
    for (long n = 0; n < c->V; n++)
        for (int p = 0; p < 6; p++) {
            cplx M[9];
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++) {
                    cplx acc = 0;
                    for (int s = 0; s < 4; s++)
                        for (int t = 0; t < 4; t++)
                            acc += SIG[p][s][t] * x[n * 12 + t * 3 + a] * conj(y[n * 12 + s * 3 + b]);
                    M[a * 3 + b] = acc;
                }
            const cplx tr = (M[0] + M[4] + M[8]) / 3.0;
            M[0] -= tr; M[4] -= tr; M[8] -= tr;
            cplx K[9];
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++) K[a * 3 + b] = M[a * 3 + b] + conj(M[b * 3 + a]);

            long site[4][4];
            int dag[4][4], dirn[4][4];
            leaves(c, n, PMU[p], PNU[p], site, dag, dirn);
            for (int l = 0; l < 4; l++) {
                cplx f[4][9];
                for (int k = 0; k < 4; k++) {
                    const cplx *u = link(c, site[l][k], dirn[l][k]);
                    if (dag[l][k]) m3_dag(u, f[k]); else memcpy(f[k], u, sizeof(f[k]));
                }
                for (int j = 0; j < 4; j++) {
                    /* X = f[j+1] ... f[3] K f[0] ... f[j-1] */
                    cplx X[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
                    for (int k = j + 1; k < 4; k++) m3_mul(X, f[k], X);
                    m3_mul(X, K, X);
                    for (int k = 0; k < j; k++) m3_mul(X, f[k], X);
                    cplx *g = G + (site[l][j] * 4 + dirn[l][j]) * 9;
                    if (!dag[l][j]) {
                        for (int a = 0; a < 3; a++)
                            for (int b = 0; b < 3; b++) g[a * 3 + b] += conj(z) * conj(X[b * 3 + a]);
                    } else {
                        for (int a = 0; a < 3; a++)
                            for (int b = 0; b < 3; b++) g[a * 3 + b] += z * X[a * 3 + b];
                    }
                }
            }
        }

    /* kappa */
    cplx *hx = vnew(c), *cx = vnew(c);
    hop_all(c, x, hx);
    wco_clover_C(c, xd, (double *)cx);
    const long N = 12 * c->V;
    *gkappa = creal(vdot(N, y, hx)) + c->csw * creal(vdot(N, y, cx));
    free(hx); free(cx);
}
