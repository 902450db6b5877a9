// kernels.hip -- layout conversion, gauge ingest, clover build and inversion,
// the even/odd hopping kernel with its fused epilogues, precision conversion
// and the BLAS-1 / reduction kernels of the solvers.
//
// The operator (Wilson-Clover, paper Sec. 1 and Sec. 2):
//   D = T - kappa H,  (H psi)(x) = sum_mu (1 - g_mu) U_mu(x) psi(x+mu)
//                                     + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu),
//   T = 1 - c_sw kappa sum_{mu<nu} sigma_{mu nu} F_{mu nu}  (clover leaves),
// in the chiral basis; H maps one parity onto the other ("hopping matrix
// multiplication", the paper's measured kernel, Sec. 3).
#include "hop_dev.h"

namespace wcl {

// ---------------------------------------------------------------------------
// Geometry helpers for the setup kernels (divisions are fine there).
WCL_D void canon_coords(const Geom &g, int n, int x[4])
{
    x[0] = n % g.L[0]; n /= g.L[0];
    x[1] = n % g.L[1]; n /= g.L[1];
    x[2] = n % g.L[2];
    x[3] = n / g.L[2];
}

WCL_D int coords_to_h(const Geom &g, const int x[4])
{
    int blk = 0, lin = 0;
#pragma unroll
    for (int mu = 0; mu < 4; mu++) {
        const int b = x[mu] / g.B[mu];
        blk += b * g.sb[mu];
        lin += (x[mu] - b * g.B[mu]) * g.sl[mu];
    }
    return blk * g.Hb + (lin >> 1);
}

// ---------------------------------------------------------------------------
// Canonical <-> e/o FP64 spinors.
__global__ void k_pack_spinor(Geom g, const double2 *__restrict__ canon, double2 *__restrict__ eo)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    const int V = 2 * g.Vh;
    if (n >= V) return;
    int x[4];
    canon_coords(g, n, x);
    const int p = (x[0] + x[1] + x[2] + x[3]) & 1;
    const size_t h = coords_to_h(g, x);
    double2 *dst = eo + (size_t)p * 12 * g.Vh;
    const double2 *src = canon + (size_t)n * 12;
#pragma unroll
    for (int i = 0; i < 12; i++) dst[i * (size_t)g.Vh + h] = src[i];
}

__global__ void k_unpack_spinor(Geom g, const double2 *__restrict__ eo, double2 *__restrict__ canon)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    const int V = 2 * g.Vh;
    if (n >= V) return;
    int x[4];
    canon_coords(g, n, x);
    const int p = (x[0] + x[1] + x[2] + x[3]) & 1;
    const size_t h = coords_to_h(g, x);
    const double2 *src = eo + (size_t)p * 12 * g.Vh;
    double2 *dst = canon + (size_t)n * 12;
#pragma unroll
    for (int i = 0; i < 12; i++) dst[i] = src[i * (size_t)g.Vh + h];
}

hipError_t launch_pack_spinor(const Geom &g, const double *canon, void *eo, hipStream_t st)
{
    const int V = 2 * g.Vh;
    k_pack_spinor<<<(V + 255) / 256, 256, 0, st>>>(g, (const double2 *)canon, (double2 *)eo);
    return hipGetLastError();
}

hipError_t launch_unpack_spinor(const Geom &g, const void *eo, double *canon, hipStream_t st)
{
    const int V = 2 * g.Vh;
    k_unpack_spinor<<<(V + 255) / 256, 256, 0, st>>>(g, (const double2 *)eo, (double2 *)canon);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gauge ingest: canonical U[V][4][3][3] complex128 -> internal link fields.
__global__ void k_ingest_gauge(Geom g, const double2 *__restrict__ canon, void *u64, void *u32, void *u16)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    const int V = 2 * g.Vh;
    if (n >= V) return;
    int x[4];
    canon_coords(g, n, x);
    const int p = (x[0] + x[1] + x[2] + x[3]) & 1;
    const size_t h = coords_to_h(g, x);
    for (int mu = 0; mu < 4; mu++) {
        cplx<double> u[9];
#pragma unroll
        for (int k = 0; k < 9; k++) {
            const double2 d = canon[((size_t)n * 4 + mu) * 9 + k];
            u[k] = {d.x, d.y};
        }
        if (u64) store_link<double, double>(u64, mu, p, h, g.Vh, u);
        if (u32) store_link<float, double>(u32, mu, p, h, g.Vh, u);
        if (u16) store_link<__half, double>(u16, mu, p, h, g.Vh, u);
    }
}

// Two-row (12-real) FP32 and FP16 copies of the FP64 links.
__global__ void k_compress_links(Geom g, const void *u64, void *u32c, void *u16c, void *u32s)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 8 * g.Vh) return;
    const int mp = i / g.Vh, h = i - mp * g.Vh;
    cplx<double> u[9];
    load_link<double, double>(u64, mp >> 1, mp & 1, h, g.Vh, u);
    store_link<R12f, double>(u32c, mp >> 1, mp & 1, h, g.Vh, u);
    store_link<R12h, double>(u16c, mp >> 1, mp & 1, h, g.Vh, u);
    store_link_site<double>(u32s, mp >> 1, mp & 1, h, g.Vh, u);
}

hipError_t launch_compress_links(const Geom &g, const void *u64, void *u32c, void *u16c, void *u32s, hipStream_t st)
{
    k_compress_links<<<(8 * g.Vh + 255) / 256, 256, 0, st>>>(g, u64, u32c, u16c, u32s);
    return hipGetLastError();
}

// Largest |row2 - conj(row0 x row1)| over the FP64 links (per-workgroup maxima).
// max that keeps a NaN (fmax would drop it)
WCL_D double nanmax(double m, double d) { return (d > m || d != d) ? d : m; }

__global__ void __launch_bounds__(256) k_su3_check(Geom g, const void *u64, double *partial)
{
    __shared__ double red[256];
    double m = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < 8 * g.Vh; i += gridDim.x * blockDim.x) {
        const int mp = i / g.Vh, h = i - mp * g.Vh;
        cplx<double> u[9], r[9];
        load_link<double, double>(u64, mp >> 1, mp & 1, h, g.Vh, u);
#pragma unroll
        for (int k = 0; k < 9; k++) r[k] = u[k];
        su3_third_row(r);
#pragma unroll
        for (int k = 6; k < 9; k++) m = nanmax(m, fmax(fabs(r[k].re - u[k].re), fabs(r[k].im - u[k].im)));
        cplx<double> ip = {0.0, 0.0};
        double n0 = 0.0, n1 = 0.0;
#pragma unroll
        for (int c = 0; c < 3; c++) {
            const cplx<double> a = u[c], b = u[3 + c];
            n0 += a.re * a.re + a.im * a.im;
            n1 += b.re * b.re + b.im * b.im;
            ip.re += a.re * b.re + a.im * b.im;
            ip.im += a.re * b.im - a.im * b.re;
        }
        m = nanmax(m, fabs(n0 - 1.0));
        m = nanmax(m, fabs(n1 - 1.0));
        m = nanmax(m, sqrt(ip.re * ip.re + ip.im * ip.im));
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] = nanmax(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

hipError_t launch_su3_check(const Geom &g, const void *u64, double *partial, int nblocks, hipStream_t st)
{
    k_su3_check<<<nblocks, 256, 0, st>>>(g, u64, partial);
    return hipGetLastError();
}

hipError_t launch_ingest_gauge(const Geom &g, const double *canon, void *u64, void *u32, void *u16,
                               hipStream_t st)
{
    const int V = 2 * g.Vh;
    k_ingest_gauge<<<(V + 127) / 128, 128, 0, st>>>(g, (const double2 *)canon, u64, u32, u16);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Clover term.  For each site, F_{mu nu} = (Q - Q^dag)/(8i) made traceless,
// Q the sum of the four plaquette leaves in the mu-nu plane.  In the chiral
// basis sum_{mu<nu} sigma_{mu nu} F_{mu nu} is block diagonal:
//   chirality +: sum_k s_k (x) (E_k - B_k),   chirality -: sum_k s_k (x) (-E_k - B_k)
// with E_k = F_{k t} and B = (F_yz, F_zx, F_xy), and s_k (x) G written out as
// [[G_3, G_1 - i G_2], [G_1 + i G_2, -G_3]].
struct M3 {
    cplx<double> a[9];
};

WCL_D M3 m3_mul(const M3 &A, const M3 &B)
{
    M3 C;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            cplx<double> s = A.a[i * 3] * B.a[j];
            s = cfma(A.a[i * 3 + 1], B.a[3 + j], s);
            s = cfma(A.a[i * 3 + 2], B.a[6 + j], s);
            C.a[i * 3 + j] = s;
        }
    return C;
}

WCL_D M3 m3_dag(const M3 &A)
{
    M3 C;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) C.a[i * 3 + j] = {A.a[j * 3 + i].re, -A.a[j * 3 + i].im};
    return C;
}

// link U_mu at global coordinates x + d (periodic wrap)
WCL_D M3 link_at(const Geom &g, const void *u64, const int x[4], const int d[4], int mu)
{
    int y[4];
#pragma unroll
    for (int k = 0; k < 4; k++) y[k] = (x[k] + d[k] + g.L[k]) % g.L[k];
    const int p = (y[0] + y[1] + y[2] + y[3]) & 1;
    M3 m;
    load_link<double, double>(u64, mu, p, coords_to_h(g, y), g.Vh, m.a);
    return m;
}

// Inverse of a Hermitian positive definite 6x6 by Cholesky: A = L L^dag,
// A^-1 = W^dag W with W = L^-1.  Returns false on a non-positive pivot.
WCL_D bool hpd_inverse6(const cplx<double> A[36], cplx<double> Ai[36])
{
    cplx<double> L[36];
#pragma unroll
    for (int k = 0; k < 36; k++) L[k] = {0.0, 0.0};
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 6; j++) {
        double d = A[j * 6 + j].re;
#pragma unroll
        for (int k = 0; k < j; k++) d -= L[j * 6 + k].re * L[j * 6 + k].re + L[j * 6 + k].im * L[j * 6 + k].im;
        if (!(d > 0.0)) { ok = false; d = 1.0; }
        const double ljj = sqrt(d);
        L[j * 6 + j] = {ljj, 0.0};
        const double inv = 1.0 / ljj;
#pragma unroll
        for (int i = j + 1; i < 6; i++) {
            cplx<double> s = A[i * 6 + j];
#pragma unroll
            for (int k = 0; k < j; k++) s = s - L[i * 6 + k] * cplx<double>{L[j * 6 + k].re, -L[j * 6 + k].im};
            L[i * 6 + j] = inv * s;
        }
    }
    // W = L^-1 (lower triangular), forward substitution column by column
    cplx<double> W[36];
#pragma unroll
    for (int k = 0; k < 36; k++) W[k] = {0.0, 0.0};
#pragma unroll
    for (int j = 0; j < 6; j++) {
        W[j * 6 + j] = {1.0 / L[j * 6 + j].re, 0.0};
#pragma unroll
        for (int i = j + 1; i < 6; i++) {
            cplx<double> s = {0.0, 0.0};
#pragma unroll
            for (int k = j; k < i; k++) s = cfma(L[i * 6 + k], W[k * 6 + j], s);
            W[i * 6 + j] = (-1.0 / L[i * 6 + i].re) * s;
        }
    }
    // Ai = W^dag W
#pragma unroll
    for (int i = 0; i < 6; i++)
#pragma unroll
        for (int j = 0; j < 6; j++) {
            cplx<double> s = {0.0, 0.0};
            const int k0 = i > j ? i : j;
#pragma unroll
            for (int k = k0; k < 6; k++) s = cjfma(W[k * 6 + i], W[k * 6 + j], s);
            Ai[i * 6 + j] = s;
        }
    return ok;
}

WCL_D void pack_block(const cplx<double> A[36], double *out36)
{
#pragma unroll
    for (int i = 0; i < 6; i++) out36[i] = A[i * 6 + i].re;
    int k = 0;
#pragma unroll
    for (int i = 0; i < 6; i++)
#pragma unroll
        for (int j = i + 1; j < 6; j++) {
            out36[6 + 2 * k] = A[i * 6 + j].re;
            out36[7 + 2 * k] = A[i * 6 + j].im;
            k++;
        }
}

// One clover leaf of plane (mu, nu) at x (leaf 0: x -> x+mu -> x+mu+nu ->
// x+nu; 1: x -> x+nu -> x-mu+nu -> x-mu; 2: x -> x-mu -> x-mu-nu -> x-nu;
// 3: x -> x-nu -> x+mu-nu -> x+mu; each back to x).
WCL_D M3 clover_leaf(const Geom &g, const void *u64, const int x[4], int mu, int nu, int leaf)
{
    int o[4] = {0, 0, 0, 0};
    int pm[4] = {0, 0, 0, 0}, pn[4] = {0, 0, 0, 0}, mm[4] = {0, 0, 0, 0}, mn[4] = {0, 0, 0, 0};
    int mmpn[4] = {0, 0, 0, 0}, mmmn[4] = {0, 0, 0, 0}, pmmn[4] = {0, 0, 0, 0};
    pm[mu] = 1; pn[nu] = 1; mm[mu] = -1; mn[nu] = -1;
    mmpn[mu] = -1; mmpn[nu] = 1;
    mmmn[mu] = -1; mmmn[nu] = -1;
    pmmn[mu] = 1; pmmn[nu] = -1;
    if (leaf == 0)
        return m3_mul(m3_mul(link_at(g, u64, x, o, mu), link_at(g, u64, x, pm, nu)),
                      m3_mul(m3_dag(link_at(g, u64, x, pn, mu)), m3_dag(link_at(g, u64, x, o, nu))));
    if (leaf == 1)
        return m3_mul(m3_mul(link_at(g, u64, x, o, nu), m3_dag(link_at(g, u64, x, mmpn, mu))),
                      m3_mul(m3_dag(link_at(g, u64, x, mm, nu)), link_at(g, u64, x, mm, mu)));
    if (leaf == 2)
        return m3_mul(m3_mul(m3_dag(link_at(g, u64, x, mm, mu)), m3_dag(link_at(g, u64, x, mmmn, nu))),
                      m3_mul(link_at(g, u64, x, mmmn, mu), link_at(g, u64, x, mn, nu)));
    return m3_mul(m3_mul(m3_dag(link_at(g, u64, x, mn, nu)), link_at(g, u64, x, mn, mu)),
                  m3_mul(link_at(g, u64, x, pmmn, nu), m3_dag(link_at(g, u64, x, o, mu))));
}

// Clover setup in two passes.  Pass 1: a workgroup takes 64 sites of one
// plane, each wave one of the four leaves; the leaves meet in LDS and the
// first wave forms the traceless Hermitian F_{mu nu} = (Q - Q^dag)/(8i) - tr
// (Q = leaf 0 + 1 + 2 + 3) and stores its upper triangle (F00, F11, F22,
// Re/Im F01, F02, F12: 9 reals) in F[plane][9][2 Vh].  Planes: E_k = F_{k t}
// (0..2), B_x = F_yz, -B_y = F_xz, B_z = F_xy (3..5).
__global__ void __launch_bounds__(256) k_clover_fs(Geom g, const void *u64, double *F)
{
    __shared__ double lq[4][18][64];
    const int n = 2 * g.Vh;
    const int lane = threadIdx.x & 63, leaf = threadIdx.x >> 6;
    const int idx = blockIdx.x * 64 + lane;
    const int plane = blockIdx.y;
    // (mu, nu) of the planes: (0,3) (1,3) (2,3) (1,2) (0,2) (0,1)
    const int mu = plane < 3 ? plane : (plane == 3 ? 1 : 0);
    const int nu = plane < 3 ? 3 : (plane == 5 ? 1 : 2);
    if (idx < n) {
        const int p = idx / g.Vh;
        const Site s = decompose(g, idx - p * g.Vh, p);
        const M3 l = clover_leaf(g, u64, s.x, mu, nu, leaf);
#pragma unroll
        for (int k = 0; k < 9; k++) {
            lq[leaf][2 * k][lane] = l.a[k].re;
            lq[leaf][2 * k + 1][lane] = l.a[k].im;
        }
    }
    __syncthreads();
    if (leaf != 0 || idx >= n) return;
    M3 Q;
#pragma unroll
    for (int k = 0; k < 9; k++) Q.a[k] = {lq[0][2 * k][lane], lq[0][2 * k + 1][lane]};
#pragma unroll
    for (int q = 1; q < 4; q++)
#pragma unroll
        for (int k = 0; k < 9; k++) Q.a[k] = Q.a[k] + cplx<double>{lq[q][2 * k][lane], lq[q][2 * k + 1][lane]};
    M3 f;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const double wr = Q.a[i * 3 + j].re - Q.a[j * 3 + i].re;
            const double wi = Q.a[i * 3 + j].im + Q.a[j * 3 + i].im;
            f.a[i * 3 + j] = {wi * 0.125, -wr * 0.125};
        }
    const double tr = (f.a[0].re + f.a[4].re + f.a[8].re) / 3.0;
    double *o = F + (size_t)plane * 9 * n + idx;
    o[0] = f.a[0].re - tr;
    o[(size_t)n] = f.a[4].re - tr;
    o[2 * (size_t)n] = f.a[8].re - tr;
    o[3 * (size_t)n] = f.a[1].re;
    o[4 * (size_t)n] = f.a[1].im;
    o[5 * (size_t)n] = f.a[2].re;
    o[6 * (size_t)n] = f.a[2].im;
    o[7 * (size_t)n] = f.a[5].re;
    o[8 * (size_t)n] = f.a[5].im;
}

// Entry (a, b) of plane `plane` of the stored F (the lower triangle by
// Hermiticity).
WCL_D cplx<double> f_entry(const double *F, size_t n, int idx, int plane, int a, int b)
{
    const double *q = F + (size_t)plane * 9 * n + idx;
    if (a == b) return {q[(size_t)a * n], 0.0};
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    const int k = lo == 0 ? (hi == 1 ? 3 : 5) : 7;
    const double re = q[(size_t)k * n], im = q[(size_t)(k + 1) * n];
    return a < b ? cplx<double>{re, im} : cplx<double>{re, -im};
}

// Half (chirality block chi) of a packed clover site in storage S: FP64 and
// FP32 blocks fill whole 16-byte words; FP16 block 0 ends and block 1 starts
// in word 4, whose other half is carried in `keep`.
template <typename S>
WCL_D void store_clover_block(void *base, int p, uint32_t h, uint32_t Vh, int chi, const double c[36], uint2 &keep)
{
    if constexpr (sizeof(S) == 8) {
#pragma unroll
        for (uint32_t k = 0; k < 18; k++)
            stf(base, (((uint32_t)p * 36 + 18 * chi + k) * Vh + h) * 16u, make_double2(c[2 * k], c[2 * k + 1]));
    } else if constexpr (sizeof(S) == 4) {
#pragma unroll
        for (uint32_t k = 0; k < 9; k++)
            stf(base, (((uint32_t)p * 18 + 9 * chi + k) * Vh + h) * 16u,
                make_float4((float)c[4 * k], (float)c[4 * k + 1], (float)c[4 * k + 2], (float)c[4 * k + 3]));
    } else {
        uint32_t w[18];
#pragma unroll
        for (int k = 0; k < 18; k++) w[k] = f22h((float)c[2 * k], (float)c[2 * k + 1]);
        if (chi == 0) {
#pragma unroll
            for (uint32_t k = 0; k < 4; k++)
                stf(base, (((uint32_t)p * 9 + k) * Vh + h) * 16u, make_uint4(w[4 * k], w[4 * k + 1], w[4 * k + 2], w[4 * k + 3]));
            keep = make_uint2(w[16], w[17]);
        } else {
            stf(base, (((uint32_t)p * 9 + 4) * Vh + h) * 16u, make_uint4(keep.x, keep.y, w[0], w[1]));
#pragma unroll
            for (uint32_t k = 0; k < 4; k++)
                stf(base, (((uint32_t)p * 9 + 5 + k) * Vh + h) * 16u,
                    make_uint4(w[2 + 4 * k], w[3 + 4 * k], w[4 + 4 * k], w[5 + 4 * k]));
        }
    }
}

// Pass 2: one thread per site builds T = 1 - c_sw kappa sigma.F one
// chirality block at a time from the stored F, inverts it (FP64 Cholesky)
// and writes both into every requested storage.
__global__ void __launch_bounds__(64) k_clover_inv(Geom g, const double *F, double ck, void *t64, void *ti64,
                                                   void *t32, void *ti32, void *t16, void *ti16, int *info)
{
    const size_t n = 2 * (size_t)g.Vh;
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int)n) return;
    const int p = idx / g.Vh;
    const int h = idx - p * g.Vh;
    bool ok = true;
    uint2 keepT = make_uint2(0u, 0u), keepTi = make_uint2(0u, 0u);
    for (int chi = 0; chi < 2; chi++) {
        const double se = chi == 0 ? 1.0 : -1.0;
        // G_k = se * E_k - B_k
        cplx<double> A[36];
#pragma unroll
        for (int a = 0; a < 3; a++)
#pragma unroll
            for (int b = 0; b < 3; b++) {
                const cplx<double> G1 = se * f_entry(F, n, idx, 0, a, b) - f_entry(F, n, idx, 3, a, b);
                const cplx<double> G2 = se * f_entry(F, n, idx, 1, a, b) + f_entry(F, n, idx, 4, a, b);
                const cplx<double> G3 = se * f_entry(F, n, idx, 2, a, b) - f_entry(F, n, idx, 5, a, b);
                const cplx<double> iG2 = {-G2.im, G2.re};
                const double id = (a == b) ? 1.0 : 0.0;
                A[a * 6 + b] = cplx<double>{id, 0.0} - ck * G3;
                A[(3 + a) * 6 + 3 + b] = cplx<double>{id, 0.0} + ck * G3;
                A[a * 6 + 3 + b] = -ck * (G1 - iG2);
                A[(3 + a) * 6 + b] = -ck * (G1 + iG2);
            }
        double packed[36];
        pack_block(A, packed);
        if (t64) store_clover_block<double>(t64, p, h, g.Vh, chi, packed, keepT);
        if (t32) store_clover_block<float>(t32, p, h, g.Vh, chi, packed, keepT);
        if (t16) store_clover_block<__half>(t16, p, h, g.Vh, chi, packed, keepT);
        cplx<double> Ai[36];
        ok = hpd_inverse6(A, Ai) && ok;
        pack_block(Ai, packed);
        if (ti64) store_clover_block<double>(ti64, p, h, g.Vh, chi, packed, keepTi);
        if (ti32) store_clover_block<float>(ti32, p, h, g.Vh, chi, packed, keepTi);
        if (ti16) store_clover_block<__half>(ti16, p, h, g.Vh, chi, packed, keepTi);
    }
    if (!ok) atomicAdd(info, 1);
}

hipError_t launch_clover_build(const Geom &g, const void *u64, double ck, void *t64, void *ti64, void *t32,
                               void *ti32, void *t16, void *ti16, int *info, double *fbuf, hipStream_t st)
{
    const int n = 2 * g.Vh;
    k_clover_fs<<<dim3((n + 63) / 64, 6), 256, 0, st>>>(g, u64, fbuf);
    k_clover_inv<<<(n + 63) / 64, 64, 0, st>>>(g, fbuf, ck, t64, ti64, t32, ti32, t16, ti16, info);
    return hipGetLastError();
}

// NT: links and clover loaded non-temporally (a single right-hand side reads
// them once per launch).  Off by default: repeated applications in a solver
// find the links in the Infinity Cache only when they were loaded normally.
template <typename SL, typename SS, int MODE, bool DAG, int DEPTH, bool NT, int NS>
__global__ void __launch_bounds__(256) k_hop(HopArgs a)
{
    // workgroup id = site block * nrhs + rhs: the nrhs workgroups of one site
    // block are neighbours in dispatch order (and on one XCD), so each link
    // is fetched from HBM once and served to the other right-hand sides by L2
    // A workgroup takes tpw consecutive site blocks (one contiguous range of
    // every field), one after another.
    const int lin = a.xcd ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int rhs = lin % a.nrhs;
    const int grp = lin / a.nrhs;
    if (a.sc && a.sc[rhs].done) return;
    constexpr int NWORDS = (int)sizeof(SS) * 24 / 16;
    __shared__ uint4 sin[NS > 0 ? NWORDS * NS : 1];
    const int nb = (a.g.Vh + blockDim.x - 1) / blockDim.x;
    for (int k = 0; k < a.tpw; k++) {
        const int bid = grp * a.tpw + k;
        if (bid >= nb) break;                 // uniform in the workgroup
        if (NS > 0 && k) __syncthreads();     // the previous block's staged input is read
        hop_block<SL, SS, MODE, DAG, DEPTH, NT, NS>(a, bid, rhs, sin);
    }
}

// ---------------------------------------------------------------------------
// Several right-hand sides per thread (batched inner solves): each link and
// clover block is loaded once into registers and applied to the NR
// right-hand sides of a group, whose neighbour spinors are loaded together.
// FP32 spinors; modes HOP, CLOV_H, XPAY; no dagger.  A right-hand side whose
// scalars say done is neither computed nor stored.
template <typename SL, int K, int NR>
WCL_D void hop_mr_hop(const HopArgs &a, const Site &s, uint32_t h0, const bool act[NR], const char *const in[NR],
                      cplx<float> acc[NR][12])
{
    constexpr int MU = K >> 1;
    constexpr bool FWD = (K & 1) == 0;
    constexpr int S = FWD ? -1 : 1;
    const Geom &g = a.g;
    const uint32_t Vh = g.Vh;
    uint32_t hn = (uint32_t)neighbour(g, s, MU, FWD ? +1 : -1);
    uint32_t h = h0;
    // this hop's loads wait for the previous hop's work on the first group member
    pipeline_fence(acc[0], hn, h);
    LinkRaw<SL> lr;
    if (FWD) load_link_raw<SL>(a.links, MU, a.p, h, Vh, lr);
    else load_link_raw<SL>(a.links, MU, 1 - a.p, hn, Vh, lr);
    cplx<float> psi[NR][12];
#pragma unroll
    for (int r = 0; r < NR; r++)
        if (act[r]) load_spinor<float, float>(in[r], hn, Vh, psi[r]);
    float sign = 1.f;
    if (MU == 3 && g.tbc < 0 && s.x[3] == (FWD ? g.L[3] - 1 : 0)) sign = -1.f;
    cplx<float> u[9];
    expand_link<SL, float>(lr, u);
#pragma unroll
    for (int r = 0; r < NR; r++) {
        if (!act[r]) continue;
        cplx<float> hh[6], uh[6];
        project<MU, S, float>(psi[r], hh);
        if (MU == 3) {
#pragma unroll
            for (int k = 0; k < 6; k++) hh[k] = sign * hh[k];
        }
        if (FWD) su3_mul(u, hh, uh);
        else su3_dag_mul(u, hh, uh);
        accumulate<MU, S, float>(acc[r], uh);
    }
}

template <typename SL, int K, int NR>
WCL_D void hop_mr_all(const HopArgs &a, const Site &s, uint32_t h, const bool act[NR], const char *const in[NR],
                      cplx<float> acc[NR][12])
{
    if constexpr (K < 8) {
        hop_mr_hop<SL, K, NR>(a, s, h, act, in, acc);
        hop_mr_all<SL, K + 1, NR>(a, s, h, act, in, acc);
    }
}

template <typename SL, int MODE, int NR>
__global__ void __launch_bounds__(256) k_hop_mr(HopArgs a)
{
    // workgroup id = site block * groups + group (the groups of one site block
    // run back to back on one XCD, so L2 serves the links to all of them)
    const int ngr = (a.nrhs + NR - 1) / NR;
    const int lin = a.xcd ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int grp = lin % ngr;
    const int bid = lin / ngr;
    const int r0 = grp * NR;
    bool act[NR];
    bool any = false;
#pragma unroll
    for (int r = 0; r < NR; r++) {
        act[r] = (r0 + r < a.nrhs) && !(a.sc && a.sc[r0 + r].done);
        any = any || act[r];
    }
    if (!any) return;
    const int h = bid * blockDim.x + threadIdx.x;
    if (h >= a.g.Vh) return;
    const uint32_t Vh = a.g.Vh;
    const char *in[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) in[r] = (const char *)a.in + (act[r] ? r0 + r : 0) * a.in_stride;
    const Site s = decompose(a.g, h, a.p);
    cplx<float> acc[NR][12];
#pragma unroll
    for (int r = 0; r < NR; r++)
#pragma unroll
        for (int i = 0; i < 12; i++) acc[r][i] = {0.f, 0.f};
    hop_mr_all<SL, 0, NR>(a, s, h, act, in, acc);

    if constexpr (MODE == HOP) {
#pragma unroll
        for (int r = 0; r < NR; r++)
            if (act[r]) store_spinor<float, float>((char *)a.out + (r0 + r) * a.out_stride, h, Vh, acc[r]);
    } else {
        // one clover chirality block at a time, shared by the group
#pragma unroll
        for (int half = 0; half < 2; half++) {
            float c[36];
            load_clover_half<typename ClovS<SL>::T, float>(a.clov, a.p, h, Vh, half, c);
#pragma unroll
            for (int r = 0; r < NR; r++) {
                if (!act[r]) continue;
                cplx<float> o[6];
                clover_mul_half(c, acc[r] + 6 * half, o);
                char *out = (char *)a.out + (r0 + r) * a.out_stride;
                if constexpr (MODE == XPAY) {
                    const char *x = (const char *)a.x + (r0 + r) * a.x_stride;
                    const float cf = (float)a.coef;
#pragma unroll
                    for (int k = 0; k < 3; k++) {
                        const float4 xv = ldf<float4>(x, ((3 * half + k) * Vh + h) * 16u);
                        o[2 * k] = {fmaf(cf, o[2 * k].re, xv.x), fmaf(cf, o[2 * k].im, xv.y)};
                        o[2 * k + 1] = {fmaf(cf, o[2 * k + 1].re, xv.z), fmaf(cf, o[2 * k + 1].im, xv.w)};
                    }
                }
#pragma unroll
                for (int k = 0; k < 3; k++)
                    stf(out, ((3 * half + k) * Vh + h) * 16u,
                        make_float4(o[2 * k].re, o[2 * k].im, o[2 * k + 1].re, o[2 * k + 1].im));
            }
        }
    }
}

template <typename SL, int NR>
static hipError_t hop_mr_dispatch(const HopLaunch &L, const HopArgs &a, dim3 block, hipStream_t st)
{
    const int ngr = (a.nrhs + NR - 1) / NR;
    dim3 grid(((a.g.Vh + block.x - 1) / block.x) * ngr);
    switch (L.mode) {
    case HOP: ext_launch(k_hop_mr<SL, HOP, NR>, grid, block, 0, st, L.ev, a); break;
    case CLOV_H: ext_launch(k_hop_mr<SL, CLOV_H, NR>, grid, block, 0, st, L.ev, a); break;
    case XPAY: ext_launch(k_hop_mr<SL, XPAY, NR>, grid, block, 0, st, L.ev, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename SL>
static hipError_t hop_mr_nr(const HopLaunch &L, const HopArgs &a, dim3 block, hipStream_t st)
{
    if (L.rhs_per_thread == 4) return hop_mr_dispatch<SL, 4>(L, a, block, st);
    return hop_mr_dispatch<SL, 2>(L, a, block, st);
}

// Pipeline-depth variants (hops whose operands are in flight: 2, 3) times
// temporal / non-temporal operator loads.  D^dag launches use depth 2.
template <typename SL, typename SS, int MODE>
static void hop_dispatch_dag(const HopLaunch &L, const HopArgs &a, dim3 grid, dim3 block, hipStream_t st)
{
    const bool nt = L.nontemporal && a.nrhs == 1;
    // staged input spinors (depth 2, non-dagger): one LDS slot per thread;
    // with non-temporal operator loads for single-use (cold) calls
    const bool staged = L.lds_stage && !L.dagger && L.depth == 2;
    if (staged && nt && block.x == 64) ext_launch(k_hop<SL, SS, MODE, false, 2, true, 64>, grid, block, 0, st, L.ev, a);
    else if (staged && nt && block.x == 128) ext_launch(k_hop<SL, SS, MODE, false, 2, true, 128>, grid, block, 0, st, L.ev, a);
    else if (staged && nt && block.x == 256) ext_launch(k_hop<SL, SS, MODE, false, 2, true, 256>, grid, block, 0, st, L.ev, a);
    else if (staged && !nt && block.x == 64) ext_launch(k_hop<SL, SS, MODE, false, 2, false, 64>, grid, block, 0, st, L.ev, a);
    else if (staged && !nt && block.x == 128) ext_launch(k_hop<SL, SS, MODE, false, 2, false, 128>, grid, block, 0, st, L.ev, a);
    else if (staged && !nt && block.x == 256) ext_launch(k_hop<SL, SS, MODE, false, 2, false, 256>, grid, block, 0, st, L.ev, a);
    else if (L.dagger) ext_launch(k_hop<SL, SS, MODE, true, 2, false, 0>, grid, block, 0, st, L.ev, a);
    else if (L.depth == 3 && nt) ext_launch(k_hop<SL, SS, MODE, false, 3, true, 0>, grid, block, 0, st, L.ev, a);
    else if (L.depth == 3) ext_launch(k_hop<SL, SS, MODE, false, 3, false, 0>, grid, block, 0, st, L.ev, a);
    else if (nt) ext_launch(k_hop<SL, SS, MODE, false, 2, true, 0>, grid, block, 0, st, L.ev, a);
    else ext_launch(k_hop<SL, SS, MODE, false, 2, false, 0>, grid, block, 0, st, L.ev, a);
}

template <typename SL, typename SS>
static void hop_dispatch_mode(const HopLaunch &L, const HopArgs &a, dim3 grid, dim3 block, hipStream_t st)
{
    switch (L.mode) {
    case HOP: hop_dispatch_dag<SL, SS, HOP>(L, a, grid, block, st); break;
    case CLOV_H: hop_dispatch_dag<SL, SS, CLOV_H>(L, a, grid, block, st); break;
    case XPAY: hop_dispatch_dag<SL, SS, XPAY>(L, a, grid, block, st); break;
    default: hop_dispatch_dag<SL, SS, CLOVX>(L, a, grid, block, st); break;
    }
}

int hop_parts(const HopLaunch &L)
{
    const int bs = L.block > 0 ? L.block : 256;
    return (L.g->Vh + bs - 1) / bs;
}

hipError_t launch_hop(const HopLaunch &L, hipStream_t st)
{
    if (L.nrhs < 1 || L.nrhs > 4096) return hipErrorInvalidValue;
    if (L.nrhs > 1) {
        const size_t sb = spinor_bytes(L.spin_prec == P64 ? 8 : L.spin_prec == P32 ? 4 : 2, (size_t)L.g->Vh);
        if (L.in_stride < sb || L.out_stride < sb || (L.mode >= XPAY && L.x_stride < sb)) return hipErrorInvalidValue;
    }
    HopArgs a;
    a.g = *L.g;
    a.in = L.in;
    a.out = L.out;
    a.links = L.links;
    a.clov = L.clov;
    a.x = L.x;
    a.coef = L.coef;
    a.in_stride = L.in_stride;
    a.out_stride = L.out_stride;
    a.x_stride = L.x_stride;
    a.p = L.p;
    a.xcd = L.xcd;
    a.sc = L.sc;
    a.nrhs = L.nrhs;
    a.tpw = 1;
    const int bs = L.block > 0 ? L.block : 256;
    if (bs > 256 || bs % 64) return hipErrorInvalidValue;
    const int nb = (a.g.Vh + bs - 1) / bs;
    dim3 grid(nb * a.nrhs);
    dim3 block(bs);
    if (L.ndot) return launch_hop_dot(L, a, grid, block, st);
    if (L.tpw > 1) {
        if (L.tpw > 64) return hipErrorInvalidValue;
        a.tpw = L.tpw;
        grid = dim3(((nb + L.tpw - 1) / L.tpw) * a.nrhs);
    }
    if ((L.rhs_per_thread == 2 || L.rhs_per_thread == 4) && a.nrhs >= 2 && L.spin_prec == P32 && !L.dagger &&
        L.mode != CLOVX) {
        switch (L.link_prec) {
        case P32: return hop_mr_nr<float>(L, a, block, st);
        case P16: return hop_mr_nr<__half>(L, a, block, st);
        case P32C: return hop_mr_nr<R12f>(L, a, block, st);
        case P16C: return hop_mr_nr<R12h>(L, a, block, st);
        default: break;
        }
    }
    if (L.link_prec == P64 && L.spin_prec == P64) hop_dispatch_mode<double, double>(L, a, grid, block, st);
    else if (L.link_prec == P32 && L.spin_prec == P32) hop_dispatch_mode<float, float>(L, a, grid, block, st);
    else if (L.link_prec == P16 && L.spin_prec == P32) hop_dispatch_mode<__half, float>(L, a, grid, block, st);
    else if (L.link_prec == P16 && L.spin_prec == P16) hop_dispatch_mode<__half, __half>(L, a, grid, block, st);
    else if (L.link_prec == P32C && L.spin_prec == P32) hop_dispatch_mode<R12f, float>(L, a, grid, block, st);
    else if (L.link_prec == P16C && L.spin_prec == P32) hop_dispatch_mode<R12h, float>(L, a, grid, block, st);
    else if (L.link_prec == P16C && L.spin_prec == P16) hop_dispatch_mode<R12h, __half>(L, a, grid, block, st);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Clover apply: out = A in on one parity (504 flop per site).
template <typename SL, typename SS>
__global__ void __launch_bounds__(256) k_clover(Geom g, int p, const void *clov, const char *in, char *out,
                                               size_t in_stride, size_t out_stride)
{
    using R = typename Real<SL>::T;
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= g.Vh) return;
    in += blockIdx.y * in_stride;
    out += blockIdx.y * out_stride;
    R c[72];
    cplx<R> v[12], o[12];
    load_clover<SL, R>(clov, p, h, g.Vh, c);
    load_spinor<SS, R>(in, h, g.Vh, v);
    clover_mul(c, v, o);
    store_spinor<SS, R>(out, h, g.Vh, o);
}

hipError_t launch_clover(const Geom &g, int lp, int sp, int p, const void *clov, const void *in, void *out,
                         hipStream_t st, int nrhs, size_t in_stride, size_t out_stride, LaunchEvents ev)
{
    dim3 grid((g.Vh + 255) / 256, nrhs), block(256);
    const char *i = (const char *)in;
    char *o = (char *)out;
    if (lp == P32C) lp = P32;
    if (lp == P16C) lp = P16;
    if (lp == P64 && sp == P64) ext_launch(k_clover<double, double>, grid, block, 0, st, ev, g, p, clov, i, o, in_stride, out_stride);
    else if (lp == P32 && sp == P32) ext_launch(k_clover<float, float>, grid, block, 0, st, ev, g, p, clov, i, o, in_stride, out_stride);
    else if (lp == P16 && sp == P32) ext_launch(k_clover<__half, float>, grid, block, 0, st, ev, g, p, clov, i, o, in_stride, out_stride);
    else if (lp == P16 && sp == P16) ext_launch(k_clover<__half, __half>, grid, block, 0, st, ev, g, p, clov, i, o, in_stride, out_stride);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Precision conversion of spinor sections (each section Vh sites).
template <typename SI, typename SO>
__global__ void k_convert(size_t nsites, size_t Vi, size_t Vo, const char *in, char *out, const double *sdev,
                          int mode, double shost, int sec_per_scale, int sdev_stride)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsites) return;
    const size_t sec = i / Vi, h = i - sec * Vi;
    double sc = shost;
    if (mode) {
        const double v = sdev[(sec / sec_per_scale) * sdev_stride];
        if (mode == 1) sc = (v > 0.0) ? shost / sqrt(v) : 0.0;
        else sc = shost * sqrt(v);
    }
    cplx<double> v[12];
    load_spinor<SI, double>(in + sec * spinor_bytes(sizeof(SI), Vi), h, Vi, v);
#pragma unroll
    for (int k = 0; k < 12; k++) v[k] = sc * v[k];
    store_spinor<SO, double>(out + sec * spinor_bytes(sizeof(SO), Vo), h, Vo, v);
}

hipError_t launch_convert(int ip, int op, size_t nsites, size_t Vi, size_t Vo, const void *in, void *out,
                          const double *sdev, int mode, double shost, hipStream_t st, int sec_per_scale,
                          int sdev_stride)
{
    dim3 grid((unsigned)((nsites + 255) / 256)), block(256);
    const char *i = (const char *)in;
    char *o = (char *)out;
#define WCL_CONV(A, B) \
    k_convert<A, B><<<grid, block, 0, st>>>(nsites, Vi, Vo, i, o, sdev, mode, shost, sec_per_scale, sdev_stride)
    if (ip == P64 && op == P32) WCL_CONV(double, float);
    else if (ip == P32 && op == P64) WCL_CONV(float, double);
    else if (ip == P64 && op == P16) WCL_CONV(double, __half);
    else if (ip == P16 && op == P64) WCL_CONV(__half, double);
    else if (ip == P64 && op == P64) WCL_CONV(double, double);
    else if (ip == P32 && op == P32) WCL_CONV(float, float);
    else if (ip == P32 && op == P16) WCL_CONV(float, __half);
    else if (ip == P16 && op == P32) WCL_CONV(__half, float);
    else return hipErrorInvalidValue;
#undef WCL_CONV
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Reductions: wavefront butterfly (DPP / ds_swizzle through __shfl_xor), then
// one value per wave through LDS.
WCL_D double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int NV>
WCL_D void block_sum(double v[NV], double *lds /* [NV][16] */)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; k++) {
        v[k] = wave_sum(v[k]);
        if (lane == 0) lds[k * 16 + wid] = v[k];
    }
    __syncthreads();
    if (wid == 0) {
#pragma unroll
        for (int k = 0; k < NV; k++) {
            double t = lane < nw ? lds[k * 16 + lane] : 0.0;
            v[k] = wave_sum(t);
        }
    }
}

// Storage of one complex number (V) and the arithmetic type (C) of the
// flat-vector kernels: FP16 vectors are stored as half2 and computed in FP32.
template <typename T>
struct CT;
template <> struct CT<double> { using V = double2; using C = double; };
template <> struct CT<float> { using V = float2; using C = float; };
template <> struct CT<__half> { using V = __half2; using C = float; };

WCL_D double2 ldv(const double2 &v) { return v; }
WCL_D float2 ldv(const float2 &v) { return v; }
WCL_D float2 ldv(const __half2 &v) { return __half22float2(v); }
WCL_D void stv(double2 &d, double x, double y) { d = make_double2(x, y); }
WCL_D void stv(float2 &d, float x, float y) { d = make_float2(x, y); }
WCL_D void stv(__half2 &d, float x, float y)
{
    fp32_as_computed(x, y);
    d = __floats2half2_rn(x, y);
}

// partials[rhs][(2*k + {0,1}) * RED_BLOCKS + block] = (Re, Im) of sum conj(a_k) b_k
// over the rhs-th slice (stride elements apart); blockIdx.y = rhs.
template <typename T, int NP>
__global__ void __launch_bounds__(RED_THREADS) k_dots(size_t n, size_t stride, const typename CT<T>::V *a0,
                                                      const typename CT<T>::V *b0, const typename CT<T>::V *a1,
                                                      const typename CT<T>::V *b1, const typename CT<T>::V *a2,
                                                      const typename CT<T>::V *b2, double *partials, const Scalars *sc,
                                                      int pstride)
{
    const int rhs = blockIdx.y;
    if (sc && sc[rhs].done) return;
    __shared__ double lds[2 * NP * 16];
    double v[2 * NP];
#pragma unroll
    for (int k = 0; k < 2 * NP; k++) v[k] = 0.0;
    const size_t off = rhs * stride;
    const typename CT<T>::V *A[3] = {a0 + off, a1 + off, a2 + off}, *B[3] = {b0 + off, b1 + off, b2 + off};
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int k = 0; k < NP; k++) {
            const auto x = ldv(A[k][i]), y = ldv(B[k][i]);
            v[2 * k] += (double)x.x * (double)y.x + (double)x.y * (double)y.y;
            v[2 * k + 1] += (double)x.x * (double)y.y - (double)x.y * (double)y.x;
        }
    }
    block_sum<2 * NP>(v, lds);
    if (threadIdx.x == 0) {
        double *pr = partials + (size_t)rhs * 6 * pstride;
#pragma unroll
        for (int k = 0; k < 2 * NP; k++) pr[k * pstride + blockIdx.x] = v[k];
    }
}

hipError_t launch_dots(int prec, size_t n, int np, const void *const *a, const void *const *b, double *partials,
                       const Scalars *sc, hipStream_t st, int nrhs, size_t stride, int pstride)
{
    if (pstride < RED_BLOCKS) return hipErrorInvalidValue;
    const void *A[3] = {a[0], np > 1 ? a[1] : a[0], np > 2 ? a[2] : a[0]};
    const void *B[3] = {b[0], np > 1 ? b[1] : b[0], np > 2 ? b[2] : b[0]};
    dim3 grid(RED_BLOCKS, nrhs), block(RED_THREADS);
#define WCL_DOTS(T, NP)                                                                                   \
    k_dots<T, NP><<<grid, block, 0, st>>>(n, stride, (const CT<T>::V *)A[0], (const CT<T>::V *)B[0],      \
                                          (const CT<T>::V *)A[1], (const CT<T>::V *)B[1],                 \
                                          (const CT<T>::V *)A[2], (const CT<T>::V *)B[2], partials, sc, pstride)
    if (prec == P64) {
        if (np == 1) WCL_DOTS(double, 1);
        else if (np == 2) WCL_DOTS(double, 2);
        else WCL_DOTS(double, 3);
    } else if (prec == P32) {
        if (np == 1) WCL_DOTS(float, 1);
        else if (np == 2) WCL_DOTS(float, 2);
        else WCL_DOTS(float, 3);
    } else if (prec == P16) {
        if (np == 1) WCL_DOTS(__half, 1);
        else if (np == 2) WCL_DOTS(__half, 2);
        else WCL_DOTS(__half, 3);
    } else {
        return hipErrorInvalidValue;
    }
#undef WCL_DOTS
    return hipGetLastError();
}

WCL_D void cdiv(const double a[2], const double b[2], double o[2])
{
    const double d = b[0] * b[0] + b[1] * b[1];
    o[0] = (a[0] * b[0] + a[1] * b[1]) / d;
    o[1] = (a[1] * b[0] - a[0] * b[1]) / d;
}

// One workgroup per right-hand side.  gate (optional): a right-hand side
// whose gate scalars are done is marked done at BICG_INIT_RHO.
__global__ void __launch_bounds__(512) k_finalize(int step, int nterms, const double *partials_all, Scalars *sc_all,
                                                  const Scalars *gate, int pstride, int nparts)
{
    const int rhs = blockIdx.x;
    Scalars *sc = sc_all + rhs;
    const double *partials = partials_all + (size_t)rhs * 6 * pstride;
    if (sc->done && (step == BICG_ALPHA || step == BICG_OMEGA || step == BICG_RHO)) return;
    __shared__ double lds[6 * 16];
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    // each thread adds partials j = tid, tid + 512, ... in that order; eight of
    // them per term are loaded before any is added, so the loads overlap
    constexpr int U = 8;
    for (int j0 = threadIdx.x; j0 < nparts; j0 += U * blockDim.x) {
        double p[6][U];
#pragma unroll
        for (int k = 0; k < 6; k++)
#pragma unroll
            for (int u = 0; u < U; u++) {
                const int j = j0 + u * (int)blockDim.x;
                p[k][u] = (k < nterms && j < nparts) ? partials[k * pstride + j] : 0.0;
            }
#pragma unroll
        for (int k = 0; k < 6; k++)
#pragma unroll
            for (int u = 0; u < U; u++)
                if (k < nterms && j0 + u * (int)blockDim.x < nparts) v[k] += p[k][u];
    }
    block_sum<6>(v, lds);
    if (threadIdx.x != 0) return;
    switch (step) {
    case BICG_INIT_RHO:
        // pairs (rt, r), (r, r)
        sc->rho[0] = v[0]; sc->rho[1] = v[1];
        sc->r2 = v[2];
        sc->b2 = v[2];
        sc->rho_old[0] = 1.0; sc->rho_old[1] = 0.0;
        sc->alpha[0] = 1.0; sc->alpha[1] = 0.0;
        sc->omega[0] = 1.0; sc->omega[1] = 0.0;
        sc->iter = 0;
        sc->done = (v[2] == 0.0) ? 1 : 0;
        if (gate && gate[rhs].done) sc->done = 1;
        break;
    case BICG_ALPHA: {
        const double d[2] = {v[0], v[1]};
        if (d[0] == 0.0 && d[1] == 0.0) { sc->done = 2; break; }
        cdiv(sc->rho, d, sc->alpha);
        break;
    }
    case BICG_OMEGA: {
        // pairs (t, s), (t, t)
        const double tt = v[2];
        if (tt == 0.0) { sc->omega[0] = 0.0; sc->omega[1] = 0.0; }
        else { sc->omega[0] = v[0] / tt; sc->omega[1] = v[1] / tt; }
        break;
    }
    case BICG_RHO:
        sc->rho_old[0] = sc->rho[0]; sc->rho_old[1] = sc->rho[1];
        sc->rho[0] = v[0]; sc->rho[1] = v[1];
        sc->r2 = v[2];
        sc->iter += 1;
        if (!(v[2] <= sc->stop2 * sc->b2) && !(v[2] >= 0.0)) sc->done = 2;     // NaN
        else if (v[2] <= sc->stop2 * sc->b2) sc->done = 1;
        else if ((sc->omega[0] == 0.0 && sc->omega[1] == 0.0) || (v[0] == 0.0 && v[1] == 0.0)) sc->done = 2;
        break;
    case NORM_ONLY:
        sc->t[0] = v[0];
        break;
    default:
        break;
    }
}

hipError_t launch_finalize(int step, int nterms, const double *partials, Scalars *sc, hipStream_t st, int nrhs,
                           const Scalars *gate, int pstride, int nparts)
{
    if (nparts < 1 || nparts > pstride) return hipErrorInvalidValue;
    k_finalize<<<nrhs, 512, 0, st>>>(step, nterms, partials, sc, gate, pstride, nparts);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// BiCGStab vector updates (complex scalars from the device), blockIdx.y = rhs.
template <typename T>
__global__ void __launch_bounds__(256) k_bicg_p(size_t n, size_t stride, const typename CT<T>::V *r,
                                               typename CT<T>::V *p, const typename CT<T>::V *v, const Scalars *sc_all)
{
    const Scalars *sc = sc_all + blockIdx.y;
    if (sc->done) return;
    const size_t off = blockIdx.y * stride;
    r += off; p += off; v += off;
    // beta = (rho / rho_old) (alpha / omega)
    double q1[2], q2[2], beta[2];
    cdiv(sc->rho, sc->rho_old, q1);
    cdiv(sc->alpha, sc->omega, q2);
    beta[0] = q1[0] * q2[0] - q1[1] * q2[1];
    beta[1] = q1[0] * q2[1] + q1[1] * q2[0];
    using C = typename CT<T>::C;
    const C br = (C)beta[0], bi = (C)beta[1], wr = (C)sc->omega[0], wi = (C)sc->omega[1];
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const auto pv = ldv(p[i]), vv = ldv(v[i]), rv = ldv(r[i]);
        // d = p - omega v
        const C dr = pv.x - (wr * vv.x - wi * vv.y);
        const C di = pv.y - (wr * vv.y + wi * vv.x);
        stv(p[i], rv.x + br * dr - bi * di, rv.y + br * di + bi * dr);
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_bicg_s(size_t n, size_t stride, const typename CT<T>::V *r,
                                               const typename CT<T>::V *v, typename CT<T>::V *s, const Scalars *sc_all)
{
    const Scalars *sc = sc_all + blockIdx.y;
    if (sc->done) return;
    const size_t off = blockIdx.y * stride;
    r += off; v += off; s += off;
    using C = typename CT<T>::C;
    const C ar = (C)sc->alpha[0], ai = (C)sc->alpha[1];
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const auto rv = ldv(r[i]), vv = ldv(v[i]);
        stv(s[i], rv.x - (ar * vv.x - ai * vv.y), rv.y - (ar * vv.y + ai * vv.x));
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_bicg_xr(size_t n, size_t stride, typename CT<T>::V *x,
                                                const typename CT<T>::V *ph, const typename CT<T>::V *sh,
                                                typename CT<T>::V *r, const typename CT<T>::V *s,
                                                const typename CT<T>::V *t, const Scalars *sc_all)
{
    const Scalars *sc = sc_all + blockIdx.y;
    if (sc->done) return;
    const size_t off = blockIdx.y * stride;
    x += off; ph += off; sh += off; r += off; s += off; t += off;
    using C = typename CT<T>::C;
    const C ar = (C)sc->alpha[0], ai = (C)sc->alpha[1], wr = (C)sc->omega[0], wi = (C)sc->omega[1];
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const auto xv = ldv(x[i]), pv = ldv(ph[i]), sv = ldv(sh[i]), s2 = ldv(s[i]), tv = ldv(t[i]);
        stv(x[i], xv.x + (ar * pv.x - ai * pv.y) + (wr * sv.x - wi * sv.y),
            xv.y + (ar * pv.y + ai * pv.x) + (wr * sv.y + wi * sv.x));
        stv(r[i], s2.x - (wr * tv.x - wi * tv.y), s2.y - (wr * tv.y + wi * tv.x));
    }
}

// x += alpha ph + omega sh; r = s - omega t, with the partials of <rt, r>
// and <r, r> (of the stored r) per workgroup: terms 0, 1 = Re, Im <rt, r>,
// 2 = <r, r>, 3 = 0 at partials[rhs][k][block] (stride pstride).
template <typename T>
__global__ void __launch_bounds__(256) k_bicg_xr_dots(size_t n, size_t stride, typename CT<T>::V *x,
                                                     const typename CT<T>::V *ph, const typename CT<T>::V *sh,
                                                     typename CT<T>::V *r, const typename CT<T>::V *s,
                                                     const typename CT<T>::V *t, const typename CT<T>::V *rt,
                                                     const Scalars *sc_all, double *partials, int pstride)
{
    const Scalars *sc = sc_all + blockIdx.y;
    if (sc->done) return;
    __shared__ double lds[4 * 16];
    const size_t off = blockIdx.y * stride;
    x += off; ph += off; sh += off; r += off; s += off; t += off; rt += off;
    using C = typename CT<T>::C;
    const C ar = (C)sc->alpha[0], ai = (C)sc->alpha[1], wr = (C)sc->omega[0], wi = (C)sc->omega[1];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const auto xv = ldv(x[i]), pv = ldv(ph[i]), sv = ldv(sh[i]), s2 = ldv(s[i]), tv = ldv(t[i]);
        stv(x[i], xv.x + (ar * pv.x - ai * pv.y) + (wr * sv.x - wi * sv.y),
            xv.y + (ar * pv.y + ai * pv.x) + (wr * sv.y + wi * sv.x));
        stv(r[i], s2.x - (wr * tv.x - wi * tv.y), s2.y - (wr * tv.y + wi * tv.x));
        const auto rn = ldv(r[i]), rr = ldv(rt[i]);
        v[0] += (double)rr.x * (double)rn.x + (double)rr.y * (double)rn.y;
        v[1] += (double)rr.x * (double)rn.y - (double)rr.y * (double)rn.x;
        v[2] += (double)rn.x * (double)rn.x + (double)rn.y * (double)rn.y;
    }
    block_sum<4>(v, lds);
    if (threadIdx.x == 0) {
        double *pr = partials + (size_t)blockIdx.y * 6 * pstride;
#pragma unroll
        for (int k = 0; k < 4; k++) pr[k * pstride + blockIdx.x] = v[k];
    }
}

static dim3 blas_grid(size_t n, int nrhs = 1)
{
    size_t b = (n + 255) / 256;
    const size_t cap = nrhs > 1 ? 2048 : 8192;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return dim3((unsigned)b, nrhs);
}

// Flat-vector launchers: P64, P32 or P16 storage (n complex numbers per
// right-hand side); any other precision code is refused.
#define WCL_BY_PREC(CALL)                                 \
    do {                                                  \
        if (prec == P64) {                                \
            using T = double;                             \
            CALL;                                         \
        } else if (prec == P32) {                         \
            using T = float;                              \
            CALL;                                         \
        } else if (prec == P16) {                         \
            using T = __half;                             \
            CALL;                                         \
        } else {                                          \
            return hipErrorInvalidValue;                  \
        }                                                 \
    } while (0)
#define WCL_V(x) ((typename CT<T>::V *)(x))
#define WCL_CV(x) ((const typename CT<T>::V *)(x))

hipError_t launch_bicg_p(int prec, size_t n, const void *r, void *p, const void *v, const Scalars *sc,
                         hipStream_t st, int nrhs, size_t stride)
{
    WCL_BY_PREC((k_bicg_p<T><<<blas_grid(n, nrhs), 256, 0, st>>>(n, stride, WCL_CV(r), WCL_V(p), WCL_CV(v), sc)));
    return hipGetLastError();
}

hipError_t launch_bicg_s(int prec, size_t n, const void *r, const void *v, void *s, const Scalars *sc,
                         hipStream_t st, int nrhs, size_t stride)
{
    WCL_BY_PREC((k_bicg_s<T><<<blas_grid(n, nrhs), 256, 0, st>>>(n, stride, WCL_CV(r), WCL_CV(v), WCL_V(s), sc)));
    return hipGetLastError();
}

hipError_t launch_bicg_xr(int prec, size_t n, void *x, const void *ph, const void *sh, void *r, const void *s,
                          const void *t, const Scalars *sc, hipStream_t st, int nrhs, size_t stride)
{
    WCL_BY_PREC((k_bicg_xr<T><<<blas_grid(n, nrhs), 256, 0, st>>>(n, stride, WCL_V(x), WCL_CV(ph), WCL_CV(sh),
                                                                   WCL_V(r), WCL_CV(s), WCL_CV(t), sc)));
    return hipGetLastError();
}

hipError_t launch_bicg_xr_dots(int prec, size_t n, void *x, const void *ph, const void *sh, void *r,
                               const void *s, const void *t, const void *rt, const Scalars *sc, hipStream_t st,
                               int nrhs, size_t stride, double *partials, int pstride, int *nparts)
{
    // at most RED_BLOCKS workgroups per right-hand side, so that the finaliser
    // adds few partials
    dim3 grid = blas_grid(n, nrhs);
    if (grid.x > (unsigned)RED_BLOCKS) grid.x = RED_BLOCKS;
    if ((int)grid.x > pstride) return hipErrorInvalidValue;
    *nparts = (int)grid.x;
    WCL_BY_PREC((k_bicg_xr_dots<T><<<grid, 256, 0, st>>>(n, stride, WCL_V(x), WCL_CV(ph), WCL_CV(sh), WCL_V(r),
                                                          WCL_CV(s), WCL_CV(t), WCL_CV(rt), sc, partials,
                                                          pstride)));
    return hipGetLastError();
}

template <typename T>
__global__ void __launch_bounds__(256) k_axpby(size_t n, double ar, double ai, const typename CT<T>::V *x, double br,
                                              double bi, typename CT<T>::V *y)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        using C = typename CT<T>::C;
        const auto xv = ldv(x[i]), yv = ldv(y[i]);
        stv(y[i], (C)(ar * xv.x - ai * xv.y + br * yv.x - bi * yv.y), (C)(ar * xv.y + ai * xv.x + br * yv.y + bi * yv.x));
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_copy(size_t n, const typename CT<T>::V *x, typename CT<T>::V *y)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        y[i] = x[i];
}

template <typename T>
__global__ void __launch_bounds__(256) k_zero(size_t n, typename CT<T>::V *y)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        stv(y[i], (typename CT<T>::C)0, (typename CT<T>::C)0);
}

hipError_t launch_axpby(int prec, size_t n, double2 a, const void *x, double2 b, void *y, hipStream_t st)
{
    WCL_BY_PREC((k_axpby<T><<<blas_grid(n), 256, 0, st>>>(n, a.x, a.y, WCL_CV(x), b.x, b.y, WCL_V(y))));
    return hipGetLastError();
}

hipError_t launch_copy(int prec, size_t n, const void *x, void *y, hipStream_t st)
{
    WCL_BY_PREC((k_copy<T><<<blas_grid(n), 256, 0, st>>>(n, WCL_CV(x), WCL_V(y))));
    return hipGetLastError();
}

hipError_t launch_zero(int prec, size_t n, void *y, hipStream_t st)
{
    WCL_BY_PREC((k_zero<T><<<blas_grid(n), 256, 0, st>>>(n, WCL_V(y))));
    return hipGetLastError();
}
#undef WCL_BY_PREC
#undef WCL_V
#undef WCL_CV

}  // namespace wcl

namespace wcl {

static double link_site_bytes(int prec)
{
    return prec == P64 ? 144.0 : prec == P32 ? 72.0 : prec == P16 ? 36.0 : prec == P32C ? 48.0 : 24.0;
}
static double spinor_site_bytes(int prec) { return prec == P64 ? 192.0 : prec == P32 ? 96.0 : 48.0; }
static double clover_site_bytes(int prec)
{
    return prec == P64 ? 576.0 : (prec == P32 || prec == P32C) ? 288.0 : 144.0;
}

void hop_work(const HopLaunch &a, double *bytes, double *flops)
{
    const double sites = (double)a.g->Vh * (a.nrhs > 0 ? a.nrhs : 1);
    double b = (a.nrhs > 0 ? 8.0 * link_site_bytes(a.link_prec) / a.nrhs : 8.0 * link_site_bytes(a.link_prec));
    b += 2.0 * spinor_site_bytes(a.spin_prec);
    double f = 1320.0;
    if (a.mode != HOP) {
        b += clover_site_bytes(a.link_prec) / (a.nrhs > 0 ? a.nrhs : 1);
        f += 504.0;
    }
    if (a.mode == XPAY || a.mode == CLOVX) {
        b += spinor_site_bytes(a.spin_prec);
        f += 48.0;
    }
    if (a.ndot) {   // fused reductions: the second vector and 96 flop per inner product
        b += spinor_site_bytes(a.spin_prec);
        f += a.ndot == 1 ? 96.0 : 144.0;
    }
    *bytes = b * sites;
    *flops = f * sites;
}

// ---------------------------------------------------------------------------
// Streaming ceilings for the roofline.  Read: each workgroup streams one
// contiguous chunk with 16 independent 16-byte non-temporal loads in flight
// per thread (the fastest of a sweep over chunked / grid-stride order,
// temporal / non-temporal loads, 4 / 8 / 16 loads in flight and 1024 ...
// 32768 workgroups of 256 ... 1024 threads); one word written per thread.
// Copy: the same order with 8 loads and 8 stores in flight.
__global__ void __launch_bounds__(256) k_stream_read(const u32x4 *__restrict__ a, size_t n, size_t chunk, float *out)
{
    constexpr int U = 16;
    u32x4 s = {0u, 0u, 0u, 0u};
    const size_t base = (size_t)blockIdx.x * chunk, end = base + chunk < n ? base + chunk : n;
    for (size_t i = base + threadIdx.x; i < end; i += U * blockDim.x) {
        u32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const size_t j = i + u * blockDim.x;
            v[u] = j < end ? __builtin_nontemporal_load(a + j) : u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int u = 0; u < U; u++) s ^= v[u];
    }
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = __uint_as_float(s.x ^ s.y ^ s.z ^ s.w);
}

__global__ void __launch_bounds__(256) k_stream_copy(const u32x4 *__restrict__ a, u32x4 *__restrict__ b, size_t n,
                                                    size_t chunk)
{
    constexpr int U = 8;
    const size_t base = (size_t)blockIdx.x * chunk, end = base + chunk < n ? base + chunk : n;
    for (size_t i = base + threadIdx.x; i < end; i += U * blockDim.x) {
        u32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
            const size_t j = i + u * blockDim.x;
            if (j < end) v[u] = __builtin_nontemporal_load(a + j);
        }
#pragma unroll
        for (int u = 0; u < U; u++) {
            const size_t j = i + u * blockDim.x;
            if (j < end) __builtin_nontemporal_store(v[u], b + j);
        }
    }
}

hipError_t launch_stream(int copy, const void *a, void *b, size_t n16, float *out, int blocks, hipStream_t st)
{
    const size_t chunk = (n16 + blocks - 1) / blocks;
    if (copy) k_stream_copy<<<blocks, 256, 0, st>>>((const u32x4 *)a, (u32x4 *)b, n16, chunk);
    else k_stream_read<<<blocks, 256, 0, st>>>((const u32x4 *)a, n16, chunk, out);
    return hipGetLastError();
}

}  // namespace wcl
