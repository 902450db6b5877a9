// grad.hip -- gradient of L = Re<eta, D^-1 b> with respect to the links and
// kappa, given x = D^-1 b and y = D^-dag eta (FP64).
//
// With dL = -Re<y, dD x> and D = T - kappa H, T = 1 - c_sw kappa C,
// C = sum_{mu<nu} sigma_{mu nu} F_{mu nu}:
//   link gradient G (dL = Re sum conj(G_ab) dU_ab, PyTorch's convention)
//     hopping:  kappa s sum_spin [ ((1 - g_mu) y(x)) x(x+mu)^dag + x(x) ((1 + g_mu) y(x+mu))^dag ]
//     clover :  every plaquette loop E0 E1 E2 E3 (corners c0..c3, c_j at the
//               start of edge E_j) enters Q at each of its corners, so
//               dL = sum_plaquettes sum_j Re[z tr(rot_j(E0 E1 E2 E3) K(c_j))],
//               z = -i c_sw kappa / 8, K = M' + M'^dag, M' the traceless part
//               of M_ab = sum_{s,t} sigma_st x_t,a conj(y_s,b).  For the edge at
//               position i the derivative is X_i = sum_j (loop from edge i+1
//               round to edge i-1 with K(c_j) inserted at corner j), and
//               G += conj(z) X_i^dag (edge U) or z X_i (edge U^dag).
//   kappa:  dL/dkappa = Re<y, H x> + c_sw Re<y, C x>.
// The kernel gathers, for each link, the 6 plaquettes that contain it.
#include "wcl_launch.h"

namespace wcl {

// --- 3x3 helpers (FP64) -------------------------------------------------------
struct Mat {
    cplx<double> a[9];
};

WCL_D Mat mmul(const Mat &A, const Mat &B)
{
    Mat C;
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

WCL_D Mat mdag(const Mat &A)
{
    Mat C;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) C.a[i * 3 + j] = {A.a[j * 3 + i].re, -A.a[j * 3 + i].im};
    return C;
}

WCL_D Mat madd(const Mat &A, const Mat &B)
{
    Mat C;
#pragma unroll
    for (int k = 0; k < 9; k++) C.a[k] = A.a[k] + B.a[k];
    return C;
}

WCL_D int gcoords_to_h(const Geom &g, const int x[4])
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

// site x + d (periodic), its parity and half index
WCL_D void shifted(const Geom &g, const int x[4], const int d[4], int &p, int &h)
{
    int y[4];
#pragma unroll
    for (int k = 0; k < 4; k++) y[k] = (x[k] + d[k] + 2 * g.L[k]) % g.L[k];
    p = (y[0] + y[1] + y[2] + y[3]) & 1;
    h = gcoords_to_h(g, y);
}

WCL_D Mat link_at_d(const Geom &g, const void *u64, const int x[4], const int d[4], int mu)
{
    int p, h;
    shifted(g, x, d, p, h);
    Mat m;
    load_link<double, double>(u64, mu, p, h, g.Vh, m.a);
    return m;
}

// K field: double2 [2 p][6 planes][9][Vh]
WCL_D Mat K_at(const Geom &g, const double2 *K, const int x[4], const int d[4], int plane)
{
    int p, h;
    shifted(g, x, d, p, h);
    Mat m;
    const size_t base = ((size_t)p * 6 + plane) * 9;
#pragma unroll
    for (int k = 0; k < 9; k++) {
        const double2 v = K[(base + k) * g.Vh + h];
        m.a[k] = {v.x, v.y};
    }
    return m;
}

// sigma_{mu nu} in the chiral basis is diag(e_up s_m, e_lo s_m) (2x2 blocks):
//   xy: -s3, xz: +s2, yz: -s1 (both blocks);  xt: s1, yt: s2, zt: s3 (upper), minus them (lower).
// plane order: (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)
__host__ __device__ constexpr int plane_pauli(int p) { return p == 0 ? 3 : p == 1 ? 2 : p == 2 ? 1 : p == 3 ? 1 : p == 4 ? 2 : 3; }
__host__ __device__ constexpr double plane_up(int p) { return (p == 0 || p == 3) ? -1.0 : 1.0; }
__host__ __device__ constexpr double plane_lo(int p) { return (p == 2 || p == 4 || p == 5) ? -1.0 : (p == 0 || p == 3 ? -1.0 : 1.0); }

// Pauli matrix entries (s, t)
WCL_D cplx<double> pauli(int m, int s, int t)
{
    if (m == 1) return (s != t) ? cplx<double>{1.0, 0.0} : cplx<double>{0.0, 0.0};
    if (m == 2) {
        if (s == 0 && t == 1) return {0.0, -1.0};
        if (s == 1 && t == 0) return {0.0, 1.0};
        return {0.0, 0.0};
    }
    if (s != t) return {0.0, 0.0};
    return {s == 0 ? 1.0 : -1.0, 0.0};
}

// K_plane(x) for all 6 planes at one site.
__global__ void __launch_bounds__(128) k_grad_K(Geom g, const double2 *X, const double2 *Y, double2 *K)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 2 * g.Vh) return;
    const int p = idx / g.Vh;
    const int h = idx - p * g.Vh;
    cplx<double> xs[12], ys[12];
    load_spinor<double, double>(X + (size_t)p * 12 * g.Vh, h, g.Vh, xs);
    load_spinor<double, double>(Y + (size_t)p * 12 * g.Vh, h, g.Vh, ys);
    for (int pl = 0; pl < 6; pl++) {
        const int m = plane_pauli(pl);
        cplx<double> M[9];
#pragma unroll
        for (int k = 0; k < 9; k++) M[k] = {0.0, 0.0};
        for (int blk = 0; blk < 2; blk++) {
            const double e = blk == 0 ? plane_up(pl) : plane_lo(pl);
            for (int s = 0; s < 2; s++)
                for (int t = 0; t < 2; t++) {
                    const cplx<double> sg = e * pauli(m, s, t);
                    if (sg.re == 0.0 && sg.im == 0.0) continue;
                    // M_ab += sigma_st x_t,a conj(y_s,b)
                    for (int a = 0; a < 3; a++)
                        for (int b = 0; b < 3; b++) {
                            const cplx<double> xy = {xs[(2 * blk + t) * 3 + a].re, xs[(2 * blk + t) * 3 + a].im};
                            const cplx<double> yc = {ys[(2 * blk + s) * 3 + b].re, -ys[(2 * blk + s) * 3 + b].im};
                            M[a * 3 + b] = M[a * 3 + b] + sg * (xy * yc);
                        }
                }
        }
        cplx<double> tr = {(M[0].re + M[4].re + M[8].re) / 3.0, (M[0].im + M[4].im + M[8].im) / 3.0};
        M[0] = M[0] - tr; M[4] = M[4] - tr; M[8] = M[8] - tr;
        const size_t base = ((size_t)p * 6 + pl) * 9;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                const cplx<double> v = {M[a * 3 + b].re + M[b * 3 + a].re, M[a * 3 + b].im - M[b * 3 + a].im};
                K[(base + a * 3 + b) * g.Vh + h] = make_double2(v.re, v.im);
            }
    }
}

WCL_D int plane_index(int a, int b)
{
    // a < b
    return a == 0 ? (b - 1) : a == 1 ? (b + 1) : 5;
}

// Link gradient at (parity p, h, direction mu): hopping + clover.
__global__ void __launch_bounds__(64) k_grad_link(Geom g, const void *u64, const double2 *X, const double2 *Y,
                                                  const double2 *K, double kappa, double csw, void *G)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 8 * g.Vh) return;
    const int mu = idx / (2 * g.Vh);
    const int rem = idx - mu * 2 * g.Vh;
    const int p = rem / g.Vh;
    const int h = rem - p * g.Vh;
    const Site s = decompose(g, h, p);
    const int *x = s.x;
    Mat Gm;
#pragma unroll
    for (int k = 0; k < 9; k++) Gm.a[k] = {0.0, 0.0};

    // hopping part
    {
        int d[4] = {0, 0, 0, 0};
        d[mu] = 1;
        int pf, hf;
        shifted(g, x, d, pf, hf);
        cplx<double> xn[12], yn[12], xf[12], yf[12];
        load_spinor<double, double>(X + (size_t)p * 12 * g.Vh, h, g.Vh, xn);
        load_spinor<double, double>(Y + (size_t)p * 12 * g.Vh, h, g.Vh, yn);
        load_spinor<double, double>(X + (size_t)pf * 12 * g.Vh, hf, g.Vh, xf);
        load_spinor<double, double>(Y + (size_t)pf * 12 * g.Vh, hf, g.Vh, yf);
        cplx<double> w[12], v[12], hh[6];
#pragma unroll
        for (int k = 0; k < 12; k++) { w[k] = {0.0, 0.0}; v[k] = {0.0, 0.0}; }
        switch (mu) {
        case 0: project<0, -1, double>(yn, hh); accumulate<0, -1, double>(w, hh);
                project<0, 1, double>(yf, hh); accumulate<0, 1, double>(v, hh); break;
        case 1: project<1, -1, double>(yn, hh); accumulate<1, -1, double>(w, hh);
                project<1, 1, double>(yf, hh); accumulate<1, 1, double>(v, hh); break;
        case 2: project<2, -1, double>(yn, hh); accumulate<2, -1, double>(w, hh);
                project<2, 1, double>(yf, hh); accumulate<2, 1, double>(v, hh); break;
        default: project<3, -1, double>(yn, hh); accumulate<3, -1, double>(w, hh);
                 project<3, 1, double>(yf, hh); accumulate<3, 1, double>(v, hh); break;
        }
        const double sgn = (mu == 3 && g.tbc < 0 && x[3] == g.L[3] - 1) ? -1.0 : 1.0;
        const double c = kappa * sgn;
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                cplx<double> acc = {0.0, 0.0};
                for (int sp = 0; sp < 4; sp++) {
                    acc = cjfma(xf[sp * 3 + b], w[sp * 3 + a], acc);   // w_a conj(x'_b)
                    acc = cjfma(v[sp * 3 + b], xn[sp * 3 + a], acc);   // x_a conj(v_b)
                }
                Gm.a[a * 3 + b] = Gm.a[a * 3 + b] + c * acc;
            }
    }

    // clover part: the 6 plaquettes containing U_mu(x)
    const cplx<double> z = {0.0, -csw * kappa / 8.0};
    for (int nu = 0; nu < 4; nu++) {
        if (nu == mu) continue;
        const int a = mu < nu ? mu : nu, b = mu < nu ? nu : mu;
        const int pl = plane_index(a, b);
        for (int which = 0; which < 2; which++) {
            // lower-left corner c0 and the position i of U_mu(x) in E0 E1 E2 E3
            int c0[4] = {x[0], x[1], x[2], x[3]};
            int pos;
            if (mu == a) {
                pos = which == 0 ? 0 : 2;
                if (which == 1) c0[nu] -= 1;
            } else {
                pos = which == 0 ? 1 : 3;
                if (which == 0) c0[nu] -= 1;
            }
            int da[4] = {0, 0, 0, 0}, db[4] = {0, 0, 0, 0}, dab[4] = {0, 0, 0, 0}, o[4] = {0, 0, 0, 0};
            da[a] = 1; db[b] = 1; dab[a] = 1; dab[b] = 1;
            Mat E[4], Kc[4];
            E[0] = link_at_d(g, u64, c0, o, a);
            E[1] = link_at_d(g, u64, c0, da, b);
            E[2] = mdag(link_at_d(g, u64, c0, db, a));
            E[3] = mdag(link_at_d(g, u64, c0, o, b));
            Kc[0] = K_at(g, K, c0, o, pl);
            Kc[1] = K_at(g, K, c0, da, pl);
            Kc[2] = K_at(g, K, c0, dab, pl);
            Kc[3] = K_at(g, K, c0, db, pl);
            // X_i = sum_j (E_{i+1} .. with K_j inserted at corner j)
            const int i1 = (pos + 1) & 3, i2 = (pos + 2) & 3, i3 = (pos + 3) & 3;
            Mat X = mmul(mmul(Kc[i1], E[i1]), mmul(E[i2], E[i3]));
            X = madd(X, mmul(mmul(E[i1], Kc[i2]), mmul(E[i2], E[i3])));
            X = madd(X, mmul(mmul(E[i1], E[i2]), mmul(Kc[i3], E[i3])));
            X = madd(X, mmul(mmul(E[i1], E[i2]), mmul(E[i3], Kc[pos])));
            const bool daggered = (pos >= 2);
            if (!daggered) {
                const Mat Xd = mdag(X);
                const cplx<double> zc = {z.re, -z.im};
#pragma unroll
                for (int k = 0; k < 9; k++) Gm.a[k] = Gm.a[k] + zc * Xd.a[k];
            } else {
#pragma unroll
                for (int k = 0; k < 9; k++) Gm.a[k] = Gm.a[k] + z * X.a[k];
            }
        }
    }
    store_link<double, double>(G, mu, p, h, g.Vh, Gm.a);
}

// C x = sum_{mu<nu} sigma_{mu nu} F_{mu nu} x on one parity, from the links.
WCL_D Mat fs_from_links(const Geom &g, const void *u64, const int x[4], int mu, int nu)
{
    int o[4] = {0, 0, 0, 0};
    int pm[4] = {0, 0, 0, 0}, pn[4] = {0, 0, 0, 0}, mm[4] = {0, 0, 0, 0}, mn[4] = {0, 0, 0, 0};
    int mmpn[4] = {0, 0, 0, 0}, mmmn[4] = {0, 0, 0, 0}, pmmn[4] = {0, 0, 0, 0};
    pm[mu] = 1; pn[nu] = 1; mm[mu] = -1; mn[nu] = -1;
    mmpn[mu] = -1; mmpn[nu] = 1;
    mmmn[mu] = -1; mmmn[nu] = -1;
    pmmn[mu] = 1; pmmn[nu] = -1;
    const Mat Umu = link_at_d(g, u64, x, o, mu), Unu = link_at_d(g, u64, x, o, nu);
    Mat Q = mmul(mmul(Umu, link_at_d(g, u64, x, pm, nu)), mmul(mdag(link_at_d(g, u64, x, pn, mu)), mdag(Unu)));
    Q = madd(Q, mmul(mmul(Unu, mdag(link_at_d(g, u64, x, mmpn, mu))),
                     mmul(mdag(link_at_d(g, u64, x, mm, nu)), link_at_d(g, u64, x, mm, mu))));
    Q = madd(Q, mmul(mmul(mdag(link_at_d(g, u64, x, mm, mu)), mdag(link_at_d(g, u64, x, mmmn, nu))),
                     mmul(link_at_d(g, u64, x, mmmn, mu), link_at_d(g, u64, x, mn, nu))));
    Q = madd(Q, mmul(mmul(mdag(link_at_d(g, u64, x, mn, nu)), link_at_d(g, u64, x, mn, mu)),
                     mmul(link_at_d(g, u64, x, pmmn, nu), mdag(Umu))));
    Mat F;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            const double wr = Q.a[i * 3 + j].re - Q.a[j * 3 + i].re;
            const double wi = Q.a[i * 3 + j].im + Q.a[j * 3 + i].im;
            F.a[i * 3 + j] = {wi * 0.125, -wr * 0.125};
        }
    const double tr = (F.a[0].re + F.a[4].re + F.a[8].re) / 3.0;
    F.a[0].re -= tr; F.a[4].re -= tr; F.a[8].re -= tr;
    F.a[0].im = F.a[4].im = F.a[8].im = 0.0;
    return F;
}

__global__ void __launch_bounds__(64) k_sigmaF(Geom g, const void *u64, const double2 *X, double2 *out)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 2 * g.Vh) return;
    const int p = idx / g.Vh;
    const int h = idx - p * g.Vh;
    const Site s = decompose(g, h, p);
    cplx<double> xs[12], o[12];
    load_spinor<double, double>(X + (size_t)p * 12 * g.Vh, h, g.Vh, xs);
#pragma unroll
    for (int k = 0; k < 12; k++) o[k] = {0.0, 0.0};
    const int pa[6] = {0, 0, 0, 1, 1, 2}, pb[6] = {1, 2, 3, 2, 3, 3};
    for (int pl = 0; pl < 6; pl++) {
        const Mat F = fs_from_links(g, u64, s.x, pa[pl], pb[pl]);
        const int m = plane_pauli(pl);
        for (int blk = 0; blk < 2; blk++) {
            const double e = blk == 0 ? plane_up(pl) : plane_lo(pl);
            for (int sp = 0; sp < 2; sp++)
                for (int t = 0; t < 2; t++) {
                    const cplx<double> sg = e * pauli(m, sp, t);
                    if (sg.re == 0.0 && sg.im == 0.0) continue;
                    for (int a = 0; a < 3; a++) {
                        cplx<double> acc = {0.0, 0.0};
                        for (int b = 0; b < 3; b++) acc = cfma(F.a[a * 3 + b], xs[(2 * blk + t) * 3 + b], acc);
                        o[(2 * blk + sp) * 3 + a] = o[(2 * blk + sp) * 3 + a] + sg * acc;
                    }
                }
        }
    }
    store_spinor<double, double>(out + (size_t)p * 12 * g.Vh, h, g.Vh, o);
}

// Internal link field -> canonical [V][4][3][3] complex128.
__global__ void k_export_links(Geom g, const void *G, double2 *canon)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= 2 * g.Vh) return;
    int x[4];
    int r = n;
    x[0] = r % g.L[0]; r /= g.L[0];
    x[1] = r % g.L[1]; r /= g.L[1];
    x[2] = r % g.L[2];
    x[3] = r / g.L[2];
    const int p = (x[0] + x[1] + x[2] + x[3]) & 1;
    const int h = gcoords_to_h(g, x);
    for (int mu = 0; mu < 4; mu++) {
        cplx<double> u[9];
        load_link<double, double>(G, mu, p, h, g.Vh, u);
        for (int k = 0; k < 9; k++) canon[((size_t)n * 4 + mu) * 9 + k] = make_double2(u[k].re, u[k].im);
    }
}

// gamma5 on FP64 e/o fields (nsec sections of Vh sites): negate spins 2, 3.
__global__ void k_gamma5(size_t nsec, size_t Vh, double2 *f)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nsec * Vh) return;
    const size_t sec = i / Vh, h = i - sec * Vh;
    double2 *b = f + sec * 12 * Vh;
#pragma unroll
    for (int c = 6; c < 12; c++) {
        const double2 v = b[c * Vh + h];
        b[c * Vh + h] = make_double2(-v.x, -v.y);
    }
}

hipError_t launch_grad(const Geom &g, const void *u64, const void *X, const void *Y, void *K, double kappa,
                       double csw, void *G, hipStream_t st)
{
    const int n2 = 2 * g.Vh;
    k_grad_K<<<(n2 + 127) / 128, 128, 0, st>>>(g, (const double2 *)X, (const double2 *)Y, (double2 *)K);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int n8 = 8 * g.Vh;
    k_grad_link<<<(n8 + 63) / 64, 64, 0, st>>>(g, u64, (const double2 *)X, (const double2 *)Y, (const double2 *)K,
                                               kappa, csw, G);
    return hipGetLastError();
}

hipError_t launch_sigmaF(const Geom &g, const void *u64, const void *X, void *out, hipStream_t st)
{
    const int n2 = 2 * g.Vh;
    k_sigmaF<<<(n2 + 63) / 64, 64, 0, st>>>(g, u64, (const double2 *)X, (double2 *)out);
    return hipGetLastError();
}

hipError_t launch_export_links(const Geom &g, const void *G, double *canon, hipStream_t st)
{
    const int n = 2 * g.Vh;
    k_export_links<<<(n + 127) / 128, 128, 0, st>>>(g, G, (double2 *)canon);
    return hipGetLastError();
}

hipError_t launch_gamma5(size_t nsec, size_t Vh, void *f, hipStream_t st)
{
    const size_t n = nsec * Vh;
    k_gamma5<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(nsec, Vh, (double2 *)f);
    return hipGetLastError();
}

}  // namespace wcl
