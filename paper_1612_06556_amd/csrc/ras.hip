// ras.hip -- overlapped Restricted Additive Schwarz (paper Sec. 2: the
// single-precision BiCGStab is preconditioned with even/odd sites and the
// overlapped RAS of Osaki & Ishikawa).
//
// One workgroup per core tile.  The core (the tile of the blocked layout) is
// extended by `overlap` sites on every side; the block operator is the even/odd
// Schur complement of D restricted to the extended block with every hop that
// leaves it dropped (Dirichlet cut), using the global clover inverse.  The
// block system is solved by `iters` minimal-residual steps from zero and the
// result is kept on the even sites of the core only (the "restricted" part).
//
// Residency: the two parities of the block vector (the MR residual r, read by
// the odd half of the operator, and the intermediate odd vector y, read by the
// even half) live in LDS as FP32 (2 x 12 x 648 complex = 124 KB for a 4^4 core
// with overlap 1); the iterate z, the residual and the operator output stay in
// registers of the thread that owns the site; links and clover inverse stream
// from L2 / the Infinity Cache on every iteration.
#include "wcl_launch.h"

namespace wcl {

struct RasArgs {
    Geom g;
    int overlap, iters;
    const float4 *in;   // even field, float4 [6][Vh]
    float4 *out;
    const void *links;
    const void *clov_inv;
    float kappa2;
    const Scalars *sc;
};

// global (tile coordinate, in-tile coordinate) of extended-block coordinate a
WCL_D void ext_to_global(const Geom &g, int mu, int b, int a, int delta, int &tile, int &loc, int &x)
{
    if (a < delta) {
        tile = b == 0 ? g.NB[mu] - 1 : b - 1;
        loc = g.B[mu] - delta + a;
    } else if (a >= delta + g.B[mu]) {
        tile = b == g.NB[mu] - 1 ? 0 : b + 1;
        loc = a - delta - g.B[mu];
    } else {
        tile = b;
        loc = a - delta;
    }
    x = tile * g.B[mu] + loc;
}

template <int MU, int S>
WCL_D void ras_hop_dir(const float2 *src, int Ne, int nidx, float sgn, const cplx<float> u[9], bool dag,
                       cplx<float> acc[12])
{
    cplx<float> psi[12], hh[6], uh[6];
#pragma unroll
    for (int c = 0; c < 12; c++) {
        const float2 v = src[c * Ne + nidx];
        psi[c] = {v.x, v.y};
    }
    project<MU, S, float>(psi, hh);
#pragma unroll
    for (int k = 0; k < 6; k++) hh[k] = sgn * hh[k];
    if (dag) su3_dag_mul(u, hh, uh);
    else su3_mul(u, hh, uh);
    accumulate<MU, S, float>(acc, uh);
}

// Hop on one parity q of the extended block, reading the other parity from
// LDS.  nb[2*mu+0/1] = local half index of the forward / backward neighbour
// or -1 outside the block; gq = global half index of the site; gnb = global
// half index table of the other parity.
template <typename SL, int MU>
WCL_D void ras_dir(const RasArgs &a, int q, int gq, const int nb[8], const int *gnb, const float2 *src, int Ne,
                   float sf, float sb, cplx<float> acc[12])
{
    const size_t Vh = a.g.Vh;
    if (nb[2 * MU] >= 0) {
        cplx<float> u[9];
        load_link<SL, float>(a.links, MU, q, gq, Vh, u);
        ras_hop_dir<MU, -1>(src, Ne, nb[2 * MU], MU == 3 ? sf : 1.0f, u, false, acc);
    }
    if (nb[2 * MU + 1] >= 0) {
        cplx<float> u[9];
        load_link<SL, float>(a.links, MU, 1 - q, gnb[nb[2 * MU + 1]], Vh, u);
        ras_hop_dir<MU, 1>(src, Ne, nb[2 * MU + 1], MU == 3 ? sb : 1.0f, u, true, acc);
    }
}

template <int NV>
WCL_D void block_allreduce(double v[NV], double *red)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < NV; k++) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
        if (lane == 0) red[k * 16 + wid] = v[k];
    }
    __syncthreads();
    if (wid == 0) {
#pragma unroll
        for (int k = 0; k < NV; k++) {
            double t = lane < nw ? red[k * 16 + lane] : 0.0;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
            if (lane == 0) red[NV * 16 + k] = t;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; k++) v[k] = red[NV * 16 + k];
}

template <typename SL, int MAXNE>
__global__ void __launch_bounds__(MAXNE == 648 ? 704 : 128) k_ras(RasArgs a)
{
    if (a.sc && a.sc->done) return;
    __shared__ float2 sE[12 * MAXNE];
    __shared__ float2 sO[12 * MAXNE];
    __shared__ int gh[2 * MAXNE];
    __shared__ double red[4 * 16 + 4];

    const Geom &g = a.g;
    const int d = a.overlap;
    const int e0 = g.B[0] + 2 * d, e1 = g.B[1] + 2 * d, e2 = g.B[2] + 2 * d, e3 = g.B[3] + 2 * d;
    const int Ne = (e0 * e1 * e2 * e3) >> 1;
    const int e0h = e0 >> 1;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    int bc[4];
    {
        int r = blk;
        bc[0] = r % g.NB[0]; r /= g.NB[0];
        bc[1] = r % g.NB[1]; r /= g.NB[1];
        bc[2] = r % g.NB[2];
        bc[3] = r / g.NB[2];
    }

    // global half index of every site of the extended block, both parities
    for (int i = threadIdx.x; i < 2 * Ne; i += blockDim.x) {
        const int q = i >= Ne ? 1 : 0;
        int li = i - q * Ne;
        const int a0h = li % e0h; li /= e0h;
        const int a1 = li % e1; li /= e1;
        const int a2 = li % e2;
        const int a3 = li / e2;
        const int a0 = 2 * a0h + ((q + a1 + a2 + a3) & 1);
        const int av[4] = {a0, a1, a2, a3};
        int blkid = 0, lin = 0;
#pragma unroll
        for (int mu = 0; mu < 4; mu++) {
            int tile, loc, x;
            ext_to_global(g, mu, bc[mu], av[mu], d, tile, loc, x);
            blkid += tile * g.sb[mu];
            lin += loc * g.sl[mu];
        }
        gh[i] = blkid * g.Hb + (lin >> 1);
    }

    // the sites of this thread: local half index t on both parities
    const int t = threadIdx.x;
    const bool active = t < Ne;
    int nbE[8], nbO[8];
    float sfE = 1.f, sbE = 1.f, sfO = 1.f, sbO = 1.f;
    bool core = false;
#pragma unroll
    for (int k = 0; k < 8; k++) { nbE[k] = -1; nbO[k] = -1; }
    if (active) {
#pragma unroll
        for (int q = 0; q < 2; q++) {
            int li = t;
            const int a0h = li % e0h; li /= e0h;
            const int a1 = li % e1; li /= e1;
            const int a2 = li % e2;
            const int a3 = li / e2;
            const int a0 = 2 * a0h + ((q + a1 + a2 + a3) & 1);
            const int av[4] = {a0, a1, a2, a3};
            const int ev[4] = {e0, e1, e2, e3};
            const int lin = a0 + e0 * (a1 + e1 * (a2 + e2 * a3));
            int st = 1;
            int *nb = q == 0 ? nbE : nbO;
#pragma unroll
            for (int mu = 0; mu < 4; mu++) {
                nb[2 * mu] = (av[mu] + 1 < ev[mu]) ? ((lin + st) >> 1) : -1;
                nb[2 * mu + 1] = (av[mu] >= 1) ? ((lin - st) >> 1) : -1;
                st *= ev[mu];
            }
            int tile, loc, xt;
            ext_to_global(g, 3, bc[3], a3, d, tile, loc, xt);
            const float sf = (g.tbc < 0 && xt == g.L[3] - 1) ? -1.f : 1.f;
            const float sb = (g.tbc < 0 && xt == 0) ? -1.f : 1.f;
            if (q == 0) {
                sfE = sf; sbE = sb;
                core = true;
#pragma unroll
                for (int mu = 0; mu < 4; mu++)
                    if (av[mu] < d || av[mu] >= d + g.B[mu]) core = false;
            } else {
                sfO = sf; sbO = sb;
            }
        }
    }
    __syncthreads();
    const int gE = active ? gh[t] : 0;
    const int gO = active ? gh[Ne + t] : 0;
    const size_t Vh = g.Vh;

    cplx<float> r[12], z[12];
#pragma unroll
    for (int c = 0; c < 12; c++) { r[c] = {0.f, 0.f}; z[c] = {0.f, 0.f}; }
    if (active) load_spinor<float, float>(a.in, gE, Vh, r);

    for (int it = 0; it < a.iters; it++) {
        if (active) {
#pragma unroll
            for (int c = 0; c < 12; c++) sE[c * Ne + t] = make_float2(r[c].re, r[c].im);
        }
        __syncthreads();
        // odd half: y = A_oo^-1 H_oe r on the odd block sites
        if (active) {
            cplx<float> acc[12], y[12];
#pragma unroll
            for (int c = 0; c < 12; c++) acc[c] = {0.f, 0.f};
            ras_dir<SL, 0>(a, 1, gO, nbO, gh, sE, Ne, sfO, sbO, acc);
            ras_dir<SL, 1>(a, 1, gO, nbO, gh, sE, Ne, sfO, sbO, acc);
            ras_dir<SL, 2>(a, 1, gO, nbO, gh, sE, Ne, sfO, sbO, acc);
            ras_dir<SL, 3>(a, 1, gO, nbO, gh, sE, Ne, sfO, sbO, acc);
            float cl[72];
            load_clover<SL, float>(a.clov_inv, 1, gO, Vh, cl);
            clover_mul(cl, acc, y);
#pragma unroll
            for (int c = 0; c < 12; c++) sO[c * Ne + t] = make_float2(y[c].re, y[c].im);
        }
        __syncthreads();
        // even half: q = r - kappa^2 A_ee^-1 H_eo y
        cplx<float> qv[12];
#pragma unroll
        for (int c = 0; c < 12; c++) qv[c] = {0.f, 0.f};
        double dots[3] = {0.0, 0.0, 0.0};
        if (active) {
            cplx<float> acc[12], w[12];
#pragma unroll
            for (int c = 0; c < 12; c++) acc[c] = {0.f, 0.f};
            ras_dir<SL, 0>(a, 0, gE, nbE, gh + Ne, sO, Ne, sfE, sbE, acc);
            ras_dir<SL, 1>(a, 0, gE, nbE, gh + Ne, sO, Ne, sfE, sbE, acc);
            ras_dir<SL, 2>(a, 0, gE, nbE, gh + Ne, sO, Ne, sfE, sbE, acc);
            ras_dir<SL, 3>(a, 0, gE, nbE, gh + Ne, sO, Ne, sfE, sbE, acc);
            float cl[72];
            load_clover<SL, float>(a.clov_inv, 0, gE, Vh, cl);
            clover_mul(cl, acc, w);
            float qr = 0.f, qi = 0.f, qq = 0.f;
#pragma unroll
            for (int c = 0; c < 12; c++) {
                qv[c] = {fmaf(-a.kappa2, w[c].re, r[c].re), fmaf(-a.kappa2, w[c].im, r[c].im)};
                qr += qv[c].re * r[c].re + qv[c].im * r[c].im;
                qi += qv[c].re * r[c].im - qv[c].im * r[c].re;
                qq += qv[c].re * qv[c].re + qv[c].im * qv[c].im;
            }
            dots[0] = qr; dots[1] = qi; dots[2] = qq;
        }
        block_allreduce<3>(dots, red);
        if (dots[2] == 0.0) break;
        const float ar = (float)(dots[0] / dots[2]), ai = (float)(dots[1] / dots[2]);
#pragma unroll
        for (int c = 0; c < 12; c++) {
            z[c] = {z[c].re + ar * r[c].re - ai * r[c].im, z[c].im + ar * r[c].im + ai * r[c].re};
            r[c] = {r[c].re - (ar * qv[c].re - ai * qv[c].im), r[c].im - (ar * qv[c].im + ai * qv[c].re)};
        }
    }
    if (active && core) store_spinor<float, float>(a.out, gE, Vh, z);
}

int ras_threads(const Geom &g, int overlap)
{
    int n = 1;
    for (int mu = 0; mu < 4; mu++) n *= g.B[mu] + 2 * overlap;
    n >>= 1;
    return ((n + 63) / 64) * 64;
}

hipError_t launch_ras(const RasLaunch &L, hipStream_t st)
{
    const Geom &g = *L.g;
    for (int mu = 0; mu < 4; mu++)
        if (L.overlap > g.B[mu] || g.L[mu] < g.B[mu] + 2 * L.overlap) return hipErrorInvalidValue;
    int ne = 1;
    for (int mu = 0; mu < 4; mu++) ne *= g.B[mu] + 2 * L.overlap;
    ne >>= 1;
    RasArgs a;
    a.g = g;
    a.overlap = L.overlap;
    a.iters = L.iters;
    a.in = (const float4 *)L.in;
    a.out = (float4 *)L.out;
    a.links = L.links;
    a.clov_inv = L.clov_inv;
    a.kappa2 = L.kappa2;
    a.sc = L.sc;
    const int nblk = g.NB[0] * g.NB[1] * g.NB[2] * g.NB[3];
    const int threads = ras_threads(g, L.overlap);
    if (threads > 1024) return hipErrorInvalidValue;
    dim3 grid(nblk), block(threads);
    if (ne <= 128) {
        if (L.link_prec == P32) k_ras<float, 128><<<grid, block, 0, st>>>(a);
        else if (L.link_prec == P16) k_ras<__half, 128><<<grid, block, 0, st>>>(a);
        else return hipErrorInvalidValue;
    } else if (ne <= 648) {
        if (L.link_prec == P32) k_ras<float, 648><<<grid, block, 0, st>>>(a);
        else if (L.link_prec == P16) k_ras<__half, 648><<<grid, block, 0, st>>>(a);
        else return hipErrorInvalidValue;
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace wcl

namespace wcl {

void ras_work(const RasLaunch &L, double *bytes, double *flops)
{
    const Geom &g = *L.g;
    const double lb = L.link_prec == P32 ? 72.0 : 36.0, cb = L.link_prec == P32 ? 288.0 : 144.0;
    *bytes = (double)g.Vh * (8.0 * lb + 2.0 * cb + 2.0 * 96.0);
    int e[4];
    double ext = 1.0;
    for (int mu = 0; mu < 4; mu++) {
        e[mu] = g.B[mu] + 2 * L.overlap;
        ext *= e[mu];
    }
    double hops = 0.0;  // directed in-block hops per block and iteration, both parities
    for (int mu = 0; mu < 4; mu++) hops += 2.0 * (e[mu] - 1) * ext / e[mu];
    const double ne = ext / 2.0;
    // per iteration: hops, clover on every site, q = r - k^2 w (48 per even site),
    // two dot products (96) and the z, r updates (96)
    const double per_iter = hops * 168.0 + ext * 504.0 + ne * (48.0 + 96.0 + 96.0);
    const double nblk = (double)g.NB[0] * g.NB[1] * g.NB[2] * g.NB[3];
    *flops = per_iter * L.iters * nblk;
}

}  // namespace wcl
