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
    int nrhs;
    size_t stride;   // bytes between right-hand sides
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

// One hop of the block operator: the neighbour spinor comes from LDS, the
// link from global memory; a neighbour outside the extended block is replaced
// by the site itself with weight 0 (Dirichlet cut without divergent branches).
struct RasStage {
    cplx<float> u[9];
    uint32_t ln;   // local half index of the neighbour (other parity)
    float w;       // 0 (outside the block), else the t boundary sign
};

WCL_D void ras_fence(cplx<float> acc[12], uint32_t &a, uint32_t &b)
{
    asm volatile(""
                 : "+v"(acc[0].re), "+v"(acc[0].im), "+v"(acc[1].re), "+v"(acc[1].im), "+v"(acc[2].re),
                   "+v"(acc[2].im), "+v"(acc[3].re), "+v"(acc[3].im), "+v"(acc[4].re), "+v"(acc[4].im),
                   "+v"(acc[5].re), "+v"(acc[5].im), "+v"(acc[6].re), "+v"(acc[6].im), "+v"(acc[7].re),
                   "+v"(acc[7].im), "+v"(acc[8].re), "+v"(acc[8].im), "+v"(acc[9].re), "+v"(acc[9].im),
                   "+v"(acc[10].re), "+v"(acc[10].im), "+v"(acc[11].re), "+v"(acc[11].im), "+v"(a), "+v"(b));
}

// nb: packed neighbour table, entry K = forward (K even) / backward (K odd)
// in direction K/2: the local half index of the other parity, 0xffff if the
// neighbour is outside the block.  The link of hop K is prefetched (global
// memory, long latency) one hop ahead; the neighbour spinor is read from LDS
// when the hop is computed.
template <typename SL, int K>
WCL_D void ras_load(const void *links, int q, uint32_t gq, uint32_t Vh, uint32_t t, const uint32_t nb[4],
                    const int *gnb, float sf, float sb, RasStage &st, cplx<float> acc[12])
{
    constexpr int MU = K >> 1;
    constexpr bool FWD = (K & 1) == 0;
    uint32_t ln = (nb[MU] >> (FWD ? 0 : 16)) & 0xffffu;
    const bool in = ln != 0xffffu;
    if (!in) ln = t;                       // any valid site; its weight is 0
    uint32_t gl = FWD ? gq : (uint32_t)gnb[ln];
    ras_fence(acc, ln, gl);
    load_link<SL, float>(links, MU, FWD ? q : 1 - q, gl, Vh, st.u);
    st.ln = ln;
    st.w = in ? (MU == 3 ? (FWD ? sf : sb) : 1.f) : 0.f;
}

template <int K, int NE>
WCL_D void ras_compute(const RasStage &st, const float2 *src, cplx<float> acc[12])
{
    constexpr int MU = K >> 1;
    constexpr bool FWD = (K & 1) == 0;
    constexpr int S = FWD ? -1 : 1;
    cplx<float> psi[12], hh[6], uh[6];
#pragma unroll
    for (int c = 0; c < 12; c++) {
        const float2 v = src[c * NE + st.ln];
        psi[c] = {v.x, v.y};
    }
    project<MU, S, float>(psi, hh);
#pragma unroll
    for (int k = 0; k < 6; k++) hh[k] = st.w * hh[k];
    if (FWD) su3_mul(st.u, hh, uh);
    else su3_dag_mul(st.u, hh, uh);
    accumulate<MU, S, float>(acc, uh);
}

// acc = (block hop of the other parity, read from src) at this thread's site
template <typename SL, int NE>
WCL_D void ras_hop(const void *links, int q, uint32_t gq, uint32_t Vh, uint32_t t, const uint32_t nb[4],
                   const int *gnb, const float2 *src, float sf, float sb, cplx<float> acc[12])
{
    RasStage A, B;
#pragma unroll
    for (int c = 0; c < 12; c++) acc[c] = {0.f, 0.f};
    ras_load<SL, 0>(links, q, gq, Vh, t, nb, gnb, sf, sb, A, acc);
    ras_load<SL, 1>(links, q, gq, Vh, t, nb, gnb, sf, sb, B, acc);
    ras_compute<0, NE>(A, src, acc);
    ras_load<SL, 2>(links, q, gq, Vh, t, nb, gnb, sf, sb, A, acc);
    ras_compute<1, NE>(B, src, acc);
    ras_load<SL, 3>(links, q, gq, Vh, t, nb, gnb, sf, sb, B, acc);
    ras_compute<2, NE>(A, src, acc);
    ras_load<SL, 4>(links, q, gq, Vh, t, nb, gnb, sf, sb, A, acc);
    ras_compute<3, NE>(B, src, acc);
    ras_load<SL, 5>(links, q, gq, Vh, t, nb, gnb, sf, sb, B, acc);
    ras_compute<4, NE>(A, src, acc);
    ras_load<SL, 6>(links, q, gq, Vh, t, nb, gnb, sf, sb, A, acc);
    ras_compute<5, NE>(B, src, acc);
    ras_load<SL, 7>(links, q, gq, Vh, t, nb, gnb, sf, sb, B, acc);
    ras_compute<6, NE>(A, src, acc);
    ras_compute<7, NE>(B, src, acc);
}

// out = A acc, one chirality block at a time; each block's loads wait for
// the preceding work (fence), which keeps 36 clover reals live, not 72.
template <typename SL>
WCL_D void ras_clover(const void *clov, int q, uint32_t gq, uint32_t Vh, cplx<float> acc[12], cplx<float> out[12])
{
#pragma unroll
    for (int half = 0; half < 2; half++) {
        uint32_t gc = gq, dummy = 0;
        ras_fence(acc, gc, dummy);
        float cl[36];
        load_clover_half<typename ClovS<SL>::T, float>(clov, q, gc, Vh, half, cl);
        clover_mul_half(cl, acc + 6 * half, out + 6 * half);
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
    // workgroup id = tile * nrhs + rhs (the right-hand sides of one tile share
    // its links and clover through L2)
    const int lin = xcd_block(blockIdx.x, gridDim.x);
    const int rhs = lin % a.nrhs;
    const int blk = lin / a.nrhs;
    if (a.sc && a.sc[rhs].done) return;
    const float4 *rin = (const float4 *)((const char *)a.in + rhs * a.stride);
    float4 *rout = (float4 *)((char *)a.out + rhs * a.stride);
    // component-major with the compile-time stride MAXNE (immediate LDS offsets)
    __shared__ float2 sE[12 * MAXNE];   // MR residual r on the even block sites
    __shared__ float2 sO[12 * MAXNE];   // y = A_oo^-1 H_oe r on the odd block sites
    __shared__ int gh[2 * MAXNE];       // global half index of every block site
    __shared__ double red[4 * 16 + 4];

    const Geom &g = a.g;
    const int d = a.overlap;
    const int e0 = g.B[0] + 2 * d, e1 = g.B[1] + 2 * d, e2 = g.B[2] + 2 * d, e3 = g.B[3] + 2 * d;
    const int Ne = (e0 * e1 * e2 * e3) >> 1;
    const int e0h = e0 >> 1;
    int bc[4];
    {
        int r = blk;
        bc[0] = r % g.NB[0]; r /= g.NB[0];
        bc[1] = r % g.NB[1]; r /= g.NB[1];
        bc[2] = r % g.NB[2];
        bc[3] = r / g.NB[2];
    }

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
        gh[q * MAXNE + (i - q * Ne)] = blkid * g.Hb + (lin >> 1);
    }

    // this thread owns local half index t on both parities
    const uint32_t t = threadIdx.x;
    const bool active = (int)t < Ne;
    uint32_t nbE[4], nbO[4];
    float sfE = 1.f, sbE = 1.f, sfO = 1.f, sbO = 1.f;
    bool core = false;
#pragma unroll
    for (int k = 0; k < 4; k++) { nbE[k] = 0xffffffffu; nbO[k] = 0xffffffffu; }
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
            uint32_t *nb = q == 0 ? nbE : nbO;
#pragma unroll
            for (int mu = 0; mu < 4; mu++) {
                const uint32_t f = (av[mu] + 1 < ev[mu]) ? (uint32_t)((lin + st) >> 1) : 0xffffu;
                const uint32_t bk = (av[mu] >= 1) ? (uint32_t)((lin - st) >> 1) : 0xffffu;
                nb[mu] = f | (bk << 16);
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
    const uint32_t gE = active ? (uint32_t)gh[t] : 0u;
    const uint32_t gO = active ? (uint32_t)gh[MAXNE + t] : 0u;
    const uint32_t Vh = g.Vh;

    // r = the input on the even block sites (zero start: z = 0, r = rhs)
    if (active) {
        cplx<float> r[12];
        load_spinor<float, float>(rin, gE, Vh, r);
#pragma unroll
        for (int c = 0; c < 12; c++) sE[c * MAXNE + t] = make_float2(r[c].re, r[c].im);
    }

    for (int it = 0; it < a.iters; it++) {
        __syncthreads();
        // odd half: y = A_oo^-1 H_oe r on the odd block sites
        if (active) {
            cplx<float> acc[12], y[12];
            ras_hop<SL, MAXNE>(a.links, 1, gO, Vh, t, nbO, gh, sE, sfO, sbO, acc);
            ras_clover<SL>(a.clov_inv, 1, gO, Vh, acc, y);
#pragma unroll
            for (int c = 0; c < 12; c++) sO[c * MAXNE + t] = make_float2(y[c].re, y[c].im);
        }
        __syncthreads();
        // even half: q = r - kappa^2 A_ee^-1 H_eo y
        cplx<float> qv[12];
        double dots[3] = {0.0, 0.0, 0.0};
        if (active) {
            cplx<float> acc[12], w[12];
            ras_hop<SL, MAXNE>(a.links, 0, gE, Vh, t, nbE, gh + MAXNE, sO, sfE, sbE, acc);
            ras_clover<SL>(a.clov_inv, 0, gE, Vh, acc, w);
            float qr = 0.f, qi = 0.f, qq = 0.f;
#pragma unroll
            for (int c = 0; c < 12; c++) {
                const float2 r = sE[c * MAXNE + t];
                qv[c] = {fmaf(-a.kappa2, w[c].re, r.x), fmaf(-a.kappa2, w[c].im, r.y)};
                qr += qv[c].re * r.x + qv[c].im * r.y;
                qi += qv[c].re * r.y - qv[c].im * r.x;
                qq += qv[c].re * qv[c].re + qv[c].im * qv[c].im;
            }
            dots[0] = qr; dots[1] = qi; dots[2] = qq;
        } else {
#pragma unroll
            for (int c = 0; c < 12; c++) qv[c] = {0.f, 0.f};
        }
        block_allreduce<3>(dots, red);
        if (dots[2] == 0.0) break;
        const float ar = (float)(dots[0] / dots[2]), ai = (float)(dots[1] / dots[2]);
        if (active) {
            // z += alpha r (kept only where it is written: the core), r -= alpha q
            cplx<float> z[12];
            if (core) {
                if (it == 0) {
#pragma unroll
                    for (int c = 0; c < 12; c++) z[c] = {0.f, 0.f};
                } else {
                    load_spinor<float, float>(rout, gE, Vh, z);
                }
            }
#pragma unroll
            for (int c = 0; c < 12; c++) {
                const float2 r = sE[c * MAXNE + t];
                if (core) z[c] = {z[c].re + ar * r.x - ai * r.y, z[c].im + ar * r.y + ai * r.x};
                sE[c * MAXNE + t] = make_float2(r.x - (ar * qv[c].re - ai * qv[c].im), r.y - (ar * qv[c].im + ai * qv[c].re));
            }
            if (core) store_spinor<float, float>(rout, gE, Vh, z);
        }
    }
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
    // several right-hand sides need a stride of at least one even field
    if (L.nrhs < 1 || L.nrhs > 4096) return hipErrorInvalidValue;
    if (L.nrhs > 1 && L.stride < spinor_bytes(4, (size_t)g.Vh)) return hipErrorInvalidValue;
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
    a.nrhs = L.nrhs;
    a.stride = L.stride;
    const int nblk = g.NB[0] * g.NB[1] * g.NB[2] * g.NB[3];
    const int threads = ras_threads(g, L.overlap);
    if (threads > 1024) return hipErrorInvalidValue;
    dim3 grid(nblk * a.nrhs), block(threads);
    if (ne <= 128) {
        if (L.link_prec == P32) k_ras<float, 128><<<grid, block, 0, st>>>(a);
        else if (L.link_prec == P16) k_ras<__half, 128><<<grid, block, 0, st>>>(a);
        else if (L.link_prec == P32C) k_ras<R12f, 128><<<grid, block, 0, st>>>(a);
        else if (L.link_prec == P16C) k_ras<R12h, 128><<<grid, block, 0, st>>>(a);
        else return hipErrorInvalidValue;
    } else if (ne <= 648) {
        if (L.link_prec == P32) k_ras<float, 648><<<grid, block, 0, st>>>(a);
        else if (L.link_prec == P16) k_ras<__half, 648><<<grid, block, 0, st>>>(a);
        else if (L.link_prec == P32C) k_ras<R12f, 648><<<grid, block, 0, st>>>(a);
        else if (L.link_prec == P16C) k_ras<R12h, 648><<<grid, block, 0, st>>>(a);
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
    const double lb = L.link_prec == P32 ? 72.0 : L.link_prec == P16 ? 36.0 : L.link_prec == P32C ? 48.0 : 24.0;
    const double cb = (L.link_prec == P32 || L.link_prec == P32C) ? 288.0 : 144.0;
    const double nr = L.nrhs > 0 ? L.nrhs : 1;
    *bytes = (double)g.Vh * (8.0 * lb + 2.0 * cb + nr * 2.0 * 96.0);
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
    *flops = per_iter * L.iters * nblk * nr;
}

}  // namespace wcl
