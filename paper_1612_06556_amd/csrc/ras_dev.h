// ras_dev.h -- device code of the overlapped Restricted Additive Schwarz
// block solve, shared by the per-launch kernel (k_ras) and the persistent
// inner solver.  See ras.hip for the method.
#pragma once

#include "wcl_launch.h"

namespace wcl {

struct RasArgs {
    Geom g;
    int overlap, iters;
    const void *in;     // even field (FP32 or FP16 storage, per the SV parameter)
    void *out;
    const void *links;
    const void *clov_inv;
    float kappa2;
    const Scalars *sc;
    int nrhs;
    size_t stride;   // bytes between right-hand sides
    int colour;      // 0: every block; k + 1: only the blocks of colour k
    int accumulate;  // add the restricted result to the output instead of writing it
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
// link from global memory (held encoded until the hop is computed); a hop
// that leaves the extended block reads a zero link and any valid LDS site
// (Dirichlet cut without divergent branches).
template <typename SL>
struct RasStage {
    LinkRaw<SL> u;
    uint32_t ln;   // local half index of the neighbour (other parity)
    float w;       // the t boundary sign (t hops only)
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

// Per-thread constants of one parity's half of the block operator.
struct RasSite {
    uint32_t g;      // global half index of the site
    uint32_t nb[4];  // packed neighbour table (see ras_load)
    float sf, sb;    // t boundary signs of the forward / backward t hop
};

// nb: entry K = forward (K even) / backward (K odd) in direction K/2: the
// local half index of the other parity, 0xffff if the neighbour is outside
// the block.  The link of hop K is loaded (global memory, long latency) one
// hop ahead; the neighbour spinor is read from LDS when the hop is computed.
template <typename SL, int K>
WCL_D void ras_load(const void *links, int q, const RasSite &S, uint32_t Vh, uint32_t t, const int *gnb,
                    RasStage<SL> &st, cplx<float> acc[12])
{
    constexpr int MU = K >> 1;
    constexpr bool FWD = (K & 1) == 0;
    uint32_t ln = (S.nb[MU] >> (FWD ? 0 : 16)) & 0xffffu;
    const bool in = ln != 0xffffu;
    if (!in) ln = t;                       // any valid site; its weight is 0
    uint32_t gl = FWD ? S.g : (uint32_t)gnb[ln];
    ras_fence(acc, ln, gl);
    // a cut hop reads a zero link (out-of-range buffer offsets: no memory
    // traffic, no branch)
    load_link_raw_or_zero<SL>(field_rsrc(links), MU, FWD ? q : 1 - q, gl, in, Vh, st.u);
    st.ln = ln;
    st.w = MU == 3 ? (FWD ? S.sf : S.sb) : 1.f;   // used on t hops only
}

template <typename SL, int K, int NE>
WCL_D void ras_compute(const RasStage<SL> &st, const float2 *src, cplx<float> acc[12])
{
    constexpr int MU = K >> 1;
    constexpr bool FWD = (K & 1) == 0;
    constexpr int S = FWD ? -1 : 1;
    cplx<float> psi[12], hh[6], uh[6], u[9];
#pragma unroll
    for (int c = 0; c < 12; c++) {
        const float2 v = src[c * NE + st.ln];
        psi[c] = {v.x, v.y};
    }
    project<MU, S, float>(psi, hh);
    // the weight carries the t boundary sign (a cut hop has a zero link)
    if constexpr (MU == 3) {
#pragma unroll
        for (int k = 0; k < 6; k++) hh[k] = st.w * hh[k];
    }
    expand_link<SL, float>(st.u, u);
    if (FWD) su3_mul(u, hh, uh);
    else su3_dag_mul(u, hh, uh);
    accumulate<MU, S, float>(acc, uh);
}

// The first two link loads of a pass, then acc = 0.  The loads' fences take
// the previous pass's accumulator, so they wait for the work that consumed
// it.  (The workgroup barriers wait for LDS operations only, so loads issued
// before the barrier that ends the previous pass would stay in flight across
// it; that measured no faster, and the longer live ranges spill.)
template <typename SL>
WCL_D void ras_hop_start(const void *links, int q, const RasSite &S, uint32_t Vh, uint32_t t, const int *gnb,
                         RasStage<SL> &A, RasStage<SL> &B, cplx<float> acc[12])
{
    ras_load<SL, 0>(links, q, S, Vh, t, gnb, A, acc);
    ras_load<SL, 1>(links, q, S, Vh, t, gnb, B, acc);
#pragma unroll
    for (int c = 0; c < 12; c++) acc[c] = {0.f, 0.f};
}

// acc = (block hop of the other parity, read from src) at this thread's
// site, then out = A^-1 acc.  Each clover half's loads wait for the
// preceding work (fence), which keeps 36 clover reals live, not 72; with an
// FP16 clover (18 registers a half) the first half is loaded while the last
// hop is computed (with FP32 the extra registers spill).
template <typename SL, int NE>
WCL_D void ras_hop_finish(const void *links, const void *clov, int q, const RasSite &S, uint32_t Vh, uint32_t t,
                          const int *gnb, const float2 *src, RasStage<SL> &A, RasStage<SL> &B, cplx<float> acc[12],
                          cplx<float> out[12])
{
    using CS = typename ClovS<SL>::T;
    ras_compute<SL, 0, NE>(A, src, acc);
    ras_load<SL, 2>(links, q, S, Vh, t, gnb, A, acc);
    ras_compute<SL, 1, NE>(B, src, acc);
    ras_load<SL, 3>(links, q, S, Vh, t, gnb, B, acc);
    ras_compute<SL, 2, NE>(A, src, acc);
    ras_load<SL, 4>(links, q, S, Vh, t, gnb, A, acc);
    ras_compute<SL, 3, NE>(B, src, acc);
    ras_load<SL, 5>(links, q, S, Vh, t, gnb, B, acc);
    ras_compute<SL, 4, NE>(A, src, acc);
    ras_load<SL, 6>(links, q, S, Vh, t, gnb, A, acc);
    ras_compute<SL, 5, NE>(B, src, acc);
    ras_load<SL, 7>(links, q, S, Vh, t, gnb, B, acc);
    ras_compute<SL, 6, NE>(A, src, acc);
    if constexpr (sizeof(CS) == 2) {
        ClovHalfRaw<CS> c0;
        {
            uint32_t gc = S.g, dummy = 0;
            ras_fence(acc, gc, dummy);
            load_clover_half_raw<CS>(clov, q, gc, Vh, 0, c0);
        }
        ras_compute<SL, 7, NE>(B, src, acc);
        float cl[36];
        expand_clover_half<CS, float>(c0, 0, cl);
        clover_mul_half(cl, acc, out);
    } else {
        ras_compute<SL, 7, NE>(B, src, acc);
        uint32_t gc = S.g, dummy = 0;
        ras_fence(acc, gc, dummy);
        float cl[36];
        load_clover_half<CS, float>(clov, q, gc, Vh, 0, cl);
        clover_mul_half(cl, acc, out);
    }
    {
        uint32_t gc = S.g, dummy = 0;
        ras_fence(acc, gc, dummy);
        float cl[36];
        load_clover_half<CS, float>(clov, q, gc, Vh, 1, cl);
        clover_mul_half(cl, acc + 6, out + 6);
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

// JAC: block Jacobi steps (alpha = 1, no reductions) instead of minimal
// residual; a template parameter so that the minimal-residual kernel keeps
// its registers.  SV: storage of the input and output vectors (float or
// __half); the block vectors in LDS and all arithmetic stay FP32.
// The workgroup memory of one block solve: component-major vectors with the
// compile-time stride MAXNE (immediate LDS offsets).
template <int MAXNE>
struct RasLds {
    float2 sE[12 * MAXNE];   // MR residual r on the even block sites
    float2 sO[12 * MAXNE];   // y = A_oo^-1 H_oe r on the odd block sites
    int gh[2 * MAXNE];       // global half index of every block site
    double red[4 * 16 + 4];
};

// One block solve (block index blk of the grid's block list, right-hand
// side rhs); every thread of the workgroup must call it (workgroup barriers).
template <typename SL, int MAXNE, bool JAC, typename SV>
WCL_D void ras_block(const RasArgs &a, int blk, int rhs, RasLds<MAXNE> &L)
{
    const unsigned tid = tid_here();
    const char *rin = (const char *)a.in + rhs * a.stride;
    char *rout = (char *)a.out + rhs * a.stride;
    float2 *sE = L.sE;
    float2 *sO = L.sO;
    int *gh = L.gh;
    double *red = L.red;

    const Geom &g = a.g;
    const int d = a.overlap;
    const int e0 = g.B[0] + 2 * d, e1 = g.B[1] + 2 * d, e2 = g.B[2] + 2 * d, e3 = g.B[3] + 2 * d;
    const int Ne = (e0 * e1 * e2 * e3) >> 1;
    const int e0h = e0 >> 1;
    int bc[4];
    if (a.colour > 0) {
        // a colour sweep of the multiplicative scheme: the grid holds only the
        // blocks of that colour (bit mu = parity of the block coordinate)
        int r = blk;
#pragma unroll
        for (int mu = 0; mu < 4; mu++) {
            const int bit = ((a.colour - 1) >> mu) & 1;
            const int cnt = (g.NB[mu] + 1 - bit) >> 1;
            bc[mu] = 2 * (r % cnt) + bit;
            r /= cnt;
        }
    } else {
        int r = blk;
        bc[0] = r % g.NB[0]; r /= g.NB[0];
        bc[1] = r % g.NB[1]; r /= g.NB[1];
        bc[2] = r % g.NB[2];
        bc[3] = r / g.NB[2];
    }

    for (int i = tid; i < 2 * Ne; i += blockDim.x) {
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
    const uint32_t t = tid;
    const bool active = (int)t < Ne;
    RasSite SE, SO;
    SE.sf = SE.sb = SO.sf = SO.sb = 1.f;
    bool core = false;
#pragma unroll
    for (int k = 0; k < 4; k++) { SE.nb[k] = 0xffffffffu; SO.nb[k] = 0xffffffffu; }
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
            RasSite &S = q == 0 ? SE : SO;
#pragma unroll
            for (int mu = 0; mu < 4; mu++) {
                const uint32_t f = (av[mu] + 1 < ev[mu]) ? (uint32_t)((lin + st) >> 1) : 0xffffu;
                const uint32_t bk = (av[mu] >= 1) ? (uint32_t)((lin - st) >> 1) : 0xffffu;
                S.nb[mu] = f | (bk << 16);
                st *= ev[mu];
            }
            int tile, loc, xt;
            ext_to_global(g, 3, bc[3], a3, d, tile, loc, xt);
            S.sf = (g.tbc < 0 && xt == g.L[3] - 1) ? -1.f : 1.f;
            S.sb = (g.tbc < 0 && xt == 0) ? -1.f : 1.f;
            if (q == 0) {
                core = true;
#pragma unroll
                for (int mu = 0; mu < 4; mu++)
                    if (av[mu] < d || av[mu] >= d + g.B[mu]) core = false;
            }
        }
    }
    __syncthreads();
    SE.g = active ? (uint32_t)gh[t] : 0u;
    SO.g = active ? (uint32_t)gh[MAXNE + t] : 0u;
    const uint32_t Vh = g.Vh;

    // r = the input on the even block sites (zero start: z = 0, r = rhs)
    if (active) {
        cplx<float> r[12];
        load_spinor<SV, float>(rin, SE.g, Vh, r);
#pragma unroll
        for (int c = 0; c < 12; c++) sE[c * MAXNE + t] = make_float2(r[c].re, r[c].im);
    }

    RasStage<SL> A, B;
    cplx<float> acc[12];
#pragma unroll
    for (int c = 0; c < 12; c++) acc[c] = {0.f, 0.f};
    for (int it = 0; it < a.iters; it++) {
        __syncthreads();
        // odd half: y = A_oo^-1 H_oe r on the odd block sites
        if (active) {
            cplx<float> y[12];
            ras_hop_start<SL>(a.links, 1, SO, Vh, t, gh, A, B, acc);
            ras_hop_finish<SL, MAXNE>(a.links, a.clov_inv, 1, SO, Vh, t, gh, sE, A, B, acc, y);
#pragma unroll
            for (int c = 0; c < 12; c++) sO[c * MAXNE + t] = make_float2(y[c].re, y[c].im);
        }
        __syncthreads();
        // even half: q = r - kappa^2 A_ee^-1 H_eo y
        cplx<float> qv[12];
        double dots[3] = {0.0, 0.0, 0.0};
        if (active) {
            cplx<float> w[12];
            ras_hop_start<SL>(a.links, 0, SE, Vh, t, gh + MAXNE, A, B, acc);
            ras_hop_finish<SL, MAXNE>(a.links, a.clov_inv, 0, SE, Vh, t, gh + MAXNE, sO, A, B, acc, w);
            float qr = 0.f, qi = 0.f, qq = 0.f;
#pragma unroll
            for (int c = 0; c < 12; c++) {
                const float2 r = sE[c * MAXNE + t];
                qv[c] = {fmaf(-a.kappa2, w[c].re, r.x), fmaf(-a.kappa2, w[c].im, r.y)};
                if constexpr (!JAC) {
                    qr = fmaf(qv[c].re, r.x, fmaf(qv[c].im, r.y, qr));
                    qi = fmaf(qv[c].re, r.y, fmaf(-qv[c].im, r.x, qi));
                    qq = fmaf(qv[c].re, qv[c].re, fmaf(qv[c].im, qv[c].im, qq));
                }
            }
            dots[0] = qr; dots[1] = qi; dots[2] = qq;
        } else {
#pragma unroll
            for (int c = 0; c < 12; c++) qv[c] = {0.f, 0.f};
        }
        float ar = 1.f, ai = 0.f;
        if constexpr (!JAC) {
            // minimal residual: alpha = <q, r> / <q, q> over the block
            block_allreduce<3>(dots, red);
            if (dots[2] == 0.0) {
                // the block's residual is zero: its solution stands; on the first
                // step nothing has been stored yet, and the solution is zero
                if (it == 0 && active && core && !a.accumulate) {
                    cplx<float> z0[12];
#pragma unroll
                    for (int c = 0; c < 12; c++) z0[c] = {0.f, 0.f};
                    store_spinor<SV, float>(rout, SE.g, Vh, z0);
                }
                break;
            }
            ar = (float)(dots[0] / dots[2]);
            ai = (float)(dots[1] / dots[2]);
        }
        if (active) {
            // z += alpha r (kept only where it is written: the core), r -= alpha q
            cplx<float> z[12];
            if (core) {
                if (it == 0 && !a.accumulate) {
#pragma unroll
                    for (int c = 0; c < 12; c++) z[c] = {0.f, 0.f};
                } else {
                    load_spinor<SV, float>(rout, SE.g, Vh, z);
                }
            }
#pragma unroll
            for (int c = 0; c < 12; c++) {
                const float2 r = sE[c * MAXNE + t];
                if (core) z[c] = {fmaf(ar, r.x, fmaf(-ai, r.y, z[c].re)), fmaf(ar, r.y, fmaf(ai, r.x, z[c].im))};
                sE[c * MAXNE + t] = make_float2(fmaf(-ar, qv[c].re, fmaf(ai, qv[c].im, r.x)),
                                                fmaf(-ar, qv[c].im, fmaf(-ai, qv[c].re, r.y)));
            }
            if (core) store_spinor<SV, float>(rout, SE.g, Vh, z);
        }
    }
}

}  // namespace wcl
