// hop_dev.h -- device code of the even/odd hopping kernel, shared by the
// per-launch kernel (k_hop) and the persistent inner solver.
#pragma once

#include "wcl_launch.h"

namespace wcl {

// ---------------------------------------------------------------------------
// The hopping kernel.  One thread per output site of parity p; per direction
// the neighbour spinor is projected to a half spinor (12 flop), rotated by
// the link or its adjoint (132 flop) and accumulated with the sign pattern of
// the projector (24 flop): 1320 flop per site over the 8 directions.
struct HopArgs {
    Geom g;
    const void *in;
    void *out;
    const void *links;
    const void *clov;
    const void *x;
    double coef;
    size_t in_stride, out_stride, x_stride;  // bytes between right-hand sides
    int p;
    int xcd;
    int nrhs;
    const Scalars *sc;   // per right-hand side
    int tpw;             // consecutive site blocks per workgroup (k_hop)
};

// The 8 hops of a site run as a two-stage pipeline: the neighbour spinor and
// link of hop k+1 are in flight while hop k is computed; a scheduling barrier
// after each hop keeps the compiler from hoisting further loads (which would
// raise the register count and lower the occupancy).
template <typename SL, typename R>
struct HopStage {
    cplx<R> psi[12];
    LinkRaw<SL> u;   // as loaded; decoded when the hop is computed
    R sign;
};

// hop K: direction MU = K/2, forward (K even) or backward (K odd)
// The load offsets of hop K pass through an empty asm that also "rewrites"
// the accumulator: the loads of hop K then wait for the complete compute of
// hop K-2, so at most two hops' operands are live at a time (no instruction
// is emitted for the fence itself).
template <typename R>
WCL_D void pipeline_fence(cplx<R> acc[12], uint32_t &hn, uint32_t &h)
{
    asm volatile(""
                 : "+v"(acc[0].re), "+v"(acc[0].im), "+v"(acc[1].re), "+v"(acc[1].im), "+v"(acc[2].re),
                   "+v"(acc[2].im), "+v"(acc[3].re), "+v"(acc[3].im), "+v"(acc[4].re), "+v"(acc[4].im),
                   "+v"(acc[5].re), "+v"(acc[5].im), "+v"(acc[6].re), "+v"(acc[6].im), "+v"(acc[7].re),
                   "+v"(acc[7].im), "+v"(acc[8].re), "+v"(acc[8].im), "+v"(acc[9].re), "+v"(acc[9].im),
                   "+v"(acc[10].re), "+v"(acc[10].im), "+v"(acc[11].re), "+v"(acc[11].im), "+v"(hn), "+v"(h));
}

// Staged input: a workgroup first copies the input spinors of its own NS
// consecutive half-sites (its tile, or a part or pair of tiles) into LDS; a
// neighbour inside that range is then read from LDS, one outside it from
// global memory.  In the blocked layout most neighbours of a tile lie in it.
typedef const __attribute__((address_space(3))) u32x4 *lds_u4p;
struct LdsIn {
    lds_u4p s;       // uint4 [words][NS]
    uint32_t base;   // first half index of the tile
};

// A spinor from the LDS copy of the tile (same word layout as the field).
template <typename S, int NS, typename R>
WCL_D void lds_spinor(lds_u4p s, uint32_t l, cplx<R> v[12])
{
    if constexpr (sizeof(S) == 8) {
#pragma unroll
        for (uint32_t i = 0; i < 12; i++) {
            const u32x4 u = s[i * NS + l];
            v[i] = {(R)__hiloint2double(u.y, u.x), (R)__hiloint2double(u.w, u.z)};
        }
    } else if constexpr (sizeof(S) == 4) {
#pragma unroll
        for (uint32_t k = 0; k < 6; k++) {
            const u32x4 u = s[k * NS + l];
            v[2 * k] = {(R)__uint_as_float(u.x), (R)__uint_as_float(u.y)};
            v[2 * k + 1] = {(R)__uint_as_float(u.z), (R)__uint_as_float(u.w)};
        }
    } else {
#pragma unroll
        for (uint32_t k = 0; k < 3; k++) {
            const u32x4 u = s[k * NS + l];
            float2 a = h2f2(u.x), b = h2f2(u.y), c = h2f2(u.z), d = h2f2(u.w);
            v[4 * k + 0] = {(R)a.x, (R)a.y};
            v[4 * k + 1] = {(R)b.x, (R)b.y};
            v[4 * k + 2] = {(R)c.x, (R)c.y};
            v[4 * k + 3] = {(R)d.x, (R)d.y};
        }
    }
}

template <typename SL, typename SS, int K, bool NT, int NS, typename R>
WCL_D void hop_load(const HopArgs &a, const Site &s, uint32_t h0, const char *in, const LdsIn &li,
                    HopStage<SL, R> &st, cplx<R> acc[12])
{
    constexpr int MU = K >> 1;
    constexpr bool FWD = (K & 1) == 0;
    const Geom &g = a.g;
    const uint32_t Vh = g.Vh;
    uint32_t hn = (uint32_t)neighbour(g, s, MU, FWD ? +1 : -1);
    uint32_t h = h0;
    pipeline_fence(acc, hn, h);
    if constexpr (NS > 0) {
        const uint32_t l = hn - li.base;
        if (l < (uint32_t)NS) lds_spinor<SS, NS, R>(li.s, l, st.psi);
        else load_spinor<SS, R>(in, hn, Vh, st.psi);
    } else {
        load_spinor<SS, R>(in, hn, Vh, st.psi);
    }
    if (FWD) load_link_raw<SL, NT>(a.links, MU, a.p, h, Vh, st.u);
    else load_link_raw<SL, NT>(a.links, MU, 1 - a.p, hn, Vh, st.u);
    st.sign = R(1);
    if (MU == 3 && g.tbc < 0 && s.x[3] == (FWD ? g.L[3] - 1 : 0)) st.sign = R(-1);
}

// forward: (1 - SG g_mu) U_mu(x) psi(x+mu);  backward: (1 + SG g_mu) U_mu(x-mu)^dag psi(x-mu)
template <int K, int SG, typename SL, typename R>
WCL_D void hop_compute(const HopStage<SL, R> &st, cplx<R> acc[12])
{
    constexpr int MU = K >> 1;
    constexpr bool FWD = (K & 1) == 0;
    constexpr int S = FWD ? -SG : SG;
    cplx<R> hh[6], uh[6], u[9];
    project<MU, S, R>(st.psi, hh);
#pragma unroll
    for (int k = 0; k < 6; k++) hh[k] = st.sign * hh[k];
    expand_link<SL, R>(st.u, u);
    if (FWD) su3_mul(u, hh, uh);
    else su3_dag_mul(u, hh, uh);
    accumulate<MU, S, R>(acc, uh);
}

template <typename SL, typename SS, int SG, int D, int K, bool NT, int NS, typename R>
WCL_D void hop_prologue(const HopArgs &a, const Site &s, uint32_t h, const char *in, const LdsIn &li,
                        HopStage<SL, R> st[D], cplx<R> acc[12])
{
    if constexpr (K < D - 1) {
        hop_load<SL, SS, K, NT, NS, R>(a, s, h, in, li, st[K], acc);
        hop_prologue<SL, SS, SG, D, K + 1, NT, NS, R>(a, s, h, in, li, st, acc);
    }
}

// hop K is computed while the operands of hop K + D - 1 are in flight
template <typename SL, typename SS, int SG, int D, int K, bool NT, int NS, typename R>
WCL_D void hop_pipeline(const HopArgs &a, const Site &s, uint32_t h, const char *in, const LdsIn &li,
                        HopStage<SL, R> st[D], cplx<R> acc[12])
{
    if constexpr (K < 8) {
        if constexpr (K + D - 1 < 8)
            hop_load<SL, SS, K + D - 1, NT, NS, R>(a, s, h, in, li, st[(K + D - 1) % D], acc);
        hop_compute<K, SG, SL, R>(st[K % D], acc);
        hop_pipeline<SL, SS, SG, D, K + 1, NT, NS, R>(a, s, h, in, li, st, acc);
    }
}

// The hop with MODE's epilogue on the half-sites [bid * blockDim.x, +
// blockDim.x) of one right-hand side.  Every thread of the workgroup must
// call it (the staged variant, NS == blockDim.x, fills `sin` and waits on a
// workgroup barrier).  NDOT > 0: the thread's output o at its site enters
// dot[0..1] += <w, o> (w a field of the output parity, same storage), and
// with NDOT == 2 dot[2] += |o|^2, accumulated in FP64 (zero for sites past
// the lattice).
template <typename SL, typename SS, int MODE, bool DAG, int DEPTH, bool NT, int NS, int NDOT = 0>
WCL_D void hop_block(const HopArgs &a, int bid, int rhs, uint4 *sin, const void *dotw = nullptr,
                     double *dot = nullptr)
{
    using R = typename Real<SL>::T;
    const unsigned tid = tid_here();
    const int h = bid * blockDim.x + tid;
    const char *in = (const char *)a.in + rhs * a.in_stride;
    constexpr int NWORDS = (int)sizeof(SS) * 24 / 16;   // 16-byte words per input spinor
    LdsIn li{(lds_u4p)sin, 0u};
    if constexpr (NS > 0) {
        // blockDim.x == NS: thread t stages half-site base + t
        li.base = (uint32_t)(bid * NS);
        if (h < a.g.Vh) {
#pragma unroll
            for (int k = 0; k < NWORDS; k++)
                sin[k * NS + tid] = ldf<uint4>(in, ((uint32_t)k * (uint32_t)a.g.Vh + (uint32_t)h) * 16u);
        }
        __syncthreads();
    }
    if (h >= a.g.Vh) return;
    const size_t Vh = a.g.Vh;
    char *out = (char *)a.out + rhs * a.out_stride;
    const Site s = decompose(a.g, h, a.p);
    constexpr int SG = DAG ? -1 : 1;
    cplx<R> acc[12];
#pragma unroll
    for (int i = 0; i < 12; i++) acc[i] = {R(0), R(0)};
    HopStage<SL, R> st[DEPTH];
    hop_prologue<SL, SS, SG, DEPTH, 0, NT, NS, R>(a, s, h, in, li, st, acc);
    hop_pipeline<SL, SS, SG, DEPTH, 0, NT, NS, R>(a, s, h, in, li, st, acc);

    cplx<R> o[12];
    if constexpr (MODE == HOP) {
#pragma unroll
        for (int i = 0; i < 12; i++) o[i] = acc[i];
    } else {
        R c[72];
        load_clover<typename ClovS<SL>::T, R, NT>(a.clov, a.p, h, Vh, c);
        if constexpr (MODE == CLOV_H) {
            clover_mul(c, acc, o);
        } else if constexpr (MODE == XPAY) {
            cplx<R> xv[12], t[12];
            load_spinor<SS, R>((const char *)a.x + rhs * a.x_stride, h, Vh, xv);
            clover_mul(c, acc, t);
            const R cf = (R)a.coef;
#pragma unroll
            for (int i = 0; i < 12; i++) o[i] = {fmar(cf, t[i].re, xv[i].re), fmar(cf, t[i].im, xv[i].im)};
        } else {
            cplx<R> xv[12];
            load_spinor<SS, R>((const char *)a.x + rhs * a.x_stride, h, Vh, xv);
            clover_mul(c, xv, o);
            const R cf = (R)a.coef;
#pragma unroll
            for (int i = 0; i < 12; i++) o[i] = {fmar(cf, acc[i].re, o[i].re), fmar(cf, acc[i].im, o[i].im)};
        }
    }
    store_spinor<SS, R>(out, h, Vh, o);
    if constexpr (NDOT > 0) {
        // the dot products see the stored values (FP16 storage rounds them)
        cplx<R> ov[12], wv[12];
        if constexpr (sizeof(SS) == 2) load_spinor<SS, R>(out, h, Vh, ov);
        else {
#pragma unroll
            for (int i = 0; i < 12; i++) ov[i] = o[i];
        }
        load_spinor<SS, R>((const char *)dotw + rhs * a.out_stride, h, Vh, wv);
#pragma unroll
        for (int i = 0; i < 12; i++) {
            const double wr = wv[i].re, wi = wv[i].im, xr = ov[i].re, xi = ov[i].im;
            dot[0] += wr * xr + wi * xi;
            dot[1] += wr * xi - wi * xr;
            if constexpr (NDOT == 2) dot[2] += xr * xr + xi * xi;
        }
    }
}

struct HopLaunch;
// The XPAY hop with fused reductions (HopLaunch::ndot), grid and block as for
// k_hop with one right-hand side per workgroup.
hipError_t launch_hop_dot(const HopLaunch &L, const HopArgs &a, dim3 grid, dim3 block, hipStream_t st);

}  // namespace wcl
