// hopdot.hip -- the second half of the Schur operator, out = x + coef A H in
// (the hop with its XPAY epilogue), with the BiCGStab inner products of its
// output fused into the epilogue: each workgroup writes its FP64 partial sums
// of <w, out> (one pair) or of <out, w> and <out, out> (two pairs) for the
// single-workgroup finaliser, so the solver reads the output vector once
// instead of in a separate reduction pass.
#include "hop_dev.h"

namespace wcl {

template <typename SL, typename SS, int NS, int NDOT>
__global__ void __launch_bounds__(256) k_hop_dot(HopArgs a, const void *dotw, double *partials, int pstride)
{
    const int lin = a.xcd ? xcd_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int rhs = lin % a.nrhs;
    const int bid = lin / a.nrhs;
    if (a.sc && a.sc[rhs].done) return;   // uniform in the workgroup
    constexpr int NWORDS = (int)sizeof(SS) * 24 / 16;
    __shared__ uint4 sin[NS > 0 ? NWORDS * NS : 1];
    __shared__ double red[3 * 16];
    double d[3] = {0.0, 0.0, 0.0};
    hop_block<SL, SS, XPAY, false, 2, false, NS, NDOT>(a, bid, rhs, sin, dotw, d);
    // workgroup sums in a fixed order
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < 3; k++) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) d[k] += __shfl_xor(d[k], o, 64);
        if (lane == 0) red[k * 16 + wid] = d[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double t[3] = {0.0, 0.0, 0.0};
        for (int w = 0; w < nw; w++)
#pragma unroll
            for (int k = 0; k < 3; k++) t[k] += red[k * 16 + w];
        double *pr = partials + (size_t)rhs * 6 * pstride + bid;
        if constexpr (NDOT == 1) {
            pr[0] = t[0];
            pr[pstride] = t[1];
        } else {
            // <out, w> = conj(<w, out>)
            pr[0] = t[0];
            pr[pstride] = -t[1];
            pr[2 * (size_t)pstride] = t[2];
            pr[3 * (size_t)pstride] = 0.0;
        }
    }
}

template <typename SL, typename SS, int NDOT>
static hipError_t hop_dot_ns(const HopLaunch &L, const HopArgs &a, dim3 grid, dim3 block, hipStream_t st)
{
    // staged input (one LDS slot per thread) for depth-2 shapes, as k_hop
    const bool staged = L.lds_stage && L.depth == 2;
    if (staged && block.x == 64) ext_launch(k_hop_dot<SL, SS, 64, NDOT>, grid, block, 0, st, L.ev, a, L.dotw, L.partials, L.pstride);
    else if (staged && block.x == 128) ext_launch(k_hop_dot<SL, SS, 128, NDOT>, grid, block, 0, st, L.ev, a, L.dotw, L.partials, L.pstride);
    else if (staged && block.x == 256) ext_launch(k_hop_dot<SL, SS, 256, NDOT>, grid, block, 0, st, L.ev, a, L.dotw, L.partials, L.pstride);
    else ext_launch(k_hop_dot<SL, SS, 0, NDOT>, grid, block, 0, st, L.ev, a, L.dotw, L.partials, L.pstride);
    return hipGetLastError();
}

template <typename SL, typename SS>
static hipError_t hop_dot_n(const HopLaunch &L, const HopArgs &a, dim3 grid, dim3 block, hipStream_t st)
{
    if (L.ndot == 1) return hop_dot_ns<SL, SS, 1>(L, a, grid, block, st);
    return hop_dot_ns<SL, SS, 2>(L, a, grid, block, st);
}

hipError_t launch_hop_dot(const HopLaunch &L, const HopArgs &a, dim3 grid, dim3 block, hipStream_t st)
{
    if (L.mode != XPAY || L.dagger || (L.ndot != 1 && L.ndot != 2) || !L.dotw || !L.partials) return hipErrorInvalidValue;
    if ((int)(grid.x / a.nrhs) > L.pstride) return hipErrorInvalidValue;
    if (L.link_prec == P64 && L.spin_prec == P64) return hop_dot_n<double, double>(L, a, grid, block, st);
    if (L.link_prec == P32 && L.spin_prec == P32) return hop_dot_n<float, float>(L, a, grid, block, st);
    if (L.link_prec == P16 && L.spin_prec == P32) return hop_dot_n<__half, float>(L, a, grid, block, st);
    if (L.link_prec == P16 && L.spin_prec == P16) return hop_dot_n<__half, __half>(L, a, grid, block, st);
    if (L.link_prec == P32C && L.spin_prec == P32) return hop_dot_n<R12f, float>(L, a, grid, block, st);
    if (L.link_prec == P16C && L.spin_prec == P32) return hop_dot_n<R12h, float>(L, a, grid, block, st);
    if (L.link_prec == P16C && L.spin_prec == P16) return hop_dot_n<R12h, __half>(L, a, grid, block, st);
    return hipErrorInvalidValue;
}

}  // namespace wcl
