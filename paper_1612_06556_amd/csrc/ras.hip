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
#include "ras_dev.h"

namespace wcl {

// JAC: block Jacobi steps (alpha = 1, no reductions) instead of minimal
// residual; a template parameter so that the minimal-residual kernel keeps
// its registers.  SV: storage of the input and output vectors (float or
// __half); the block vectors in LDS and all arithmetic stay FP32.
template <typename SL, int MAXNE, bool JAC, typename SV>
__global__ void __launch_bounds__(MAXNE == 648 ? 704 : 128) k_ras(RasArgs a)
{
    // workgroup id = tile * nrhs + rhs (the right-hand sides of one tile share
    // its links and clover through L2)
    const int lin = xcd_block(blockIdx.x, gridDim.x);
    const int rhs = lin % a.nrhs;
    const int blk = lin / a.nrhs;
    if (a.sc && a.sc[rhs].done) return;
    __shared__ RasLds<MAXNE> lds;
    ras_block<SL, MAXNE, JAC, SV>(a, blk, rhs, lds);
}

int ras_threads(const Geom &g, int overlap)
{
    int n = 1;
    for (int mu = 0; mu < 4; mu++) n *= g.B[mu] + 2 * overlap;
    n >>= 1;
    return ((n + 63) / 64) * 64;
}

// FP16 vectors go with the FP16 links and clover only.
template <int MAXNE, bool JAC>
hipError_t ras_dispatch(const RasLaunch &L, const RasArgs &a, dim3 grid, dim3 block, hipStream_t st)
{
    if (L.vec_prec == P16) {
        switch (L.link_prec) {
            case P16: ext_launch(k_ras<__half, MAXNE, JAC, __half>, grid, block, 0, st, L.ev, a); break;
            case P16C: ext_launch(k_ras<R12h, MAXNE, JAC, __half>, grid, block, 0, st, L.ev, a); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (L.link_prec) {
        case P32: ext_launch(k_ras<float, MAXNE, JAC, float>, grid, block, 0, st, L.ev, a); break;
        case P16: ext_launch(k_ras<__half, MAXNE, JAC, float>, grid, block, 0, st, L.ev, a); break;
        case P32C: ext_launch(k_ras<R12f, MAXNE, JAC, float>, grid, block, 0, st, L.ev, a); break;
        case P16C: ext_launch(k_ras<R12h, MAXNE, JAC, float>, grid, block, 0, st, L.ev, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_ras(const RasLaunch &L, hipStream_t st)
{
    const Geom &g = *L.g;
    // several right-hand sides need a stride of at least one even field
    if (L.nrhs < 1 || L.nrhs > 4096) return hipErrorInvalidValue;
    const int vp = L.vec_prec ? L.vec_prec : P32;
    if (vp != P32 && vp != P16) return hipErrorInvalidValue;
    if (L.nrhs > 1 && L.stride < spinor_bytes(prec_bytes(vp), (size_t)g.Vh)) return hipErrorInvalidValue;
    for (int mu = 0; mu < 4; mu++)
        if (L.overlap > g.B[mu] || g.L[mu] < g.B[mu] + 2 * L.overlap) return hipErrorInvalidValue;
    int ne = 1;
    for (int mu = 0; mu < 4; mu++) ne *= g.B[mu] + 2 * L.overlap;
    ne >>= 1;
    RasArgs a;
    a.g = g;
    a.overlap = L.overlap;
    a.iters = L.iters;
    a.in = L.in;
    a.out = L.out;
    // the two-row FP32 links are read from their per-site copy
    if (L.link_prec == P32C && !L.links_site) return hipErrorInvalidValue;
    a.links = L.link_prec == P32C ? L.links_site : L.links;
    a.clov_inv = L.clov_inv;
    a.kappa2 = L.kappa2;
    a.sc = L.sc;
    a.nrhs = L.nrhs;
    a.stride = L.stride;
    if (L.colour < 0 || L.colour > 16) return hipErrorInvalidValue;
    a.colour = L.colour;
    a.accumulate = L.accumulate ? 1 : 0;
    int nblk = 1;
    for (int mu = 0; mu < 4; mu++) {
        const int bit = L.colour > 0 ? ((L.colour - 1) >> mu) & 1 : 0;
        nblk *= L.colour > 0 ? (g.NB[mu] + 1 - bit) / 2 : g.NB[mu];
    }
    if (nblk == 0) return hipSuccess;   // no block of that colour
    const int threads = ras_threads(g, L.overlap);
    if (threads > 1024) return hipErrorInvalidValue;
    dim3 grid(nblk * a.nrhs), block(threads);
    if (ne <= 128) {
        if (L.jacobi) return ras_dispatch<128, true>(L, a, grid, block, st);
        return ras_dispatch<128, false>(L, a, grid, block, st);
    }
    if (ne <= 648) {
        if (L.jacobi) return ras_dispatch<648, true>(L, a, grid, block, st);
        return ras_dispatch<648, false>(L, a, grid, block, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace wcl

namespace wcl {

void ras_work(const RasLaunch &L, double *bytes, double *flops)
{
    const Geom &g = *L.g;
    const double lb = L.link_prec == P32 ? 72.0 : L.link_prec == P16 ? 36.0 : L.link_prec == P32C ? 48.0 : 24.0;
    const double cb = (L.link_prec == P32 || L.link_prec == P32C) ? 288.0 : 144.0;
    const double nr = L.nrhs > 0 ? L.nrhs : 1;
    const double vb = L.vec_prec == P16 ? 48.0 : 96.0;
    *bytes = (double)g.Vh * (8.0 * lb + 2.0 * cb + nr * 2.0 * vb);
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
    // two dot products (96, minimal residual only) and the z, r updates (96)
    const double per_iter = hops * 168.0 + ext * 504.0 + ne * (48.0 + (L.jacobi ? 0.0 : 96.0) + 96.0);
    double nblk = 1.0;
    for (int mu = 0; mu < 4; mu++) {
        if (L.colour > 0) nblk *= ((L.colour - 1) >> mu & 1) ? g.NB[mu] / 2 : (g.NB[mu] + 1) / 2;
        else nblk *= g.NB[mu];
    }
    const double frac = nblk / ((double)g.NB[0] * g.NB[1] * g.NB[2] * g.NB[3]);
    *bytes *= frac;
    *flops = per_iter * L.iters * nblk * nr;
}

}  // namespace wcl
