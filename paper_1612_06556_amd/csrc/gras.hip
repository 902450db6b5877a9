// gras.hip -- Schwarz block solves with the block vectors in global memory.
//
// The fused RAS kernel keeps a block's two vectors in one workgroup's LDS,
// which caps the extended block at 648 sites per parity and the block solver
// at two vectors.  This path lifts both limits (any even core size, any
// overlap that fits the lattice, block BiCGStab besides minimal residual and
// Jacobi; Sec. 2 leaves the Schwarz recipe open): every extended block is
// copied into its own slice of a block field [block][12][nep] (FP32), the
// block operator -- the even/odd Schur complement restricted to the extended
// block with every hop that leaves it dropped, global clover inverse -- runs
// over all blocks at once, per-block dot products set per-block scalars on
// the device, and the solution's even core sites are written back (cores
// never overlap, so every even site is written once).
#include <vector>

#include "wcl_launch.h"

namespace wcl {

namespace {

constexpr uint32_t GM_MASK = 0x3fffffffu;   // global half index bits of a table entry
constexpr uint32_t GM_SF = 1u << 30;        // forward t hop crosses the antiperiodic boundary
constexpr uint32_t GM_SB = 1u << 31;        // backward t hop does
constexpr int GT = 256;                     // threads per workgroup

// Per-block solver state (FP64 scalars, complex as double2).
struct BState {
    double2 rho, rho_old, alpha, omega, beta;
    int done;   // 1: the block's solve has stopped (its iterate stands)
    int last;   // 1: stop after this iteration's update (t = 0 was met)
};

struct GArgs {
    uint32_t nblk, ne, nep, Vh;
    const uint32_t *gm;     // [2][nblk * nep]
    const uint32_t *nb;     // [2][nep][4]
    const uint8_t *core;    // [nep]
    const Scalars *sc;      // per right-hand side of the caller's solver (may be null)
    int rhs;
};

WCL_D bool skip(const GArgs &a) { return a.sc && a.sc[a.rhs].done; }

WCL_D void ldb(const float2 *f, const GArgs &a, uint32_t b, uint32_t i, cplx<float> v[12])
{
#pragma unroll
    for (int c = 0; c < 12; c++) {
        const float2 u = f[((size_t)b * 12 + c) * a.nep + i];
        v[c] = {u.x, u.y};
    }
}

WCL_D void stb(float2 *f, const GArgs &a, uint32_t b, uint32_t i, const cplx<float> v[12])
{
#pragma unroll
    for (int c = 0; c < 12; c++) f[((size_t)b * 12 + c) * a.nep + i] = make_float2(v[c].re, v[c].im);
}

WCL_D double2 cdiv(double2 a, double2 b)
{
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
WCL_D double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
WCL_D cplx<float> tof(double2 a) { return {(float)a.x, (float)a.y}; }

// Restriction of the input (SV storage, parity 0) to every extended block.
template <typename SV>
__global__ void __launch_bounds__(GT) k_gras_gather(GArgs a, const void *in, float2 *r, float2 *r2)
{
    if (skip(a)) return;
    const uint32_t id = blockIdx.x * GT + threadIdx.x;
    if (id >= a.nblk * a.nep) return;
    const uint32_t b = id / a.nep, i = id - b * a.nep;
    cplx<float> v[12];
    if (i < a.ne) load_spinor<SV, float>(in, a.gm[id] & GM_MASK, a.Vh, v);
    else
#pragma unroll
        for (int c = 0; c < 12; c++) v[c] = {0.f, 0.f};
    stb(r, a, b, i, v);
    if (r2) stb(r2, a, b, i, v);
}

// Zero block fields; reset the per-block state.
__global__ void __launch_bounds__(GT) k_gras_init(GArgs a, float2 *f0, float2 *f1, float2 *f2, BState *st)
{
    if (skip(a)) return;
    const uint32_t id = blockIdx.x * GT + threadIdx.x;
    if (id < a.nblk) {
        BState s;
        s.rho = s.rho_old = s.alpha = s.omega = s.beta = make_double2(1.0, 0.0);
        s.done = 0;
        s.last = 0;
        st[id] = s;
    }
    if (id >= a.nblk * a.nep) return;
    const uint32_t b = id / a.nep, i = id - b * a.nep;
    cplx<float> z[12];
#pragma unroll
    for (int c = 0; c < 12; c++) z[c] = {0.f, 0.f};
    stb(f0, a, b, i, z);
    if (f1) stb(f1, a, b, i, z);
    if (f2) stb(f2, a, b, i, z);
}

// One hop K (direction K/2, forward when K is even) of the block operator at
// local site i of parity Q in block b: the neighbour's spinor from the block
// field of the other parity, the link from the global field.
template <typename SL, int Q, int K>
WCL_D void ghop(const GArgs &a, const void *links, const float2 *src, uint32_t b, uint32_t i, uint32_t gq,
                cplx<float> acc[12])
{
    constexpr int MU = K >> 1;
    constexpr bool FWD = (K & 1) == 0;
    constexpr int S = FWD ? -1 : 1;
    const uint32_t ln = (a.nb[((size_t)Q * a.nep + i) * 4 + MU] >> (FWD ? 0 : 16)) & 0xffffu;
    if (ln == 0xffffu) return;   // the hop leaves the extended block: cut
    cplx<float> psi[12], hh[6], uh[6], u[9];
    ldb(src, a, b, ln, psi);
    if (FWD) {
        load_link<SL, float>(links, MU, Q, gq & GM_MASK, a.Vh, u);
    } else {
        const uint32_t gn = a.gm[(size_t)(1 - Q) * a.nblk * a.nep + (size_t)b * a.nep + ln] & GM_MASK;
        load_link<SL, float>(links, MU, 1 - Q, gn, a.Vh, u);
    }
    project<MU, S, float>(psi, hh);
    if (MU == 3 && (gq & (FWD ? GM_SF : GM_SB))) {
#pragma unroll
        for (int k = 0; k < 6; k++) hh[k] = -hh[k];
    }
    if (FWD) su3_mul(u, hh, uh);
    else su3_dag_mul(u, hh, uh);
    accumulate<MU, S, float>(acc, uh);
}

// Half of the block Schur operator.  Q = 1: dst_o = A_oo^-1 H_oe src_e.
// Q = 0: dst_e = x_e - kappa^2 A_ee^-1 H_eo src_o.
template <typename SL, int Q>
__global__ void __launch_bounds__(GT) k_gras_half(GArgs a, const void *links, const void *clov_inv, float kappa2,
                                                   const float2 *src, const float2 *x, float2 *dst)
{
    using CS = typename ClovS<SL>::T;
    if (skip(a)) return;
    const uint32_t id = blockIdx.x * GT + threadIdx.x;
    if (id >= a.nblk * a.nep) return;
    const uint32_t b = id / a.nep, i = id - b * a.nep;
    cplx<float> out[12];
    if (i >= a.ne) {
#pragma unroll
        for (int c = 0; c < 12; c++) out[c] = {0.f, 0.f};
        stb(dst, a, b, i, out);
        return;
    }
    const uint32_t gq = a.gm[(size_t)Q * a.nblk * a.nep + id];
    cplx<float> acc[12];
#pragma unroll
    for (int c = 0; c < 12; c++) acc[c] = {0.f, 0.f};
    ghop<SL, Q, 0>(a, links, src, b, i, gq, acc);
    ghop<SL, Q, 1>(a, links, src, b, i, gq, acc);
    ghop<SL, Q, 2>(a, links, src, b, i, gq, acc);
    ghop<SL, Q, 3>(a, links, src, b, i, gq, acc);
    ghop<SL, Q, 4>(a, links, src, b, i, gq, acc);
    ghop<SL, Q, 5>(a, links, src, b, i, gq, acc);
    ghop<SL, Q, 6>(a, links, src, b, i, gq, acc);
    ghop<SL, Q, 7>(a, links, src, b, i, gq, acc);
    float cl[36];
    load_clover_half<CS, float>(clov_inv, Q, gq & GM_MASK, a.Vh, 0, cl);
    clover_mul_half(cl, acc, out);
    load_clover_half<CS, float>(clov_inv, Q, gq & GM_MASK, a.Vh, 1, cl);
    clover_mul_half(cl, acc + 6, out + 6);
    if constexpr (Q == 0) {
        cplx<float> xv[12];
        ldb(x, a, b, i, xv);
#pragma unroll
        for (int c = 0; c < 12; c++)
            out[c] = {fmaf(-kappa2, out[c].re, xv[c].re), fmaf(-kappa2, out[c].im, xv[c].im)};
    }
    stb(dst, a, b, i, out);
}

// Block solver steps whose scalars come from per-block dot products.
enum GStep {
    G_MR = 0,       // alpha = <q, r> / <q, q> (stop when <q, q> = 0)
    G_RHO = 1,      // rho = <rh, r> (stop when 0); beta = (rho / rho_old)(alpha / omega)
    G_ALPHA = 2,    // alpha = rho / <rh, v> (stop when 0)
    G_OMEGA = 3,    // omega = <t, s> / <t, t> (0 when <t, t> = 0, the last step); rho_old = rho
};

// One workgroup per block: FP64 sums of conj(x) y over the block's sites for
// the pairs (x0, y0) and, for G_MR and G_OMEGA, (x0, x0); then thread 0 sets
// the block's scalars.
template <int STEP>
__global__ void __launch_bounds__(GT) k_gras_dots(GArgs a, const float2 *x0, const float2 *y0, BState *st)
{
    constexpr int NP = (STEP == G_MR || STEP == G_OMEGA) ? 2 : 1;
    __shared__ double red[2 * NP][GT / 64];
    if (skip(a)) return;
    const uint32_t b = blockIdx.x;
    double s[2 * NP];
#pragma unroll
    for (int k = 0; k < 2 * NP; k++) s[k] = 0.0;
    for (uint32_t i = threadIdx.x; i < a.ne; i += GT) {
        cplx<float> xv[12], yv[12];
        ldb(x0, a, b, i, xv);
        ldb(y0, a, b, i, yv);
#pragma unroll
        for (int c = 0; c < 12; c++) {
            s[0] += (double)xv[c].re * yv[c].re + (double)xv[c].im * yv[c].im;
            s[1] += (double)xv[c].re * yv[c].im - (double)xv[c].im * yv[c].re;
            if (NP == 2) s[2] += (double)xv[c].re * xv[c].re + (double)xv[c].im * xv[c].im;
        }
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 2 * NP; k++) {
        double v = s[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
        if (lane == 0) red[k][w] = v;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double t[2 * NP];
#pragma unroll
    for (int k = 0; k < 2 * NP; k++) {
        t[k] = 0.0;
        for (int j = 0; j < GT / 64; j++) t[k] += red[k][j];
    }
    BState S = st[b];
    if (S.done) return;
    const double2 d = make_double2(t[0], t[1]);
    if constexpr (STEP == G_MR) {
        if (t[2] == 0.0) S.done = 1;
        else S.alpha = make_double2(d.x / t[2], d.y / t[2]);
    } else if constexpr (STEP == G_RHO) {
        if (S.last || (d.x == 0.0 && d.y == 0.0)) {
            S.done = 1;
        } else {
            S.beta = cmul(cdiv(d, S.rho_old), cdiv(S.alpha, S.omega));
            S.rho = d;
        }
    } else if constexpr (STEP == G_ALPHA) {
        if (d.x == 0.0 && d.y == 0.0) S.done = 1;
        else S.alpha = cdiv(S.rho, d);
    } else {
        S.omega = t[2] == 0.0 ? make_double2(0.0, 0.0) : make_double2(d.x / t[2], d.y / t[2]);
        S.rho_old = S.rho;
        if (t[2] == 0.0) S.last = 1;
    }
    st[b] = S;
}

enum GUpd {
    U_MR = 0,    // z += alpha r ; r -= alpha q        (f0 = z, f1 = r, f2 = q)
    U_JAC = 1,   // z += r ; r -= q
    U_P = 2,     // p = r + beta (p - omega v)         (f0 = p, f1 = r, f2 = v)
    U_S = 3,     // s = r - alpha v                    (f0 = s, f1 = r, f2 = v)
    U_XR = 4,    // x += alpha p + omega s ; r = s - omega t   (f0 = x, f1 = r, f2 = p, f3 = s, f4 = t)
};

template <int U>
__global__ void __launch_bounds__(GT) k_gras_update(GArgs a, const BState *st, float2 *f0, float2 *f1,
                                                     const float2 *f2, const float2 *f3, const float2 *f4)
{
    if (skip(a)) return;
    const uint32_t id = blockIdx.x * GT + threadIdx.x;
    if (id >= a.nblk * a.nep) return;
    const uint32_t b = id / a.nep, i = id - b * a.nep;
    if (st[b].done) return;
    cplx<float> v0[12], v1[12], v2[12];
    ldb(f0, a, b, i, v0);
    ldb(f1, a, b, i, v1);
    ldb(f2, a, b, i, v2);
    if constexpr (U == U_MR || U == U_JAC) {
        const cplx<float> al = U == U_MR ? tof(st[b].alpha) : cplx<float>{1.f, 0.f};
#pragma unroll
        for (int c = 0; c < 12; c++) {
            v0[c] = cfma(al, v1[c], v0[c]);
            v1[c] = v1[c] - al * v2[c];
        }
        stb(f0, a, b, i, v0);
        stb(f1, a, b, i, v1);
    } else if constexpr (U == U_P) {
        const cplx<float> be = tof(st[b].beta), om = tof(st[b].omega);
#pragma unroll
        for (int c = 0; c < 12; c++) v0[c] = cfma(be, v0[c] - om * v2[c], v1[c]);
        stb(f0, a, b, i, v0);
    } else if constexpr (U == U_S) {
        const cplx<float> al = tof(st[b].alpha);
#pragma unroll
        for (int c = 0; c < 12; c++) v0[c] = v1[c] - al * v2[c];
        stb(f0, a, b, i, v0);
    } else {
        const cplx<float> al = tof(st[b].alpha), om = tof(st[b].omega);
        cplx<float> sv[12], tv[12];
        ldb(f3, a, b, i, sv);
        ldb(f4, a, b, i, tv);
#pragma unroll
        for (int c = 0; c < 12; c++) {
            v0[c] = cfma(om, sv[c], cfma(al, v2[c], v0[c]));
            v1[c] = sv[c] - om * tv[c];
        }
        stb(f0, a, b, i, v0);
        stb(f1, a, b, i, v1);
    }
}

// The even core sites of every block's solution into the output (SV storage).
template <typename SV>
__global__ void __launch_bounds__(GT) k_gras_scatter(GArgs a, const float2 *z, void *out)
{
    if (skip(a)) return;
    const uint32_t id = blockIdx.x * GT + threadIdx.x;
    if (id >= a.nblk * a.nep) return;
    const uint32_t b = id / a.nep, i = id - b * a.nep;
    if (i >= a.ne || !a.core[i]) return;
    cplx<float> v[12];
    ldb(z, a, b, i, v);
    store_spinor<SV, float>(out, a.gm[id] & GM_MASK, a.Vh, v);
}

// Half index of global coordinates x in the blocked even/odd layout.
uint32_t blocked_half(const Geom &g, const int x[4])
{
    int blk = 0, lin = 0;
    for (int mu = 0; mu < 4; mu++) {
        blk += (x[mu] / g.B[mu]) * g.sb[mu];
        lin += (x[mu] % g.B[mu]) * g.sl[mu];
    }
    return (uint32_t)blk * (uint32_t)g.Hb + (uint32_t)(lin >> 1);
}

template <typename SL>
void launch_halves(const GArgs &a, const RasLaunch &L, const float2 *in, float2 *y, float2 *out, unsigned grid,
                   hipStream_t st)
{
    k_gras_half<SL, 1><<<grid, GT, 0, st>>>(a, L.links, L.clov_inv, L.kappa2, in, nullptr, y);
    k_gras_half<SL, 0><<<grid, GT, 0, st>>>(a, L.links, L.clov_inv, L.kappa2, y, in, out);
}

// out = Dhat_B in on every block (two halves).
hipError_t block_op(const GArgs &a, const RasLaunch &L, const float2 *in, float2 *y, float2 *out, unsigned grid,
                    hipStream_t st)
{
    switch (L.link_prec) {
        case P32: launch_halves<float>(a, L, in, y, out, grid, st); break;
        case P16: launch_halves<__half>(a, L, in, y, out, grid, st); break;
        case P32C: launch_halves<R12f>(a, L, in, y, out, grid, st); break;
        case P16C: launch_halves<R12h>(a, L, in, y, out, grid, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

int gras_fields(int solver) { return solver == 2 ? 8 : 4; }

bool gras_fits_fused(const Geom &g, int overlap)
{
    int n = 1;
    for (int mu = 0; mu < 4; mu++) n *= g.B[mu] + 2 * overlap;
    return n / 2 <= 648;
}

hipError_t gras_tables(const Geom &g, const int cores[4], int overlap, GrasPlan *P,
                       std::vector<uint32_t> &host)
{
    int e[4], nbk[4];
    P->nblk = 1;
    int ext = 1;
    for (int mu = 0; mu < 4; mu++) {
        if (cores[mu] < 2 || (cores[mu] & 1) || g.L[mu] % cores[mu] || g.L[mu] < cores[mu] + 2 * overlap)
            return hipErrorInvalidValue;
        e[mu] = cores[mu] + 2 * overlap;
        nbk[mu] = g.L[mu] / cores[mu];
        P->nblk *= nbk[mu];
        ext *= e[mu];
        P->cores[mu] = cores[mu];
    }
    P->overlap = overlap;
    P->ne = ext / 2;
    P->nep = (P->ne + 63) / 64 * 64;
    if (P->nep >= 0xffff) return hipErrorInvalidValue;
    const size_t nb = (size_t)P->nblk, nep = (size_t)P->nep;
    // host image: gm [2][nblk][nep] | nb [2][nep][4] | core [nep] bytes (padded to words)
    const size_t ngm = 2 * nb * nep, nnb = 2 * nep * 4, ncore = (nep + 3) / 4;
    host.assign(ngm + nnb + ncore, 0u);
    uint32_t *gm = host.data(), *nbt = gm + ngm;
    uint8_t *core = reinterpret_cast<uint8_t *>(nbt + nnb);
    const int e0h = e[0] / 2;
    for (int q = 0; q < 2; q++) {
        for (int i = 0; i < P->nep; i++)
            for (int mu = 0; mu < 4; mu++) nbt[((size_t)q * nep + i) * 4 + mu] = 0xffffffffu;
        for (int li = 0; li < P->ne; li++) {
            int r = li;
            const int a0h = r % e0h; r /= e0h;
            const int a1 = r % e[1]; r /= e[1];
            const int a2 = r % e[2];
            const int a3 = r / e[2];
            const int a[4] = {2 * a0h + ((q + a1 + a2 + a3) & 1), a1, a2, a3};
            const int lin = a[0] + e[0] * (a[1] + e[1] * (a[2] + e[2] * a[3]));
            int stride = 1;
            for (int mu = 0; mu < 4; mu++) {
                const uint32_t f = a[mu] + 1 < e[mu] ? (uint32_t)((lin + stride) >> 1) : 0xffffu;
                const uint32_t bk = a[mu] >= 1 ? (uint32_t)((lin - stride) >> 1) : 0xffffu;
                nbt[((size_t)q * nep + li) * 4 + mu] = f | (bk << 16);
                stride *= e[mu];
            }
            if (q == 0) {
                bool c = true;
                for (int mu = 0; mu < 4; mu++)
                    if (a[mu] < overlap || a[mu] >= overlap + cores[mu]) c = false;
                core[li] = c ? 1 : 0;
            }
            for (int b = 0; b < P->nblk; b++) {
                int rb = b, x[4];
                for (int mu = 0; mu < 4; mu++) {
                    const int bc = rb % nbk[mu];
                    rb /= nbk[mu];
                    x[mu] = ((bc * cores[mu] - overlap + a[mu]) % g.L[mu] + g.L[mu]) % g.L[mu];
                }
                uint32_t v = blocked_half(g, x);
                if (g.tbc < 0 && x[3] == g.L[3] - 1) v |= GM_SF;
                if (g.tbc < 0 && x[3] == 0) v |= GM_SB;
                gm[(size_t)q * nb * nep + (size_t)b * nep + li] = v;
            }
        }
    }
    return hipSuccess;
}

void gras_bind(GrasPlan *P, void *tables, void *vectors, void *state)
{
    const size_t nb = (size_t)P->nblk, nep = (size_t)P->nep;
    P->gm = (const uint32_t *)tables;
    P->nb = P->gm + 2 * nb * nep;
    P->core = (const uint8_t *)(P->nb + 2 * nep * 4);
    for (int k = 0; k < 8; k++) P->vec[k] = nullptr;
    for (int k = 0; k < P->nvec; k++) P->vec[k] = (float2 *)vectors + (size_t)k * nb * 12 * nep;
    P->state = state;
}

size_t gras_vector_bytes(const GrasPlan &P) { return (size_t)P.nvec * P.nblk * 12 * (size_t)P.nep * sizeof(float2); }
size_t gras_state_bytes(const GrasPlan &P) { return (size_t)P.nblk * sizeof(BState); }

hipError_t launch_gras(const GrasPlan &P, const RasLaunch &L, int solver, hipStream_t st)
{
    if (L.colour != 0 || L.accumulate) return hipErrorInvalidValue;
    if (solver < 0 || solver > 2 || P.nvec < gras_fields(solver) || L.iters < 1) return hipErrorInvalidValue;
    const int vp = L.vec_prec ? L.vec_prec : P32;
    if (vp != P32 && vp != P16) return hipErrorInvalidValue;
    if (vp == P16 && L.link_prec != P16 && L.link_prec != P16C) return hipErrorInvalidValue;
    const size_t vb = spinor_bytes(prec_bytes(vp), (size_t)L.g->Vh);
    if (L.nrhs > 1 && L.stride < vb) return hipErrorInvalidValue;
    GArgs a;
    a.nblk = (uint32_t)P.nblk;
    a.ne = (uint32_t)P.ne;
    a.nep = (uint32_t)P.nep;
    a.Vh = (uint32_t)L.g->Vh;
    a.gm = P.gm;
    a.nb = P.nb;
    a.core = P.core;
    a.sc = L.sc;
    const unsigned grid = (unsigned)(((size_t)P.nblk * P.nep + GT - 1) / GT);
    const unsigned sgrid = (unsigned)((P.nblk + GT - 1) / GT);
    BState *S = (BState *)P.state;
    float2 *const *f = P.vec;
    for (int rhs = 0; rhs < (L.nrhs > 0 ? L.nrhs : 1); rhs++) {
        a.rhs = rhs;
        const char *in = (const char *)L.in + rhs * L.stride;
        char *out = (char *)L.out + rhs * L.stride;
        if (solver == 2) {
            // f: 0 r, 1 rh, 2 p, 3 v, 4 s, 5 t, 6 x, 7 y (odd)
            if (vp == P16) k_gras_gather<__half><<<grid, GT, 0, st>>>(a, in, f[0], f[1]);
            else k_gras_gather<float><<<grid, GT, 0, st>>>(a, in, f[0], f[1]);
            k_gras_init<<<grid > sgrid ? grid : sgrid, GT, 0, st>>>(a, f[2], f[3], f[6], S);
            for (int it = 0; it < L.iters; it++) {
                k_gras_dots<G_RHO><<<P.nblk, GT, 0, st>>>(a, f[1], f[0], S);
                k_gras_update<U_P><<<grid, GT, 0, st>>>(a, S, f[2], f[0], f[3], nullptr, nullptr);
                hipError_t e = block_op(a, L, f[2], f[7], f[3], grid, st);
                if (e != hipSuccess) return e;
                k_gras_dots<G_ALPHA><<<P.nblk, GT, 0, st>>>(a, f[1], f[3], S);
                k_gras_update<U_S><<<grid, GT, 0, st>>>(a, S, f[4], f[0], f[3], nullptr, nullptr);
                e = block_op(a, L, f[4], f[7], f[5], grid, st);
                if (e != hipSuccess) return e;
                k_gras_dots<G_OMEGA><<<P.nblk, GT, 0, st>>>(a, f[5], f[4], S);
                k_gras_update<U_XR><<<grid, GT, 0, st>>>(a, S, f[6], f[0], f[2], f[4], f[5]);
            }
            if (vp == P16) k_gras_scatter<__half><<<grid, GT, 0, st>>>(a, f[6], out);
            else k_gras_scatter<float><<<grid, GT, 0, st>>>(a, f[6], out);
        } else {
            // f: 0 r, 1 z, 2 q, 3 y (odd)
            if (vp == P16) k_gras_gather<__half><<<grid, GT, 0, st>>>(a, in, f[0], nullptr);
            else k_gras_gather<float><<<grid, GT, 0, st>>>(a, in, f[0], nullptr);
            k_gras_init<<<grid > sgrid ? grid : sgrid, GT, 0, st>>>(a, f[1], nullptr, nullptr, S);
            for (int it = 0; it < L.iters; it++) {
                hipError_t e = block_op(a, L, f[0], f[3], f[2], grid, st);
                if (e != hipSuccess) return e;
                if (solver == 0) {
                    k_gras_dots<G_MR><<<P.nblk, GT, 0, st>>>(a, f[2], f[0], S);
                    k_gras_update<U_MR><<<grid, GT, 0, st>>>(a, S, f[1], f[0], f[2], nullptr, nullptr);
                } else {
                    k_gras_update<U_JAC><<<grid, GT, 0, st>>>(a, S, f[1], f[0], f[2], nullptr, nullptr);
                }
            }
            if (vp == P16) k_gras_scatter<__half><<<grid, GT, 0, st>>>(a, f[1], out);
            else k_gras_scatter<float><<<grid, GT, 0, st>>>(a, f[1], out);
        }
    }
    return hipGetLastError();
}

void gras_work(const GrasPlan &P, const RasLaunch &L, int solver, double *bytes, double *flops)
{
    const Geom &g = *L.g;
    const double lb = L.link_prec == P32 ? 72.0 : L.link_prec == P16 ? 36.0 : L.link_prec == P32C ? 48.0 : 24.0;
    const double cb = (L.link_prec == P32 || L.link_prec == P32C) ? 288.0 : 144.0;
    const double nr = L.nrhs > 0 ? L.nrhs : 1;
    const double vb = L.vec_prec == P16 ? 48.0 : 96.0;
    *bytes = (double)g.Vh * (8.0 * lb + 2.0 * cb + nr * 2.0 * vb);
    double ext = 1.0;
    int e[4];
    for (int mu = 0; mu < 4; mu++) {
        e[mu] = P.cores[mu] + 2 * P.overlap;
        ext *= e[mu];
    }
    double hops = 0.0;
    for (int mu = 0; mu < 4; mu++) hops += 2.0 * (e[mu] - 1) * ext / e[mu];
    const double ne = ext / 2.0;
    const double apply = hops * 168.0 + ext * 504.0 + ne * 48.0;
    // vector work per even site and iteration: MR 2 dots + 2 updates (288),
    // Jacobi 2 updates (96), BiCGStab 4 dots + p, s, x, r updates (960)
    const double per_iter = solver == 2 ? 2.0 * apply + ne * 960.0 : apply + ne * (solver == 0 ? 288.0 : 96.0);
    *flops = per_iter * L.iters * P.nblk * nr;
}

}  // namespace wcl
