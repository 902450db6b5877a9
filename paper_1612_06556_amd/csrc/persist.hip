// persist.hip -- the inner single-precision BiCGStab of the paper's solver
// (Sec. 2: the FP32 BiCGStab on the even/odd preconditioned matrix, right
// preconditioned by overlapped RAS, that preconditions the FP64 flexible
// BiCGStab) as one persistent cooperative kernel per inner solve.
//
// Every workgroup of the launch is resident (cooperative launch, one
// workgroup per CU), so phases that depend on each other's results across
// the lattice are separated by a grid-wide barrier instead of a kernel
// boundary, and the inner solve runs all its iterations without returning to
// the host.  One iteration, for every right-hand side not yet converged:
//
//   p  = r + beta (p - omega v)                   elementwise
//   ph = M p                                      RAS block solves (or ph = p)
//   o  = T_oo^-1 H_oe ph                          hop, clover epilogue
//   v  = ph - k^2 T_ee^-1 H_eo o,  <rt, v>        hop, XPAY epilogue + fused dot
//   alpha = rho / <rt, v>;  s = r - alpha v       elementwise
//   sh = M s                                      (or sh = s)
//   o  = T_oo^-1 H_oe sh
//   t  = sh - k^2 T_ee^-1 H_eo o,  <t, s>, <t, t>
//   omega = <t, s> / <t, t>
//   x += alpha ph + omega sh;  r = s - omega t;  <rt, r>, <r, r>
//   rho_old = rho, rho = <rt, r>; stop when |r|^2 <= stop^2 |r_0|^2
//
// Reductions: each workgroup writes its FP64 partial sums per right-hand
// side; after the barrier every workgroup adds all partials in the same fixed
// order, so every workgroup holds bitwise the same scalars and takes the
// same decisions (no second barrier, no atomics on floating-point values).
// The scalar rules (breakdown, NaN, stopping) are those of the per-launch
// solver's finaliser.  Workgroup w works on the chunks (of sites, blocks or
// vector elements) of XCD w mod 8, in one contiguous range per XCD.
#include "hop_dev.h"
#include "ras_dev.h"

namespace wcl {

constexpr int PMAXR = PMAX_RHS;   // right-hand sides per persistent launch

struct PersistArgs {
    // every phase's arguments, prepared on the host (read from the kernel
    // argument segment, never copied into registers): [half] 0 = v = Dhat M p,
    // 1 = t = Dhat M s
    HopArgs hc[2];        // o = T_oo^-1 H_oe (M p | M s)
    HopArgs hx[2];        // (v | t) = (M p | M s) - k^2 T_ee^-1 H_eo o
    RasArgs ra[2];        // (ph | sh) = M (p | s)
    int use_ras;
    void *x, *r, *rt, *p, *v, *s, *t, *ph, *sh, *o;   // [nrhs] fields, `stride` bytes apart
    size_t stride;
    Scalars *sc;          // per right-hand side (initialised by the caller)
    double *partials;     // [gridDim][PMAXR][4]
    unsigned *bar;        // [0] arrivals, [1] generation
    int *err;             // set when a barrier wait exceeds its bound
    int nrhs, maxit;
    int nblk;             // Schwarz blocks (tiles)
};

struct PScal {
    double rho[2], rho_old[2], alpha[2], omega[2];
    double r2, b2, stop2;
    int done, iter;
};

// Grid-wide barrier.  Agent-scope release before arriving and acquire after
// leaving publish every workgroup's writes of the phase to every XCD (their
// L2 caches are not coherent with each other otherwise).  A wait beyond
// 2^22 polls sets *err and returns false: the caller leaves the kernel, so
// a launch always ends.
WCL_D bool grid_sync(unsigned *bar, int *err, unsigned nwg)
{
    __shared__ int ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned g0 = __hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __atomic_thread_fence(__ATOMIC_RELEASE);
        const unsigned prev = __hip_atomic_fetch_add(bar, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        int good = 1;
        if (prev == nwg - 1) {
            __hip_atomic_store(bar, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(bar + 1, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned n = 0;
            while (__hip_atomic_load(bar + 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g0) {
                __builtin_amdgcn_s_sleep(2);
                if (++n > (1u << 22)) {
                    __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    good = 0;
                    break;
                }
            }
        }
        __atomic_thread_fence(__ATOMIC_ACQUIRE);
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) good = 0;
        ok = good;
    }
    __syncthreads();
    return ok != 0;
}

// Item range of workgroup w for n items: the items of XCD w mod 8 form one
// contiguous range; its workgroups take every (G/8)-th item of it.
struct ItemRange {
    int first, last, step;
};
WCL_D ItemRange xcd_items(int n)
{
    const int G = gridDim.x, w = blockIdx.x;
    if (G < 8 || (G & 7)) return {w, n, G};
    const int per = (n + 7) / 8, x = w & 7, j = w >> 3;
    const int lo = x * per, hi = min(n, lo + per);
    return {lo + j, hi, G >> 3};
}

// Sum of NV doubles over the workgroup (fixed order); the result in every thread.
template <int NV>
WCL_D void wg_sum(double v[NV], double *red /* [NV * 16 + NV] */)
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
    __syncthreads();
}

// Partials of this workgroup for one right-hand side.
WCL_D void put_partials(const PersistArgs &a, int rhs, double d[3], double *red)
{
    double v[3] = {d[0], d[1], d[2]};
    wg_sum<3>(v, red);
    if (threadIdx.x == 0) {
        double *pp = a.partials + ((size_t)blockIdx.x * PMAXR + rhs) * 4;
        pp[0] = v[0];
        pp[1] = v[1];
        pp[2] = v[2];
    }
}

// The sums of all workgroups' partials for one right-hand side (same order
// in every workgroup).
WCL_D void get_sums(const PersistArgs &a, int rhs, double v[3], double *red)
{
    v[0] = v[1] = v[2] = 0.0;
    for (int w = threadIdx.x; w < (int)gridDim.x; w += blockDim.x) {
        const double *pp = a.partials + ((size_t)w * PMAXR + rhs) * 4;
        v[0] += pp[0];
        v[1] += pp[1];
        v[2] += pp[2];
    }
    wg_sum<3>(v, red);
}

WCL_D void pcdiv(const double a[2], const double b[2], double o[2])
{
    const double d = b[0] * b[0] + b[1] * b[1];
    o[0] = (a[0] * b[0] + a[1] * b[1]) / d;
    o[1] = (a[1] * b[0] - a[0] * b[1]) / d;
}

template <typename SV>
struct PVec {
    using V = typename std::conditional<std::is_same<SV, __half>::value, __half2, float2>::type;
};
WCL_D float2 pld(const float2 &v) { return v; }
WCL_D float2 pld(const __half2 &v) { return __half22float2(v); }
WCL_D void pst(float2 &d, float x, float y) { d = make_float2(x, y); }
WCL_D void pst(__half2 &d, float x, float y)
{
    fp32_as_computed(x, y);
    d = __floats2half2_rn(x, y);
}

template <typename SV>
WCL_D typename PVec<SV>::V *vec(void *base, int rhs, size_t stride)
{
    return (typename PVec<SV>::V *)((char *)base + rhs * stride);
}

// The hop phase over this workgroup's site chunks of one right-hand side.
template <typename SL, typename SV, int MODE, int NS, int NDOT>
WCL_D void hop_phase(const HopArgs &h, int rhs, uint4 *sin, const void *dotw, double *dot)
{
    const int nchunk = (h.g.Vh + NS - 1) / NS;
    const ItemRange R = xcd_items(nchunk);
    for (int c = R.first; c < R.last; c += R.step) {
        __syncthreads();   // the previous chunk's staged input is no longer read
        hop_block<SL, SV, MODE, false, 2, false, NS, NDOT>(h, c, rhs, sin, dotw, dot);
    }
}

template <typename SL, typename SV, bool RAS, int NT>
__global__ void __launch_bounds__(NT) k_inner_persist(PersistArgs a)
{
    // workgroup memory: the Schwarz block vectors or the staged hop input
    // (never live at the same time), the scalars and the reduction scratch
    constexpr int NWORDS = (int)sizeof(SV) * 24 / 16;
    constexpr size_t HOP_LDS = (size_t)NWORDS * NT * 16;
    constexpr size_t RAS_LDS = RAS ? sizeof(RasLds<648>) : 0;
    constexpr size_t UNION = HOP_LDS > RAS_LDS ? HOP_LDS : RAS_LDS;
    __shared__ __align__(16) unsigned char smem[UNION];
    __shared__ PScal ps[PMAXR];
    __shared__ double red[4 * 16 + 4];
    uint4 *sin = reinterpret_cast<uint4 *>(smem);
    using V = typename PVec<SV>::V;

    const int n = a.nrhs;
    const size_t m = 12 * (size_t)a.hc[0].g.Vh;    // complex numbers per right-hand side
    const unsigned G = gridDim.x;
    const size_t gt = (size_t)blockIdx.x * NT + threadIdx.x, T = (size_t)G * NT;

    if (threadIdx.x < (unsigned)n) {
        const Scalars &s = a.sc[threadIdx.x];
        PScal &q = ps[threadIdx.x];
        for (int k = 0; k < 2; k++) {
            q.rho[k] = s.rho[k]; q.rho_old[k] = s.rho_old[k]; q.alpha[k] = s.alpha[k]; q.omega[k] = s.omega[k];
        }
        q.r2 = s.r2; q.b2 = s.b2; q.stop2 = s.stop2; q.done = s.done; q.iter = s.iter;
    }
    __syncthreads();

    bool alive = true;
    for (int it = 0; it < a.maxit && alive; it++) {
        bool any = false;
        for (int k = 0; k < n; k++) any = any || ps[k].done == 0;
        if (!any) break;
        // p = r + beta (p - omega v), beta = (rho / rho_old)(alpha / omega)
        for (int k = 0; k < n; k++) {
            if (ps[k].done) continue;
            double q1[2], q2[2];
            pcdiv(ps[k].rho, ps[k].rho_old, q1);
            pcdiv(ps[k].alpha, ps[k].omega, q2);
            const float br = (float)(q1[0] * q2[0] - q1[1] * q2[1]), bi = (float)(q1[0] * q2[1] + q1[1] * q2[0]);
            const float wr = (float)ps[k].omega[0], wi = (float)ps[k].omega[1];
            V *p = vec<SV>(a.p, k, a.stride);
            const V *r = vec<SV>(a.r, k, a.stride), *v = vec<SV>(a.v, k, a.stride);
            for (size_t i = gt; i < m; i += T) {
                const float2 pv = pld(p[i]), vv = pld(v[i]), rv = pld(r[i]);
                const float dr = pv.x - (wr * vv.x - wi * vv.y);
                const float di = pv.y - (wr * vv.y + wi * vv.x);
                pst(p[i], rv.x + br * dr - bi * di, rv.y + br * di + bi * dr);
            }
        }
        if (!(alive = grid_sync(a.bar, a.err, G))) break;
        for (int half = 0; half < 2 && alive; half++) {
            // half 0: v = Dhat M p; half 1: t = Dhat M s
            if constexpr (RAS) {
                if (a.use_ras) {
                    RasLds<648> &L = *reinterpret_cast<RasLds<648> *>(smem);
                    const ItemRange R = xcd_items(a.nblk * n);
                    for (int b = R.first; b < R.last; b += R.step) {
                        const int rhs = b % n, blk = b / n;
                        if (ps[rhs].done) continue;
                        ras_block<SL, 648, false, SV>(a.ra[half], blk, rhs, L);
                    }
                    if (!(alive = grid_sync(a.bar, a.err, G))) break;
                }
            }
            // o = T_oo^-1 H_oe (M p | M s)
            for (int k = 0; k < n; k++)
                if (!ps[k].done) hop_phase<SL, SV, CLOV_H, NT, 0>(a.hc[half], k, sin, nullptr, nullptr);
            if (!(alive = grid_sync(a.bar, a.err, G))) break;
            // (v | t) = (M p | M s) - k^2 T_ee^-1 H_eo o, with the phase's dot products
            for (int k = 0; k < n; k++) {
                if (ps[k].done) continue;
                double d[3] = {0.0, 0.0, 0.0};
                if (half == 0) hop_phase<SL, SV, XPAY, NT, 1>(a.hx[0], k, sin, a.rt, d);
                else {
                    // <t, s>: conj(t) s = conj(<s, t>); <t, t>
                    hop_phase<SL, SV, XPAY, NT, 2>(a.hx[1], k, sin, a.s, d);
                    d[1] = -d[1];
                }
                put_partials(a, k, d, red);
            }
            if (!(alive = grid_sync(a.bar, a.err, G))) break;
            if (half == 0) {
                // alpha = rho / <rt, v>; s = r - alpha v
                for (int k = 0; k < n; k++) {
                    if (ps[k].done) continue;
                    double v3[3];
                    get_sums(a, k, v3, red);
                    if (threadIdx.x == 0) {
                        if (v3[0] == 0.0 && v3[1] == 0.0) ps[k].done = 2;
                        else {
                            const double d2[2] = {v3[0], v3[1]};
                            pcdiv(ps[k].rho, d2, ps[k].alpha);
                        }
                    }
                    __syncthreads();
                    if (ps[k].done) continue;
                    const float ar = (float)ps[k].alpha[0], ai = (float)ps[k].alpha[1];
                    const V *r = vec<SV>(a.r, k, a.stride), *v = vec<SV>(a.v, k, a.stride);
                    V *s = vec<SV>(a.s, k, a.stride);
                    for (size_t i = gt; i < m; i += T) {
                        const float2 rv = pld(r[i]), vv = pld(v[i]);
                        pst(s[i], rv.x - (ar * vv.x - ai * vv.y), rv.y - (ar * vv.y + ai * vv.x));
                    }
                }
                if (!(alive = grid_sync(a.bar, a.err, G))) break;
            }
        }
        if (!alive) break;
        // omega = <t, s> / <t, t>; x += alpha ph + omega sh; r = s - omega t; <rt, r>, <r, r>
        for (int k = 0; k < n; k++) {
            if (ps[k].done) continue;
            double v3[3];
            get_sums(a, k, v3, red);
            if (threadIdx.x == 0) {
                const double tt = v3[2];
                if (tt == 0.0) { ps[k].omega[0] = 0.0; ps[k].omega[1] = 0.0; }
                else { ps[k].omega[0] = v3[0] / tt; ps[k].omega[1] = v3[1] / tt; }
            }
            __syncthreads();
            const float ar = (float)ps[k].alpha[0], ai = (float)ps[k].alpha[1];
            const float wr = (float)ps[k].omega[0], wi = (float)ps[k].omega[1];
            V *x = vec<SV>(a.x, k, a.stride), *r = vec<SV>(a.r, k, a.stride);
            const V *pv = vec<SV>(RAS && a.use_ras ? a.ph : a.p, k, a.stride);
            const V *sv = vec<SV>(RAS && a.use_ras ? a.sh : a.s, k, a.stride);
            const V *s2 = vec<SV>(a.s, k, a.stride), *tv = vec<SV>(a.t, k, a.stride);
            const V *rt = vec<SV>(a.rt, k, a.stride);
            double d[3] = {0.0, 0.0, 0.0};
            for (size_t i = gt; i < m; i += T) {
                const float2 xv = pld(x[i]), p1 = pld(pv[i]), s1 = pld(sv[i]), ss = pld(s2[i]), t1 = pld(tv[i]);
                pst(x[i], xv.x + (ar * p1.x - ai * p1.y) + (wr * s1.x - wi * s1.y),
                    xv.y + (ar * p1.y + ai * p1.x) + (wr * s1.y + wi * s1.x));
                pst(r[i], ss.x - (wr * t1.x - wi * t1.y), ss.y - (wr * t1.y + wi * t1.x));
                const float2 rn = pld(r[i]), rr = pld(rt[i]);
                d[0] += (double)rr.x * (double)rn.x + (double)rr.y * (double)rn.y;
                d[1] += (double)rr.x * (double)rn.y - (double)rr.y * (double)rn.x;
                d[2] += (double)rn.x * (double)rn.x + (double)rn.y * (double)rn.y;
            }
            put_partials(a, k, d, red);
        }
        if (!(alive = grid_sync(a.bar, a.err, G))) break;
        for (int k = 0; k < n; k++) {
            if (ps[k].done) continue;
            double v3[3];
            get_sums(a, k, v3, red);
            if (threadIdx.x == 0) {
                PScal &q = ps[k];
                q.rho_old[0] = q.rho[0]; q.rho_old[1] = q.rho[1];
                q.rho[0] = v3[0]; q.rho[1] = v3[1];
                q.r2 = v3[2];
                q.iter += 1;
                if (!(v3[2] <= q.stop2 * q.b2) && !(v3[2] >= 0.0)) q.done = 2;
                else if (v3[2] <= q.stop2 * q.b2) q.done = 1;
                else if ((q.omega[0] == 0.0 && q.omega[1] == 0.0) || (v3[0] == 0.0 && v3[1] == 0.0)) q.done = 2;
            }
            __syncthreads();
        }
    }
    // workgroup 0 publishes the scalars
    if (blockIdx.x == 0 && threadIdx.x < (unsigned)n) {
        Scalars &s = a.sc[threadIdx.x];
        const PScal &q = ps[threadIdx.x];
        for (int k = 0; k < 2; k++) {
            s.rho[k] = q.rho[k]; s.rho_old[k] = q.rho_old[k]; s.alpha[k] = q.alpha[k]; s.omega[k] = q.omega[k];
        }
        s.r2 = q.r2;
        s.done = q.done;
        s.iter = q.iter;
    }
}

__global__ void k_persist_reset(unsigned *bar, int *err)
{
    if (threadIdx.x == 0) {
        bar[0] = 0u;
        *err = 0;
    }
}

template <typename SL, typename SV, bool RAS, int NT>
static hipError_t persist_launch(const PersistLaunch &L, PersistArgs &a, hipStream_t st)
{
    auto k = k_inner_persist<SL, SV, RAS, NT>;
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, NT, 0);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorLaunchOutOfResources;
    int G = L.num_cus;   // one workgroup per CU
    if (G > PMAX_WG) G = PMAX_WG;
    G &= ~7;
    if (G < 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_persist_reset, dim3(1), dim3(64), 0, st, a.bar, a.err);
    void *args[] = {&a};
    return hipLaunchCooperativeKernel((const void *)k, dim3(G), dim3(NT), args, 0, st);
}

template <typename SL, typename SV, bool RAS>
static hipError_t persist_nt(const PersistLaunch &L, PersistArgs &a, hipStream_t st)
{
    // the Schwarz block needs 704 threads (648 site pairs); without it 768
    // threads (3 waves per SIMD) leave the hop its registers
    if constexpr (RAS) return persist_launch<SL, SV, true, 704>(L, a, st);
    else return persist_launch<SL, SV, false, 768>(L, a, st);
}

template <typename SL, typename SV>
static hipError_t persist_ras(const PersistLaunch &L, PersistArgs &a, hipStream_t st)
{
    if (L.use_ras) return persist_nt<SL, SV, true>(L, a, st);
    return persist_nt<SL, SV, false>(L, a, st);
}

hipError_t launch_persist(const PersistLaunch &L, hipStream_t st)
{
    if (L.nrhs < 1 || L.nrhs > PMAXR || L.maxit < 1) return hipErrorInvalidValue;
    PersistArgs a{};
    const bool ras = L.use_ras != 0;
    for (int half = 0; half < 2; half++) {
        void *src = half ? L.s : L.p, *pre = ras ? (half ? L.sh : L.ph) : src;
        HopArgs h{};
        h.g = *L.g;
        h.links = L.links;
        h.clov = L.clov_inv;
        h.coef = -L.kappa2;
        h.nrhs = 1;
        h.in_stride = h.out_stride = h.x_stride = L.stride;
        h.p = 1;
        h.in = pre;
        h.out = L.o;
        a.hc[half] = h;
        h.p = 0;
        h.in = L.o;
        h.x = pre;
        h.out = half ? L.t : L.v;
        a.hx[half] = h;
    }
    a.use_ras = L.use_ras;
    if (L.use_ras) {
        // the fused Schwarz kernel's recipe: tile cores, an extended block of at
        // most 648 sites per parity, minimal residual or Jacobi steps
        int ne = 1;
        for (int mu = 0; mu < 4; mu++) {
            if (L.overlap > L.g->B[mu] || L.g->L[mu] < L.g->B[mu] + 2 * L.overlap) return hipErrorInvalidValue;
            ne *= L.g->B[mu] + 2 * L.overlap;
        }
        if (ne / 2 > 648 || L.jacobi) return hipErrorInvalidValue;
        if (L.link_prec == P32C && !L.links_site) return hipErrorInvalidValue;
        for (int half = 0; half < 2; half++) {
            RasArgs &r = a.ra[half];
            r.g = *L.g;
            r.overlap = L.overlap;
            r.iters = L.iters;
            r.in = half ? L.s : L.p;
            r.out = half ? L.sh : L.ph;
            r.links = L.link_prec == P32C ? L.links_site : L.links;
            r.clov_inv = L.clov_inv;
            r.kappa2 = (float)L.kappa2;
            r.sc = nullptr;
            r.nrhs = L.nrhs;
            r.stride = L.stride;
            r.colour = 0;
            r.accumulate = 0;
        }
        a.nblk = L.g->NB[0] * L.g->NB[1] * L.g->NB[2] * L.g->NB[3];
    }
    a.x = L.x; a.r = L.r; a.rt = L.rt; a.p = L.p; a.v = L.v; a.s = L.s; a.t = L.t;
    a.ph = L.ph; a.sh = L.sh; a.o = L.o;
    a.stride = L.stride;
    a.sc = L.sc;
    a.partials = L.partials;
    a.bar = L.bar;
    a.err = L.err;
    a.nrhs = L.nrhs;
    a.maxit = L.maxit;
    if (L.vec_prec == P16) {
        switch (L.link_prec) {
        case P16: return persist_ras<__half, __half>(L, a, st);
        case P16C: return persist_ras<R12h, __half>(L, a, st);
        default: return hipErrorInvalidValue;
        }
    }
    switch (L.link_prec) {
    case P32: return persist_ras<float, float>(L, a, st);
    case P16: return persist_ras<__half, float>(L, a, st);
    case P32C: return persist_ras<R12f, float>(L, a, st);
    case P16C: return persist_ras<R12h, float>(L, a, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace wcl
