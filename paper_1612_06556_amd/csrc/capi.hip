// capi.hip -- the C ABI (include/wcl.h): context, gauge/parameter setup,
// operator application, the solvers and the hopping benchmark.
//
// Solver structure (paper Sec. 2): an FP64 flexible BiCGStab on the even/odd
// Schur system whose preconditioner K is a single-precision BiCGStab on the
// same system, itself right-preconditioned by overlapped RAS; K is applied to
// the normalised vector and scaled back.  All vectors and every BiCGStab
// scalar live on the GPU; the host reads the convergence flags only.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/wcl.h"
#include "wcl_launch.h"

using namespace wcl;

// Fixed device scratch of wcl_apply_noalloc (for callers that cannot
// allocate): every GPU the library runs on holds its own copy until the
// process ends.  In host code `scratch` names a host-side stand-in, not the
// device array: host code uses only the per-device address that
// hipGetSymbolAddress returns (g_scratch below).
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
constexpr size_t NOALLOC_BYTES_PER_HALF_SITE = 768;   // FP64 in + out e/o fields, both parities
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg)
{
    g_err = msg;
    return code;
}

#define HIPCHK(call)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(WCL_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));      \
    } while (0)

#define CHK(call)                     \
    do {                              \
        int rc_ = (call);             \
        if (rc_ != WCL_OK) return rc_; \
    } while (0)

struct Buf {
    void *p = nullptr;
    size_t bytes = 0;
};

}  // namespace

struct wcl_ctx {
    Geom g;
    int V = 0, Vh = 0;
    hipStream_t st = nullptr;
    int device = 0;
    void *U64 = nullptr, *U32 = nullptr, *U16 = nullptr;
    void *U32c = nullptr, *U16c = nullptr;  // two-row links (built when compression is on)
    void *U32s = nullptr;                   // per-site copy of U32c (the fused Schwarz kernel's)
    int compress = 0;                       // FP32/FP16 tiers read the two-row links
    void *T64 = nullptr, *Ti64 = nullptr, *T32 = nullptr, *Ti32 = nullptr, *T16 = nullptr, *Ti16 = nullptr;
    int *info = nullptr;
    double kappa = 0, csw = 0;
    bool have_gauge = false, have_params = false;
    int ras_overlap = 1, ras_iters = 4, ras_solver = WCL_RAS_MR;
    int ras_mult = 0;   // 1: multiplicative Schwarz (colour sweeps) instead of additive
    int ras_cores[4] = {0, 0, 0, 0};   // explicit Schwarz cores (0: the tiles, fused kernel)
    GrasPlan gras{};                   // block fields of the global-memory Schwarz path
    bool gras_ready = false;
    std::vector<Buf> ws;        // workspace, indexed by slot
    double *partials = nullptr; // [cap][6][pstride]
    int pstride = 0;            // partial sums per term and right-hand side (>= every launch's workgroups)
    Scalars *sc = nullptr;      // [3][cap]: outer, inner, final/scratch scalars per right-hand side
    Scalars *sc_host = nullptr; // pinned mirror
    int cap = 0;                // right-hand sides the scalar and partial buffers hold
    // hopping-kernel launch configuration (set by wcl_set_tuning / wcl_autotune_hop)
    int hop_block = 256, hop_depth = 2, hop_xcd = 1, hop_nt = 0, hop_lds = 1;
    int hop_rhs = 1;   // right-hand sides per thread in batched launches (1, 2, 4)
    int hop_tpw = 1;   // consecutive site blocks per hop workgroup
    int num_cus = 0;   // compute units of the device (one persistent workgroup each)
    // event profiling of kernel classes
    struct Rec {
        int kclass;
        hipEvent_t e0, e1;
        double bytes, flops;
    };
    bool prof = false;
    int prof_mask = (1 << WCL_K_COUNT) - 1;   // classes whose launches carry timing events
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    wcl_kstat stats[WCL_K_COUNT];
};

namespace {

int alloc(void **p, size_t bytes)
{
    if (hipMalloc(p, bytes) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(WCL_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
    return WCL_OK;
}

// Workspace slot (allocated once, grown on demand).
int wsget(wcl_ctx *c, int slot, size_t bytes, void **out)
{
    if ((int)c->ws.size() <= slot) c->ws.resize(slot + 1);
    Buf &b = c->ws[slot];
    if (b.bytes < bytes) {
        if (b.p) {
            HIPCHK(hipStreamSynchronize(c->st));
            (void)hipFree(b.p);
        }
        b.p = nullptr;
        b.bytes = 0;
        CHK(alloc(&b.p, bytes));
        b.bytes = bytes;
    }
    *out = b.p;
    return WCL_OK;
}

// Link storage the kernels read for a precision tier (two-row links when on).
int eff_lprec(const wcl_ctx *c, int prec)
{
    if (c->compress && prec == P32) return P32C;
    if (c->compress && prec == P16) return P16C;
    return prec;
}
void *links_for(wcl_ctx *c, int prec)
{
    switch (prec) {
        case P64: return c->U64;
        case P32: return c->U32;
        case P16: return c->U16;
        case P32C: return c->U32c;
        default: return c->U16c;
    }
}
void *clov_for(wcl_ctx *c, int prec)
{
    return prec == P64 ? c->T64 : (prec == P32 || prec == P32C) ? c->T32 : c->T16;
}
void *clovinv_for(wcl_ctx *c, int prec)
{
    return prec == P64 ? c->Ti64 : (prec == P32 || prec == P32C) ? c->Ti32 : c->Ti16;
}

char *par(void *field, int prec, size_t Vh, int p) { return (char *)field + p * spinor_bytes(prec_bytes(prec), Vh); }
const char *par(const void *field, int prec, size_t Vh, int p)
{
    return (const char *)field + p * spinor_bytes(prec_bytes(prec), Vh);
}

HopLaunch hop_base(wcl_ctx *c, int lprec, int sprec)
{
    HopLaunch L;
    memset(&L, 0, sizeof(L));
    L.g = &c->g;
    L.link_prec = eff_lprec(c, lprec);
    L.spin_prec = sprec;
    L.links = links_for(c, L.link_prec);
    L.nrhs = 1;
    L.xcd = c->hop_xcd;
    L.block = c->hop_block;
    L.depth = c->hop_depth;
    L.rhs_per_thread = c->hop_rhs;
    L.tpw = c->hop_tpw;
    L.nontemporal = c->hop_nt;
    L.lds_stage = c->hop_lds;
    return L;
}

hipEvent_t take_event(wcl_ctx *c)
{
    if (!c->pool.empty()) {
        hipEvent_t e = c->pool.back();
        c->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch wrappers: with profiling on, bracket the launch with events and keep
// its algorithmic bytes and flops.
template <typename F>
int profiled(wcl_ctx *c, int kclass, double bytes, double flops, F &&launch)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool timed = c->prof && ((c->prof_mask >> kclass) & 1);
    if (timed) {
        e0 = take_event(c);
        e1 = take_event(c);
        if (!e0 || !e1) return fail(WCL_EHIP, "hipEventCreate failed");
        HIPCHK(hipEventRecord(e0, c->st));
    }
    HIPCHK(launch());
    if (timed) HIPCHK(hipEventRecord(e1, c->st));
    if (c->prof) c->recs.push_back({kclass, e0, e1, bytes, flops});
    return WCL_OK;
}

// A single-kernel launch timed by events in its own dispatch packet.
template <typename F>
int profiled_ev(wcl_ctx *c, int kclass, double bytes, double flops, F &&launch)
{
    LaunchEvents ev{nullptr, nullptr};
    if (c->prof && ((c->prof_mask >> kclass) & 1)) {
        ev.start = take_event(c);
        ev.stop = take_event(c);
        if (!ev.start || !ev.stop) return fail(WCL_EHIP, "hipEventCreate failed");
    }
    HIPCHK(launch(ev));
    if (c->prof) c->recs.push_back({kclass, ev.start, ev.stop, bytes, flops});
    return WCL_OK;
}

int run_hop(wcl_ctx *c, const HopLaunch &L)
{
    double b = 0, f = 0;
    if (c->prof) hop_work(L, &b, &f);
    return profiled_ev(c, WCL_K_HOP, b, f, [&](const LaunchEvents &ev) {
        HopLaunch T = L;
        T.ev = ev;
        return launch_hop(T, c->st);
    });
}

// The Schwarz settings need the global-memory block path: explicit cores,
// the BiCGStab block solver, or an extended block beyond the fused kernel's
// LDS (or wider than the neighbouring tile).
bool ras_generic(const wcl_ctx *c)
{
    if (c->ras_cores[0] || c->ras_solver == WCL_RAS_BICGSTAB || !gras_fits_fused(c->g, c->ras_overlap)) return true;
    for (int mu = 0; mu < 4; mu++)
        if (c->ras_overlap > c->g.B[mu]) return true;
    return false;
}

int ensure_gras(wcl_ctx *c);

int run_ras(wcl_ctx *c, const RasLaunch &R)
{
    double b = 0, f = 0;
    if (ras_generic(c)) {
        CHK(ensure_gras(c));
        if (c->prof) gras_work(c->gras, R, c->ras_solver, &b, &f);
        return profiled(c, WCL_K_RAS, b, f, [&] { return launch_gras(c->gras, R, c->ras_solver, c->st); });
    }
    if (c->prof) ras_work(R, &b, &f);
    return profiled_ev(c, WCL_K_RAS, b, f, [&](const LaunchEvents &ev) {
        RasLaunch T = R;
        T.ev = ev;
        return launch_ras(T, c->st);
    });
}

int schur(wcl_ctx *c, int lprec, int sprec, const void *in_e, void *out_e, void *tmp_o, const Scalars *sc,
          int nrhs = 1);

// Multiplicative Schwarz: out = 0; for colour k = 0 .. 15: r = in - Dhat out
// (r = in for k = 0), then the colour-k block solves of r added to out.  R
// carries the block recipe, precisions, scalars and right-hand sides; rt, tt
// and to are vectors of R's storage (residual, Dhat out, Schur odd temp).
int run_sap(wcl_ctx *c, RasLaunch R, int lprec, int vprec, const void *in, void *out, void *rt, void *tt,
            void *to)
{
    const size_t m = 12 * (size_t)c->Vh;
    HIPCHK(launch_zero(vprec, R.nrhs * m, out, c->st));
    R.out = out;
    R.accumulate = true;
    for (int k = 0; k < 16; k++) {
        R.in = in;
        if (k > 0) {
            CHK(schur(c, lprec, vprec, out, tt, to, R.sc, R.nrhs));
            HIPCHK(launch_copy(vprec, R.nrhs * m, in, rt, c->st));
            HIPCHK(launch_axpby(vprec, R.nrhs * m, make_double2(-1.0, 0.0), tt, make_double2(1.0, 0.0), rt, c->st));
            R.in = rt;
        }
        R.colour = k + 1;
        CHK(run_ras(c, R));
    }
    return WCL_OK;
}

int run_clover(wcl_ctx *c, int lp, int sp, int p, const void *clov, const void *in, void *out, int nrhs = 1,
               size_t in_stride = 0, size_t out_stride = 0)
{
    const double sb = sp == P64 ? 192.0 : sp == P32 ? 96.0 : 48.0;
    const double cb = lp == P64 ? 576.0 : lp == P32 ? 288.0 : 144.0;
    return profiled_ev(c, WCL_K_CLOVER, (2 * sb * nrhs + cb) * c->Vh, 504.0 * c->Vh * nrhs, [&](const LaunchEvents &ev) {
        return launch_clover(c->g, lp, sp, p, clov, in, out, c->st, nrhs, in_stride, out_stride, ev);
    });
}

// Byte strides of batched fields: an even (or odd) vector per right-hand
// side, and a full field (both parities) per right-hand side.
size_t half_bytes(int prec, size_t Vh) { return spinor_bytes(prec_bytes(prec), Vh); }
size_t full_bytes(int prec, size_t Vh) { return 2 * spinor_bytes(prec_bytes(prec), Vh); }

// One parity of the full operator: out_p = A_pp x_p + coef H in_{1-p}
int full_D_parity(wcl_ctx *c, int lprec, int sprec, int p, const void *field_in, void *field_out, int dagger,
                  const Scalars *sc, int nrhs)
{
    HopLaunch L = hop_base(c, lprec, sprec);
    L.mode = CLOVX;
    L.dagger = dagger;
    L.p = p;
    L.in = par(field_in, sprec, c->Vh, 1 - p);
    L.x = par(field_in, sprec, c->Vh, p);
    L.out = par(field_out, sprec, c->Vh, p);
    L.clov = clov_for(c, lprec);
    L.coef = -c->kappa;
    L.sc = sc;
    L.nrhs = nrhs;
    L.in_stride = L.out_stride = L.x_stride = full_bytes(sprec, c->Vh);
    CHK(run_hop(c, L));
    return WCL_OK;
}

int full_D(wcl_ctx *c, int lprec, int sprec, const void *in, void *out, int dagger, const Scalars *sc = nullptr,
           int nrhs = 1)
{
    CHK(full_D_parity(c, lprec, sprec, 0, in, out, dagger, sc, nrhs));
    CHK(full_D_parity(c, lprec, sprec, 1, in, out, dagger, sc, nrhs));
    return WCL_OK;
}

// Schur operator on even fields: tmp_o = A_oo^-1 H_oe in_e ; out_e = in_e - k^2 A_ee^-1 H_eo tmp_o
int schur(wcl_ctx *c, int lprec, int sprec, const void *in_e, void *out_e, void *tmp_o, const Scalars *sc,
          int nrhs)
{
    HopLaunch L = hop_base(c, lprec, sprec);
    L.clov = clovinv_for(c, lprec);
    L.sc = sc;
    L.nrhs = nrhs;
    L.in_stride = L.out_stride = L.x_stride = half_bytes(sprec, c->Vh);
    L.mode = CLOV_H;
    L.p = 1;
    L.in = in_e;
    L.out = tmp_o;
    CHK(run_hop(c, L));
    L.mode = XPAY;
    L.p = 0;
    L.in = tmp_o;
    L.x = in_e;
    L.out = out_e;
    L.coef = -c->kappa * c->kappa;
    CHK(run_hop(c, L));
    return WCL_OK;
}

// Schur operator with the BiCGStab reductions fused into its second half:
// ndot 1: partials of <w, out>; ndot 2: of <out, w> and <out, out>, at
// c->partials (stride c->pstride), *nparts per term.
int schur_dot(wcl_ctx *c, int lprec, int sprec, const void *in_e, void *out_e, void *tmp_o, const Scalars *sc,
              int nrhs, int ndot, const void *w, int *nparts)
{
    HopLaunch L = hop_base(c, lprec, sprec);
    L.clov = clovinv_for(c, lprec);
    L.sc = sc;
    L.nrhs = nrhs;
    L.in_stride = L.out_stride = L.x_stride = half_bytes(sprec, c->Vh);
    L.mode = CLOV_H;
    L.p = 1;
    L.in = in_e;
    L.out = tmp_o;
    CHK(run_hop(c, L));
    L.mode = XPAY;
    L.p = 0;
    L.in = tmp_o;
    L.x = in_e;
    L.out = out_e;
    L.coef = -c->kappa * c->kappa;
    L.ndot = ndot;
    L.dotw = w;
    L.partials = c->partials;
    L.pstride = c->pstride;
    *nparts = hop_parts(L);
    CHK(run_hop(c, L));
    return WCL_OK;
}

// bhat_e = A_ee^-1 (b_e + k H_eo A_oo^-1 b_o)  (b: full FP64 fields, bhat, tmp: even/odd FP64 vectors)
int schur_rhs64(wcl_ctx *c, const void *b, void *bhat_e, void *tmp_o, void *tmp_e, int nrhs = 1)
{
    const size_t fb = full_bytes(P64, c->Vh), hb = half_bytes(P64, c->Vh);
    CHK(run_clover(c, P64, P64, 1, c->Ti64, par(b, P64, c->Vh, 1), tmp_o, nrhs, fb, hb));
    CHK(run_clover(c, P64, P64, 0, c->Ti64, par(b, P64, c->Vh, 0), tmp_e, nrhs, fb, hb));
    HopLaunch L = hop_base(c, P64, P64);
    L.mode = XPAY;
    L.p = 0;
    L.in = tmp_o;
    L.x = tmp_e;
    L.out = bhat_e;
    L.clov = c->Ti64;
    L.coef = c->kappa;
    L.nrhs = nrhs;
    L.in_stride = L.out_stride = L.x_stride = hb;
    CHK(run_hop(c, L));
    return WCL_OK;
}

// x_o = A_oo^-1 (b_o + k H_oe x_e) into the odd half of the full fields x (even half = x_e already)
int reconstruct64(wcl_ctx *c, const void *b, void *x, void *tmp_o, int nrhs = 1)
{
    const size_t fb = full_bytes(P64, c->Vh), hb = half_bytes(P64, c->Vh);
    CHK(run_clover(c, P64, P64, 1, c->Ti64, par(b, P64, c->Vh, 1), tmp_o, nrhs, fb, hb));
    HopLaunch L = hop_base(c, P64, P64);
    L.mode = XPAY;
    L.p = 1;
    L.in = par(x, P64, c->Vh, 0);
    L.x = tmp_o;
    L.out = par(x, P64, c->Vh, 1);
    L.clov = c->Ti64;
    L.coef = c->kappa;
    L.nrhs = nrhs;
    L.in_stride = L.out_stride = fb;
    L.x_stride = hb;
    CHK(run_hop(c, L));
    return WCL_OK;
}

// Device address of `scratch` per device, taken once per device with that
// device current (wcl_create).
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch[MAX_DEVICES] = {};

int scratch_init(int device)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0 || device >= MAX_DEVICES) return fail(WCL_EINVAL, "device index beyond the scratch table");
    if (g_scratch[device]) return WCL_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(WCL_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[device] = ptr;
    return WCL_OK;
}

int check_prec(int prec) { return (prec == 64 || prec == 32 || prec == 16) ? WCL_OK : fail(WCL_EINVAL, "prec must be 64, 32 or 16"); }

// Scalar and partial buffers for n right-hand sides: outer scalars at
// sc[0, n), inner at sc[cap, cap + n), per-rhs flags/scratch at sc[2 cap, ...).
int ensure_batch(wcl_ctx *c, int n)
{
    if (n <= c->cap) return WCL_OK;
    HIPCHK(hipStreamSynchronize(c->st));
    if (c->sc) (void)hipFree(c->sc);
    if (c->partials) (void)hipFree(c->partials);
    if (c->sc_host) (void)hipHostFree(c->sc_host);
    c->sc = nullptr; c->partials = nullptr; c->sc_host = nullptr; c->cap = 0;
    CHK(alloc((void **)&c->sc, sizeof(Scalars) * 3 * n));
    CHK(alloc((void **)&c->partials, sizeof(double) * 6 * (size_t)c->pstride * n));
    if (hipHostMalloc((void **)&c->sc_host, sizeof(Scalars) * 3 * n, hipHostMallocDefault) != hipSuccess)
        return fail(WCL_ENOMEM, "hipHostMalloc failed");
    memset(c->sc_host, 0, sizeof(Scalars) * 3 * n);
    HIPCHK(hipMemcpyAsync(c->sc, c->sc_host, sizeof(Scalars) * 3 * n, hipMemcpyHostToDevice, c->st));
    c->cap = n;
    return WCL_OK;
}

Scalars *SO(wcl_ctx *c) { return c->sc; }
Scalars *SI(wcl_ctx *c) { return c->sc + c->cap; }
Scalars *SF(wcl_ctx *c) { return c->sc + 2 * c->cap; }
Scalars *HO(wcl_ctx *c) { return c->sc_host; }
Scalars *HI(wcl_ctx *c) { return c->sc_host + c->cap; }
Scalars *HF(wcl_ctx *c) { return c->sc_host + 2 * c->cap; }

int read_sc(wcl_ctx *c, Scalars *host, const Scalars *dev, int n)
{
    HIPCHK(hipMemcpyAsync(host, dev, sizeof(Scalars) * n, hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    return WCL_OK;
}

int write_sc(wcl_ctx *c, Scalars *dev, const Scalars *host, int n)
{
    HIPCHK(hipMemcpyAsync(dev, host, sizeof(Scalars) * n, hipMemcpyHostToDevice, c->st));
    return WCL_OK;
}

// |v_k|^2 of n right-hand sides (m complex numbers each, `stride` apart) into dst[k].t[0]
int norms_dev(wcl_ctx *c, int prec, size_t m, const void *v, size_t stride, int n, Scalars *dst)
{
    const void *a[1] = {v}, *b[1] = {v};
    HIPCHK(launch_dots(prec, m, 1, a, b, c->partials, nullptr, c->st, n, stride, c->pstride));
    HIPCHK(launch_finalize(NORM_ONLY, 2, c->partials, dst, c->st, n, nullptr, c->pstride));
    return WCL_OK;
}

// host copies of |v_k|^2 (uses the scratch scalars' t[0])
int norms_host(wcl_ctx *c, int prec, size_t m, const void *v, size_t stride, int n, double *out)
{
    CHK(norms_dev(c, prec, m, v, stride, n, SF(c)));
    CHK(read_sc(c, HF(c), SF(c), n));
    for (int k = 0; k < n; k++) out[k] = HF(c)[k].t[0];
    return WCL_OK;
}

enum Slot {
    S_IN64 = 0, S_OUT64, S_IN32, S_OUT32, S_TMP64E, S_TMP64O,
    // solver FP64 even vectors
    S_B64, S_X64, S_R64F, S_BH, S_XE, S_R, S_RT, S_P, S_V, S_S, S_T, S_PH, S_SH, S_O64,
    // inner FP32 even vectors
    S_RHS32, S_X32, S_R32, S_RT32, S_P32, S_V32, S_S32, S_T32, S_PH32, S_SH32, S_O32,
    // plain FP64 full-field vectors
    S_PR, S_PRT, S_PP, S_PV, S_PS, S_PT, S_PX,
    // gradient
    S_GX, S_GY, S_GK, S_GG, S_GHX, S_GCX,
    // SU(3) check partials
    S_SU3,
    // multiplicative Schwarz: residual, Dhat z, Schur odd temporary
    S_SAPR, S_SAPT, S_SAPO,
    // global-memory Schwarz path: tables, block fields, per-block state
    S_GRAS_T, S_GRAS_V, S_GRAS_S,
    // field strength planes of the clover setup
    S_CLOVF,
    // persistent inner solve: per-workgroup partial sums, barrier counters + time-out flag
    S_PPART, S_PBAR,
    // bench copies start here
    S_BENCH = 64,
};

// Tables and block fields of the global-memory Schwarz path for the current
// settings (rebuilt when the cores, overlap or the solver's field count change).
int ensure_gras(wcl_ctx *c)
{
    if (!ras_generic(c)) return WCL_OK;
    const int *cores = c->ras_cores[0] ? c->ras_cores : c->g.B;
    const int need = gras_fields(c->ras_solver);
    GrasPlan &P = c->gras;
    bool same = c->gras_ready && P.overlap == c->ras_overlap && P.nvec >= need;
    for (int mu = 0; mu < 4; mu++) same = same && P.cores[mu] == cores[mu];
    if (same) return WCL_OK;
    c->gras_ready = false;
    GrasPlan Q{};
    std::vector<uint32_t> host;
    if (gras_tables(c->g, cores, c->ras_overlap, &Q, host) != hipSuccess)
        return fail(WCL_EINVAL, "Schwarz cores must be even, divide the lattice and fit with the overlap");
    Q.nvec = need;
    void *t, *v, *st;
    CHK(wsget(c, S_GRAS_T, host.size() * sizeof(uint32_t), &t));
    CHK(wsget(c, S_GRAS_V, gras_vector_bytes(Q), &v));
    CHK(wsget(c, S_GRAS_S, gras_state_bytes(Q), &st));
    HIPCHK(hipStreamSynchronize(c->st));
    HIPCHK(hipMemcpy(t, host.data(), host.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    gras_bind(&Q, t, v, st);
    P = Q;
    c->gras_ready = true;
    return WCL_OK;
}

// Largest SU(3) defect accepted for two-row link storage (the FP32 tier's
// own rounding is 6e-8).
constexpr double SU3_TOL = 1e-7;

// Check that the FP64 links are SU(3) (two-row storage rebuilds row 2 as
// conj(row0 x row1)), then write the FP32 and FP16 two-row copies.
int build_compressed(wcl_ctx *c)
{
    const size_t Vh = c->Vh;
    // each copy on its own: a failed allocation leaves the others for the next call
    if (!c->U32c) CHK(alloc(&c->U32c, link_bytes_c(P32C, Vh)));
    if (!c->U16c) CHK(alloc(&c->U16c, link_bytes_c(P16C, Vh)));
    if (!c->U32s) CHK(alloc(&c->U32s, link_bytes_c(P32C, Vh)));
    const int nb = 256;
    void *part;
    CHK(wsget(c, S_SU3, nb * sizeof(double), &part));
    HIPCHK(launch_su3_check(c->g, c->U64, (double *)part, nb, c->st));
    std::vector<double> h(nb);
    HIPCHK(hipMemcpyAsync(h.data(), part, nb * sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    double m = 0.0;
    for (double d : h)
        if (d > m || d != d) m = d;
    if (!(m <= SU3_TOL)) {
        char msg[160];
        snprintf(msg, sizeof msg, "two-row link storage needs SU(3) links: largest defect %.3e > %.1e", m, SU3_TOL);
        return fail(WCL_EINVAL, msg);
    }
    HIPCHK(launch_compress_links(c->g, c->U64, c->U32c, c->U16c, c->U32s, c->st));
    return WCL_OK;
}

}  // namespace

// ===========================================================================
extern "C" {

const char *wcl_last_error(void) { return g_err.c_str(); }

int wcl_create(const int dims[4], int t_bc, const int tile[4], void *hip_stream, wcl_ctx **out)
{
    if (!dims || !out) return fail(WCL_EINVAL, "null argument");
    *out = nullptr;
    if (t_bc != 1 && t_bc != -1) return fail(WCL_EINVAL, "t_bc must be +1 or -1");
    int B[4];
    for (int mu = 0; mu < 4; mu++) {
        if (dims[mu] < 4 || (dims[mu] & 1)) return fail(WCL_EINVAL, "lattice extents must be even and >= 4");
    }
    if (tile) {
        for (int mu = 0; mu < 4; mu++) B[mu] = tile[mu];
    } else {
        bool four = true;
        for (int mu = 0; mu < 4; mu++) four = four && (dims[mu] % 4 == 0);
        for (int mu = 0; mu < 4; mu++) B[mu] = four ? 4 : 2;
    }
    for (int mu = 0; mu < 4; mu++)
        if (B[mu] < 2 || (B[mu] & 1) || dims[mu] % B[mu]) return fail(WCL_EINVAL, "tile extents must be even and divide the lattice");
    const long long V = (long long)dims[0] * dims[1] * dims[2] * dims[3];
    // every field is addressed with 32-bit byte offsets; the largest, the FP64
    // links (576 bytes a site), must stay below 4 GiB
    if (V * 576ll >= (1ll << 32)) return fail(WCL_EINVAL, "lattice too large (at most 7456540 sites)");
    wcl_ctx *c = new wcl_ctx();
    Geom &g = c->g;
    for (int mu = 0; mu < 4; mu++) {
        g.L[mu] = dims[mu];
        g.B[mu] = B[mu];
        g.NB[mu] = dims[mu] / B[mu];
    }
    g.Vh = (int)(V / 2);
    g.Hb = B[0] * B[1] * B[2] * B[3] / 2;
    g.tbc = t_bc;
    g.sl[0] = 1; g.sl[1] = B[0]; g.sl[2] = B[0] * B[1]; g.sl[3] = B[0] * B[1] * B[2];
    g.sb[0] = 1; g.sb[1] = g.NB[0]; g.sb[2] = g.NB[0] * g.NB[1]; g.sb[3] = g.NB[0] * g.NB[1] * g.NB[2];
    g.dHb = make_fastdiv(g.Hb);
    g.dNB0 = make_fastdiv(g.NB[0]);
    g.dNB1 = make_fastdiv(g.NB[1]);
    g.dNB2 = make_fastdiv(g.NB[2]);
    g.dBh0 = make_fastdiv(B[0] / 2);
    g.dB1 = make_fastdiv(B[1]);
    g.dB2 = make_fastdiv(B[2]);
    c->V = (int)V;
    c->Vh = g.Vh;
    // partial sums per term: the BLAS grids (<= 8192 workgroups) and the hop
    // launches with fused reductions (one workgroup per 64 or more sites)
    c->pstride = std::max(8192, (g.Vh + 63) / 64);
    c->st = (hipStream_t)hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess ||
        hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess) {
        delete c;
        return fail(WCL_EHIP, "no HIP device");
    }
    int rc = WCL_OK;
    if ((rc = scratch_init(c->device)) != WCL_OK || (rc = alloc((void **)&c->info, sizeof(int))) != WCL_OK ||
        (rc = ensure_batch(c, 1)) != WCL_OK) {
        wcl_destroy(c);
        return rc;
    }
    *out = c;
    return WCL_OK;
}

int wcl_set_stream(wcl_ctx *c, void *s)
{
    if (!c) return fail(WCL_EINVAL, "null context");
    c->st = (hipStream_t)s;
    return WCL_OK;
}

int wcl_destroy(wcl_ctx *c)
{
    if (!c) return WCL_OK;
    (void)hipStreamSynchronize(c->st);
    void *ptrs[] = {c->U64, c->U32, c->U16, c->U32c, c->U16c, c->U32s, c->T64, c->Ti64, c->T32, c->Ti32, c->T16, c->Ti16, c->info,
                    c->partials, c->sc};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (Buf &b : c->ws)
        if (b.p) (void)hipFree(b.p);
    if (c->sc_host) (void)hipHostFree(c->sc_host);
    for (auto &r : c->recs) {
        (void)hipEventDestroy(r.e0);
        (void)hipEventDestroy(r.e1);
    }
    for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
    delete c;
    return WCL_OK;
}


int wcl_set_gauge(wcl_ctx *c, const double *U)
{
    if (!c || !U) return fail(WCL_EINVAL, "null argument");
    const size_t Vh = c->Vh;
    // each field on its own: a failed allocation leaves the others for the next call
    if (!c->U64) CHK(alloc(&c->U64, link_bytes(8, Vh)));
    if (!c->U32) CHK(alloc(&c->U32, link_bytes(4, Vh)));
    if (!c->U16) CHK(alloc(&c->U16, link_bytes(2, Vh)));
    HIPCHK(launch_ingest_gauge(c->g, U, c->U64, c->U32, c->U16, c->st));
    c->have_gauge = false;
    c->have_params = false;
    if (c->compress) CHK(build_compressed(c));
    c->have_gauge = true;
    return WCL_OK;
}

extern "C" int wcl_set_compression(wcl_ctx *c, int enable)
{
    if (!c) return fail(WCL_EINVAL, "null context");
    if (enable != 0 && enable != 1) return fail(WCL_EINVAL, "enable must be 0 or 1");
    if (enable && c->have_gauge && !c->compress) {
        c->compress = 1;
        const int rc = build_compressed(c);
        if (rc != WCL_OK) {
            c->compress = 0;
            return rc;
        }
    }
    c->compress = enable;
    return WCL_OK;
}

int wcl_set_params(wcl_ctx *c, double kappa, double csw)
{
    if (!c) return fail(WCL_EINVAL, "null context");
    if (!c->have_gauge) return fail(WCL_ESTATE, "wcl_set_params before wcl_set_gauge");
    if (!std::isfinite(kappa) || !std::isfinite(csw)) return fail(WCL_EINVAL, "kappa and csw must be finite");
    const size_t Vh = c->Vh;
    void **cl[] = {&c->T64, &c->Ti64, &c->T32, &c->Ti32, &c->T16, &c->Ti16};
    const int cl_bytes[] = {8, 8, 4, 4, 2, 2};
    for (int i = 0; i < 6; ++i)
        if (!*cl[i]) CHK(alloc(cl[i], clover_bytes(cl_bytes[i], Vh)));
    c->kappa = kappa;
    c->csw = csw;
    int zero = 0, bad = 0;
    HIPCHK(hipMemcpyAsync(c->info, &zero, sizeof(int), hipMemcpyHostToDevice, c->st));
    void *fbuf;
    CHK(wsget(c, S_CLOVF, (size_t)6 * 9 * 2 * c->Vh * sizeof(double), &fbuf));
    HIPCHK(launch_clover_build(c->g, c->U64, csw * kappa, c->T64, c->Ti64, c->T32, c->Ti32, c->T16, c->Ti16,
                               c->info, (double *)fbuf, c->st));
    HIPCHK(hipMemcpyAsync(&bad, c->info, sizeof(int), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    if (bad) return fail(WCL_ENAN, std::to_string(bad) + " clover blocks are not positive definite");
    c->have_params = true;
    return WCL_OK;
}

int wcl_set_ras(wcl_ctx *c, int overlap, int iters, int solver, int multiplicative)
{
    if (c && multiplicative != 0 && multiplicative != 1) return fail(WCL_EINVAL, "multiplicative must be 0 or 1");
    if (!c) return fail(WCL_EINVAL, "null context");
    if (overlap < 0 || iters < 1) return fail(WCL_EINVAL, "overlap >= 0 and iters >= 1 required");
    if (solver != WCL_RAS_MR && solver != WCL_RAS_JACOBI && solver != WCL_RAS_BICGSTAB)
        return fail(WCL_EINVAL, "unknown RAS block solver");
    const int *cores = c->ras_cores[0] ? c->ras_cores : c->g.B;
    for (int mu = 0; mu < 4; mu++)
        if (c->g.L[mu] < cores[mu] + 2 * overlap) return fail(WCL_EINVAL, "RAS extended block does not fit the lattice");
    const int o0 = c->ras_overlap, i0 = c->ras_iters, s0 = c->ras_solver, m0 = c->ras_mult;
    c->ras_overlap = overlap;
    c->ras_iters = iters;
    c->ras_solver = solver;
    c->ras_mult = 0;
    if (multiplicative && ras_generic(c)) {
        c->ras_overlap = o0; c->ras_iters = i0; c->ras_solver = s0; c->ras_mult = m0;
        return fail(WCL_EINVAL, "multiplicative Schwarz needs tile cores, a minimal-residual or Jacobi block "
                                "solver and an extended block of at most 648 sites per parity");
    }
    c->ras_mult = multiplicative;
    const int rc = ensure_gras(c);
    if (rc != WCL_OK) {
        c->ras_overlap = o0; c->ras_iters = i0; c->ras_solver = s0; c->ras_mult = m0;
    }
    return rc;
}

int wcl_set_ras_cores(wcl_ctx *c, const int cores[4])
{
    if (!c) return fail(WCL_EINVAL, "null context");
    int nc[4] = {0, 0, 0, 0};
    if (cores && (cores[0] || cores[1] || cores[2] || cores[3])) {
        for (int mu = 0; mu < 4; mu++) {
            if (cores[mu] < 2 || (cores[mu] & 1) || c->g.L[mu] % cores[mu] ||
                c->g.L[mu] < cores[mu] + 2 * c->ras_overlap)
                return fail(WCL_EINVAL, "Schwarz cores must be even, divide the lattice and fit with the overlap");
            nc[mu] = cores[mu];
        }
        if (c->ras_mult) return fail(WCL_EINVAL, "explicit cores run the additive Schwarz only");
    }
    int old[4];
    for (int mu = 0; mu < 4; mu++) {
        old[mu] = c->ras_cores[mu];
        c->ras_cores[mu] = nc[mu];
    }
    const int rc = ensure_gras(c);
    if (rc != WCL_OK)
        for (int mu = 0; mu < 4; mu++) c->ras_cores[mu] = old[mu];
    return rc;
}

int wcl_apply_op(wcl_ctx *c, int op, const double *in, double *out, int nrhs, int prec)
{
    if (!c || !in || !out) return fail(WCL_EINVAL, "null argument");
    if (!c->have_params) return fail(WCL_ESTATE, "operator used before wcl_set_gauge and wcl_set_params");
    CHK(check_prec(prec));
    if (nrhs < 1) return fail(WCL_EINVAL, "nrhs must be >= 1");
    if (op < 0 || op > WCL_OP_DDAG) return fail(WCL_EINVAL, "unknown op");
    if (op == WCL_OP_RAS && prec == 64) return fail(WCL_EINVAL, "RAS runs in FP32 arithmetic: prec 32 or 16");
    const size_t Vh = c->Vh;
    const int lp = prec;
    const int sp = (op == WCL_OP_RAS) ? P32 : prec;  // RAS vectors are FP32 in both tiers
    void *a64, *b64, *t64e, *t64o, *a, *b;
    CHK(wsget(c, S_IN64, spinor_bytes(8, Vh) * 2, &a64));
    CHK(wsget(c, S_OUT64, spinor_bytes(8, Vh) * 2, &b64));
    CHK(wsget(c, S_TMP64E, spinor_bytes(8, Vh), &t64e));
    CHK(wsget(c, S_TMP64O, spinor_bytes(8, Vh), &t64o));
    if (sp != P64) {
        CHK(wsget(c, S_IN32, spinor_bytes(prec_bytes(sp), Vh) * 2, &a));
        CHK(wsget(c, S_OUT32, spinor_bytes(prec_bytes(sp), Vh) * 2 + spinor_bytes(prec_bytes(sp), Vh), &b));
    } else {
        a = a64;
        b = b64;
    }
    for (int k = 0; k < nrhs; k++) {
        const double *ink = in + (size_t)k * c->V * 24;
        double *outk = out + (size_t)k * c->V * 24;
        HIPCHK(launch_pack_spinor(c->g, ink, a64, c->st));
        if (sp != P64) HIPCHK(launch_convert(P64, sp, 2 * Vh, Vh, Vh, a64, a, nullptr, 0, 1.0, c->st));
        switch (op) {
        case WCL_OP_HOP:
            for (int p = 0; p < 2; p++) {
                HopLaunch L = hop_base(c, lp, sp);
                L.mode = HOP;
                L.p = p;
                L.in = par(a, sp, Vh, 1 - p);
                L.out = par(b, sp, Vh, p);
                CHK(run_hop(c, L));
            }
            break;
        case WCL_OP_CLOVER:
        case WCL_OP_CLOVER_INV:
            for (int p = 0; p < 2; p++)
                CHK(run_clover(c, lp, sp, p, op == WCL_OP_CLOVER ? clov_for(c, lp) : clovinv_for(c, lp),
                               par(a, sp, Vh, p), par(b, sp, Vh, p)));
            break;
        case WCL_OP_SCHUR:
            CHK(schur(c, lp, sp, par(a, sp, Vh, 0), par(b, sp, Vh, 0), sp == P64 ? t64o : par(b, sp, Vh, 2), nullptr));
            HIPCHK(launch_zero(P64, 12 * Vh, par(b64, P64, Vh, 1), c->st));
            break;
        case WCL_OP_SCHUR_RHS:
            if (sp != P64) return fail(WCL_EINVAL, "SCHUR_RHS is an FP64 step");
            CHK(schur_rhs64(c, a64, par(b64, P64, Vh, 0), t64o, t64e));
            HIPCHK(launch_zero(P64, 12 * Vh, par(b64, P64, Vh, 1), c->st));
            break;
        case WCL_OP_RAS: {
            RasLaunch R{};
            R.g = &c->g;
            R.overlap = c->ras_overlap;
            R.iters = c->ras_iters;
            R.jacobi = c->ras_solver == WCL_RAS_JACOBI;
            R.link_prec = eff_lprec(c, lp);
            R.in = par(a, sp, Vh, 0);
            R.out = par(b, sp, Vh, 0);
            R.links = links_for(c, R.link_prec);
            R.links_site = c->U32s;
            R.clov_inv = clovinv_for(c, lp);
            R.kappa2 = (float)(c->kappa * c->kappa);
            R.sc = nullptr;
            R.nrhs = 1;
            R.stride = 0;
            if (c->ras_mult) {
                void *rt, *tt, *to;
                CHK(wsget(c, S_SAPR, half_bytes(sp, Vh), &rt));
                CHK(wsget(c, S_SAPT, half_bytes(sp, Vh), &tt));
                CHK(wsget(c, S_SAPO, half_bytes(sp, Vh), &to));
                CHK(run_sap(c, R, lp, sp, R.in, R.out, rt, tt, to));
            } else {
                CHK(run_ras(c, R));
            }
            HIPCHK(launch_zero(P64, 12 * Vh, par(b64, P64, Vh, 1), c->st));
            break;
        }
        case WCL_OP_D:
        case WCL_OP_DDAG:
            CHK(full_D(c, lp, sp, a, b, op == WCL_OP_DDAG));
            break;
        }
        if (sp != P64) {
            const bool even_only = (op == WCL_OP_SCHUR || op == WCL_OP_RAS);
            HIPCHK(launch_convert(sp, P64, (even_only ? 1 : 2) * Vh, Vh, Vh, b, b64, nullptr, 0, 1.0, c->st));
        }
        HIPCHK(launch_unpack_spinor(c->g, b64, outk, c->st));
    }
    return WCL_OK;
}

int wcl_apply(wcl_ctx *c, const double *in, double *out, int nrhs, int dagger, int prec)
{
    return wcl_apply_op(c, dagger ? WCL_OP_DDAG : WCL_OP_D, in, out, nrhs, prec);
}

// wcl_apply without allocation: the same kernels in the same order as
// wcl_apply (pack, precision cast, the two parity launches of D, cast back,
// unpack), with every temporary in this device's fixed scratch instead of
// the context's workspace, and no profiling events.  Layout of the scratch
// per call: [0, 384 Vh) the FP64 e/o input (both parities), then either the
// FP64 e/o output or, for prec 32/16, the cast input and output (192 Vh
// each at most); the cast-back output reuses the FP64 input region.
int wcl_apply_noalloc(wcl_ctx *c, const double *in, double *out, int nrhs, int dagger, int prec)
{
    if (!c || !in || !out) return fail(WCL_EINVAL, "null argument");
    if (!c->have_params) return fail(WCL_ESTATE, "operator used before wcl_set_gauge and wcl_set_params");
    CHK(check_prec(prec));
    if (nrhs < 1) return fail(WCL_EINVAL, "nrhs must be >= 1");
    if (c->device < 0 || c->device >= MAX_DEVICES || !g_scratch[c->device])
        return fail(WCL_ESTATE, "no scratch address for the context's device");
    const size_t Vh = c->Vh;
    const size_t need = NOALLOC_BYTES_PER_HALF_SITE * Vh;
    if (need > NOALLOC_SCRATCH_BYTES) {
        char msg[200];
        snprintf(msg, sizeof msg,
                 "wcl_apply_noalloc: this lattice needs %zu bytes of scratch; the fixed scratch holds %zu "
                 "(lattices of at most %zu sites)",
                 need, NOALLOC_SCRATCH_BYTES, 2 * (NOALLOC_SCRATCH_BYTES / NOALLOC_BYTES_PER_HALF_SITE));
        return fail(WCL_EINVAL, msg);
    }
    char *base = (char *)g_scratch[c->device];
    const int sp = prec;
    void *a64 = base;                                   // 2 x spinor_bytes(8, Vh) = 384 Vh
    void *b = base + 2 * spinor_bytes(8, Vh);           // FP64 output, or the cast input ...
    void *a = b;
    void *bs = (char *)b + 2 * spinor_bytes(prec_bytes(sp), Vh);   // ... and the cast output
    if (sp == P64) bs = b;
    for (int k = 0; k < nrhs; k++) {
        const double *ink = in + (size_t)k * c->V * 24;
        double *outk = out + (size_t)k * c->V * 24;
        HIPCHK(launch_pack_spinor(c->g, ink, a64, c->st));
        const void *src = a64;
        if (sp != P64) {
            HIPCHK(launch_convert(P64, sp, 2 * Vh, Vh, Vh, a64, a, nullptr, 0, 1.0, c->st));
            src = a;
        }
        for (int p = 0; p < 2; p++) {
            HopLaunch L = hop_base(c, prec, sp);
            L.mode = CLOVX;
            L.dagger = dagger ? 1 : 0;
            L.p = p;
            L.in = par(src, sp, Vh, 1 - p);
            L.x = par(src, sp, Vh, p);
            L.out = par(bs, sp, Vh, p);
            L.clov = clov_for(c, prec);
            L.coef = -c->kappa;
            L.in_stride = L.out_stride = L.x_stride = full_bytes(sp, Vh);
            HIPCHK(launch_hop(L, c->st));
        }
        if (sp != P64) {
            HIPCHK(launch_convert(sp, P64, 2 * Vh, Vh, Vh, bs, a64, nullptr, 0, 1.0, c->st));
            HIPCHK(launch_unpack_spinor(c->g, a64, outk, c->st));
        } else {
            HIPCHK(launch_unpack_spinor(c->g, bs, outk, c->st));
        }
    }
    return WCL_OK;
}

void wcl_default_opts(wcl_solve_opts *o)
{
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->tol = 1e-10;
    o->max_outer = 100;
    o->max_inner = 500;
    o->inner_tol = 1e-2;
    o->outer = WCL_OUTER_FBICGSTAB;
    o->use_ras = 1;
    o->ras_overlap = 1;
    o->ras_iters = 4;
    o->ras_solver = WCL_RAS_MR;
    o->inner_vec_prec = 32;
    o->ras_mult = 0;
    o->inner_prec = 32;
    o->use_graph = 0;
    o->check_every = 8;
}

}  // extern "C"

// ===========================================================================
// Solvers (all right-hand sides of a call advance in lockstep; every vector
// carries a right-hand-side dimension and every BiCGStab scalar is per rhs;
// a converged right-hand side is masked out of every kernel by its scalars).
namespace {

struct SolveWs {
    int n;
    // FP64 full fields [n][2][12][Vh]
    void *b, *x, *res;
    // FP64 even vectors [n][12][Vh]
    void *bh, *xe, *r, *rt, *p, *v, *s, *t, *ph, *sh, *o, *o2;
    // FP32 even vectors [n][6][Vh] float4
    void *rhs, *x32, *r32, *rt32, *p32, *v32, *s32, *t32, *ph32, *sh32, *o32;
    // multiplicative Schwarz temporaries (same storage; null unless used)
    void *sapr = nullptr, *sapt = nullptr, *sapo = nullptr;
};

int get_ws(wcl_ctx *c, SolveWs &w, bool inner, bool plain, int n)
{
    const size_t Vh = c->Vh;
    const size_t e64 = spinor_bytes(8, Vh) * n, e32 = spinor_bytes(4, Vh) * n;
    w.n = n;
    CHK(wsget(c, S_B64, 2 * e64, &w.b));
    CHK(wsget(c, S_X64, 2 * e64, &w.x));
    CHK(wsget(c, S_R64F, 2 * e64, &w.res));
    // plain FP64 BiCGStab works on full fields: its vectors are twice as long
    const size_t ev = plain ? 2 * e64 : e64;
    void **v64[] = {&w.bh, &w.xe, &w.r, &w.rt, &w.p, &w.v, &w.s, &w.t, &w.ph, &w.sh, &w.o, &w.o2};
    for (int k = 0; k < 12; k++) CHK(wsget(c, S_BH + k, ev, v64[k]));
    if (inner) {
        void **v32[] = {&w.rhs, &w.x32, &w.r32, &w.rt32, &w.p32, &w.v32, &w.s32, &w.t32, &w.ph32, &w.sh32, &w.o32};
        for (int k = 0; k < 11; k++) CHK(wsget(c, S_RHS32 + k, e32, v32[k]));
        if (c->ras_mult) {
            CHK(wsget(c, S_SAPR, e32, &w.sapr));
            CHK(wsget(c, S_SAPT, e32, &w.sapt));
            CHK(wsget(c, S_SAPO, e32, &w.sapo));
        }
    }
    return WCL_OK;
}

struct InnerCfg {
    int lprec;
    int vprec;                     // storage of the inner vectors (P32, or P16 with FP16 links)
    double tol;
    int maxit;
    bool ras;
    int check_every;
    bool graph;                    // replay the iteration as a captured hipGraph
    hipGraphExec_t *exec;          // the captured iteration (created on first use)
    hipStream_t cap_stream;        // private stream used only for the capture
    bool persistent;               // the whole inner solve as one cooperative launch
};

// One BiCGStab iteration (right preconditioned by RAS when enabled) on the
// FP32 Schur system for n right-hand sides, scalars sc[0, n) on the device.
int inner_iteration(wcl_ctx *c, const InnerCfg &cfg, SolveWs &w, Scalars *sc, int n)
{
    const size_t m = 12 * (size_t)c->Vh;   // complex numbers per right-hand side
    const int lp = cfg.lprec, vp = cfg.vprec;
    HIPCHK(launch_bicg_p(vp, m, w.r32, w.p32, w.v32, sc, c->st, n, m));
    void *ph = w.p32, *sh = w.s32;
    RasLaunch R{};
    if (cfg.ras) {
        R.g = &c->g;
        R.overlap = c->ras_overlap;
        R.iters = c->ras_iters;
        R.jacobi = c->ras_solver == WCL_RAS_JACOBI;
        R.link_prec = eff_lprec(c, lp);
        R.links = links_for(c, R.link_prec);
        R.links_site = c->U32s;
        R.clov_inv = clovinv_for(c, lp);
        R.kappa2 = (float)(c->kappa * c->kappa);
        R.sc = sc;
        R.nrhs = n;
        R.stride = half_bytes(vp, c->Vh);
        R.vec_prec = vp;
        R.in = w.p32;
        R.out = w.ph32;
        if (c->ras_mult) CHK(run_sap(c, R, lp, vp, w.p32, w.ph32, w.sapr, w.sapt, w.sapo));
        else CHK(run_ras(c, R));
        ph = w.ph32;
    }
    // the reductions ride in the Schur operator's second half and the x, r
    // update, except with several right-hand sides per thread
    const bool fused = c->hop_rhs == 1 || n == 1;
    int np = 0;
    if (fused) {
        CHK(schur_dot(c, lp, vp, ph, w.v32, w.o32, sc, n, 1, w.rt32, &np));
        HIPCHK(launch_finalize(BICG_ALPHA, 2, c->partials, sc, c->st, n, nullptr, c->pstride, np));
    } else {
        CHK(schur(c, lp, vp, ph, w.v32, w.o32, sc, n));
        const void *a[1] = {w.rt32}, *b[1] = {w.v32};
        HIPCHK(launch_dots(vp, m, 1, a, b, c->partials, sc, c->st, n, m, c->pstride));
        HIPCHK(launch_finalize(BICG_ALPHA, 2, c->partials, sc, c->st, n, nullptr, c->pstride));
    }
    HIPCHK(launch_bicg_s(vp, m, w.r32, w.v32, w.s32, sc, c->st, n, m));
    if (cfg.ras) {
        R.in = w.s32;
        R.out = w.sh32;
        if (c->ras_mult) CHK(run_sap(c, R, lp, vp, w.s32, w.sh32, w.sapr, w.sapt, w.sapo));
        else CHK(run_ras(c, R));
        sh = w.sh32;
    }
    if (fused) {
        CHK(schur_dot(c, lp, vp, sh, w.t32, w.o32, sc, n, 2, w.s32, &np));
        HIPCHK(launch_finalize(BICG_OMEGA, 4, c->partials, sc, c->st, n, nullptr, c->pstride, np));
        HIPCHK(launch_bicg_xr_dots(vp, m, w.x32, ph, sh, w.r32, w.s32, w.t32, w.rt32, sc, c->st, n, m, c->partials,
                                   c->pstride, &np));
        HIPCHK(launch_finalize(BICG_RHO, 4, c->partials, sc, c->st, n, nullptr, c->pstride, np));
    } else {
        CHK(schur(c, lp, vp, sh, w.t32, w.o32, sc, n));
        {
            const void *a[2] = {w.t32, w.t32}, *b[2] = {w.s32, w.t32};
            HIPCHK(launch_dots(vp, m, 2, a, b, c->partials, sc, c->st, n, m, c->pstride));
            HIPCHK(launch_finalize(BICG_OMEGA, 4, c->partials, sc, c->st, n, nullptr, c->pstride));
        }
        HIPCHK(launch_bicg_xr(vp, m, w.x32, ph, sh, w.r32, w.s32, w.t32, sc, c->st, n, m));
        {
            const void *a[2] = {w.rt32, w.r32}, *b[2] = {w.r32, w.r32};
            HIPCHK(launch_dots(vp, m, 2, a, b, c->partials, sc, c->st, n, m, c->pstride));
            HIPCHK(launch_finalize(BICG_RHO, 4, c->partials, sc, c->st, n, nullptr, c->pstride));
        }
    }
    return WCL_OK;
}

// out64_k = ||in64_k|| * K(in64_k / ||in64_k||) for every right-hand side k
// whose gate (per-rhs "final" flag) is not set: the single-precision inner
// solve, all right-hand sides in one set of launches.
int inner_solve(wcl_ctx *c, const InnerCfg &cfg, SolveWs &w, const void *in64, void *out64, int n,
                std::vector<int> &iters)
{
    const size_t m = 12 * (size_t)c->Vh;
    const size_t Vh = c->Vh;
    Scalars *sc = SI(c);
    const int sstride = (int)(sizeof(Scalars) / sizeof(double));
    CHK(norms_dev(c, P64, m, in64, m, n, sc));
    const int vp = cfg.vprec;
    HIPCHK(launch_convert(P64, vp, n * Vh, Vh, Vh, in64, w.r32, &sc->t[0], 1, 1.0, c->st, 1, sstride));
    HIPCHK(launch_copy(vp, n * m, w.r32, w.rt32, c->st));
    HIPCHK(launch_zero(vp, n * m, w.x32, c->st));
    HIPCHK(launch_zero(vp, n * m, w.p32, c->st));
    HIPCHK(launch_zero(vp, n * m, w.v32, c->st));
    {
        const void *a[2] = {w.rt32, w.r32}, *b[2] = {w.r32, w.r32};
        HIPCHK(launch_dots(vp, m, 2, a, b, c->partials, nullptr, c->st, n, m, c->pstride));
        HIPCHK(launch_finalize(BICG_INIT_RHO, 4, c->partials, sc, c->st, n, SF(c), c->pstride));
    }
    if (cfg.persistent) {
        // every iteration in one cooperative launch, then one read of the scalars
        void *part, *bar;
        CHK(wsget(c, S_PPART, sizeof(double) * PMAX_WG * PMAX_RHS * 4, &part));
        CHK(wsget(c, S_PBAR, 64, &bar));
        PersistLaunch P{};
        P.g = &c->g;
        P.link_prec = eff_lprec(c, cfg.lprec);
        P.vec_prec = vp;
        P.links = links_for(c, P.link_prec);
        P.links_site = c->U32s;
        P.clov_inv = clovinv_for(c, cfg.lprec);
        P.kappa2 = c->kappa * c->kappa;
        P.use_ras = cfg.ras ? 1 : 0;
        P.overlap = c->ras_overlap;
        P.iters = c->ras_iters;
        P.jacobi = c->ras_solver == WCL_RAS_JACOBI;
        P.x = w.x32; P.r = w.r32; P.rt = w.rt32; P.p = w.p32; P.v = w.v32; P.s = w.s32; P.t = w.t32;
        P.ph = w.ph32; P.sh = w.sh32; P.o = w.o32;
        P.stride = half_bytes(vp, Vh);
        P.sc = sc;
        P.partials = (double *)part;
        P.bar = (unsigned *)bar;
        P.err = (int *)((char *)bar + 32);
        P.nrhs = n;
        P.maxit = cfg.maxit;
        P.num_cus = c->num_cus;
        const size_t rec = c->recs.size();
        CHK(profiled(c, WCL_K_INNER, 0.0, 0.0, [&] { return launch_persist(P, c->st); }));
        CHK(read_sc(c, HI(c), sc, n));   // synchronises the stream
        int err = 0;
        HIPCHK(hipMemcpy(&err, P.err, sizeof(int), hipMemcpyDeviceToHost));
        if (err) return fail(WCL_EHIP, "persistent inner solve: a grid barrier wait exceeded its bound");
        for (int k = 0; k < n; k++) iters[k] = HI(c)[k].iter;
        if (c->prof && rec < c->recs.size()) {
            // algorithmic work of the iterations run: per iteration and
            // right-hand side two Schur applications (two hop launches each),
            // two Schwarz applications and the vector updates and reductions
            double b = 0, f = 0;
            for (int k = 0; k < n; k++) {
                const int it = iters[k];
                if (it <= 0) continue;
                HopLaunch L = hop_base(c, cfg.lprec, vp);
                L.mode = CLOV_H;
                double hb, hf;
                hop_work(L, &hb, &hf);
                b += 2.0 * it * hb; f += 2.0 * it * hf;
                L.mode = XPAY;
                hop_work(L, &hb, &hf);
                b += 2.0 * it * hb; f += 2.0 * it * hf;
                if (cfg.ras) {
                    RasLaunch R{};
                    R.g = &c->g; R.overlap = c->ras_overlap; R.iters = c->ras_iters; R.jacobi = false;
                    R.link_prec = P.link_prec; R.nrhs = 1; R.vec_prec = vp;
                    double rb, rf;
                    ras_work(R, &rb, &rf);
                    b += 2.0 * it * rb; f += 2.0 * it * rf;
                }
                // p update (4 vector passes), s update (3), x / r update with dots (8), 96 flop
                // per complex number and update or dot on 12 complex numbers per site
                b += it * 15.0 * half_bytes(vp, Vh);
                f += it * (double)Vh * 12.0 * (8.0 + 6.0 + 16.0 + 3 * 8.0);
            }
            c->recs[rec].bytes = b;
            c->recs[rec].flops = f;
        }
        HIPCHK(launch_convert(vp, P64, n * Vh, Vh, Vh, w.x32, out64, &sc->t[0], 2, 1.0, c->st, 1, sstride));
        return WCL_OK;
    }
    // Iterations are queued in chunks; every kernel of an iteration queued
    // after a right-hand side converged is a no-op for it.  The chunk length
    // follows the observed convergence rate of the slowest right-hand side.
    int launched = 0;
    int chunk = std::min(cfg.check_every, 4);
    std::vector<double> r2_prev(n, 1.0);
    std::vector<int> it_prev(n, 0);
    std::vector<size_t> rec_mark;  // profile records at the start of each queued iteration
    Scalars *h = HI(c);
    while (launched < cfg.maxit) {
        chunk = std::max(1, std::min(chunk, cfg.maxit - launched));
        if (cfg.graph && !*cfg.exec) {
            // capture one iteration (kernel launches only, no memset or copy
            // nodes); the buffers and scalars it touches are fixed for the solve
            const bool prof = c->prof;
            hipStream_t st = c->st;
            c->prof = false;
            c->st = cfg.cap_stream;
            hipGraph_t graph = nullptr;
            HIPCHK(hipStreamBeginCapture(cfg.cap_stream, hipStreamCaptureModeThreadLocal));
            const int rc = inner_iteration(c, cfg, w, sc, n);
            const hipError_t ec = hipStreamEndCapture(cfg.cap_stream, &graph);
            c->st = st;
            c->prof = prof;
            if (rc != WCL_OK) return rc;
            HIPCHK(ec);
            HIPCHK(hipGraphInstantiate(cfg.exec, graph, nullptr, nullptr, 0));
            (void)hipGraphDestroy(graph);
        }
        for (int k = 0; k < chunk; k++) {
            rec_mark.push_back(c->recs.size());
            if (cfg.graph) HIPCHK(hipGraphLaunch(*cfg.exec, c->st));
            else CHK(inner_iteration(c, cfg, w, sc, n));
        }
        launched += chunk;
        CHK(read_sc(c, h, sc, n));
        bool all = true;
        double need_max = 0.0;
        for (int k = 0; k < n; k++) {
            if (h[k].done) continue;
            all = false;
            const int di = h[k].iter - it_prev[k];
            double need = 4.0;
            if (di > 0 && h[k].r2 > 0.0 && h[k].r2 < r2_prev[k]) {
                const double rate = std::log(h[k].r2 / r2_prev[k]) / di;
                need = std::log(h[k].stop2 * h[k].b2 / h[k].r2) / rate;
            }
            need_max = std::max(need_max, need);
            r2_prev[k] = h[k].r2;
            it_prev[k] = h[k].iter;
        }
        if (all) break;
        chunk = (int)std::min(16.0, std::max(1.0, std::floor(need_max)));
    }
    int max_it = 0;
    for (int k = 0; k < n; k++) {
        iters[k] = h[k].iter;
        max_it = std::max(max_it, h[k].iter);
    }
    // work of launches after every right-hand side had converged is void
    // (with several right-hand sides the per-rhs masking is not separated)
    for (size_t q = (size_t)max_it; q < rec_mark.size(); q++) {
        const size_t end = (q + 1 < rec_mark.size()) ? rec_mark[q + 1] : c->recs.size();
        for (size_t r = rec_mark[q]; r < end; r++) c->recs[r].bytes = c->recs[r].flops = 0.0;
    }
    HIPCHK(launch_convert(vp, P64, n * Vh, Vh, Vh, w.x32, out64, &sc->t[0], 2, 1.0, c->st, 1, sstride));
    return WCL_OK;
}

// true relative residuals of the full systems: ||b_k - D x_k|| / ||b_k|| (FP64)
int true_residuals(wcl_ctx *c, SolveWs &w, const std::vector<double> &bnorm2, std::vector<double> &rel)
{
    const size_t mf = 24 * (size_t)c->Vh;
    const int n = w.n;
    CHK(full_D(c, P64, P64, w.x, w.res, 0, nullptr, n));
    HIPCHK(launch_axpby(P64, n * mf, make_double2(1.0, 0.0), w.b, make_double2(-1.0, 0.0), w.res, c->st));
    std::vector<double> r2(n);
    CHK(norms_host(c, P64, mf, w.res, mf, n, r2.data()));
    for (int k = 0; k < n; k++) rel[k] = bnorm2[k] > 0.0 ? std::sqrt(r2[k] / bnorm2[k]) : 0.0;
    return WCL_OK;
}

// set the "final" flags (gate of the inner solve and mask of the outer)
int write_final(wcl_ctx *c, const std::vector<int> &final_)
{
    for (int k = 0; k < (int)final_.size(); k++) HF(c)[k].done = final_[k];
    CHK(write_sc(c, SF(c), HF(c), (int)final_.size()));
    return WCL_OK;
}

// Generic BiCGStab driver for n right-hand sides in FP64 (right
// preconditioned by K when given):
//   PLAIN    : A = full D on full fields, no K, x = w.x, rhs = w.b
//   PLAIN_EO : A = Dhat on even vectors, no K, x = w.xe, rhs = w.bh
//   FLEX     : A = Dhat on even vectors, K = inner solve, x = w.xe, rhs = w.bh
// Stops a right-hand side when its true residual of the full system is
// <= tol; a right-hand side whose recursive residual reached the threshold
// (or broke down) without a true residual <= tol gets its residual replaced
// by the true one and its recurrence restarted.
struct Driver {
    bool eo;        // A = Dhat on even vectors (else the full D)
    bool flex;      // right preconditioned by the inner solve
    size_t m;       // complex numbers per right-hand side
    void *x, *bvec;
    bool warm;      // w.x holds the initial guess (full fields), else zero start
};

int apply_A(wcl_ctx *c, const Driver &d, SolveWs &w, const void *in, void *out, const Scalars *sc)
{
    if (d.eo) return schur(c, P64, P64, in, out, w.o, sc, w.n);
    return full_D(c, P64, P64, in, out, 0, sc, w.n);
}

// true residuals; for FLEX the full solution is reconstructed first
int check_true(wcl_ctx *c, const Driver &d, SolveWs &w, const std::vector<double> &bnorm2, std::vector<double> &rel)
{
    if (d.eo) {
        HIPCHK(launch_zero(P64, w.n * 24 * (size_t)c->Vh, w.x, c->st));
        // copy x_e into the even halves of the full fields
        for (int k = 0; k < w.n; k++)
            HIPCHK(hipMemcpyAsync((char *)w.x + k * full_bytes(P64, c->Vh), (char *)w.xe + k * half_bytes(P64, c->Vh),
                                  half_bytes(P64, c->Vh), hipMemcpyDeviceToDevice, c->st));
        CHK(reconstruct64(c, w.b, w.x, w.o, w.n));
    }
    return true_residuals(c, w, bnorm2, rel);
}

// (re)start the recurrence of right-hand side k (or all with k < 0) from r
int restart(wcl_ctx *c, const Driver &d, SolveWs &w, int k, double tol, const std::vector<double> &bnorm2)
{
    const int n = w.n;
    const int k0 = k < 0 ? 0 : k, cnt = k < 0 ? n : 1;
    const size_t off = (size_t)k0 * d.m * 16;
    HIPCHK(launch_copy(P64, cnt * d.m, (char *)w.r + off, (char *)w.rt + off, c->st));
    HIPCHK(launch_zero(P64, cnt * d.m, (char *)w.p + off, c->st));
    HIPCHK(launch_zero(P64, cnt * d.m, (char *)w.v + off, c->st));
    const void *a[2] = {(char *)w.rt + off, (char *)w.r + off}, *b[2] = {(char *)w.r + off, (char *)w.r + off};
    HIPCHK(launch_dots(P64, d.m, 2, a, b, c->partials, nullptr, c->st, cnt, d.m, c->pstride));
    HIPCHK(launch_finalize(BICG_INIT_RHO, 4, c->partials, SO(c) + k0, c->st, cnt, SF(c) + k0, c->pstride));
    CHK(read_sc(c, HO(c) + k0, SO(c) + k0, cnt));
    for (int j = k0; j < k0 + cnt; j++) {
        Scalars &h = HO(c)[j];
        // stop when |r|^2 <= tol^2 |b|^2 (b2 holds |r0|^2 after the init)
        h.stop2 = h.b2 > 0.0 ? tol * tol * bnorm2[j] / h.b2 : 0.0;
    }
    CHK(write_sc(c, SO(c) + k0, HO(c) + k0, cnt));
    return WCL_OK;
}

// Initial iterate and residual r = bvec - A x of a driver.  Zero start: x = 0,
// r = bvec.  Warm start: x = the guess held in the full fields w.x (its even
// halves for the even/odd systems); a right-hand side whose guess already
// meets the tolerance (true residual of the full system) is final at once.
int initial_residual(wcl_ctx *c, const Driver &d, const wcl_solve_opts &o, SolveWs &w,
                     const std::vector<double> &bnorm2, std::vector<int> &final_, std::vector<wcl_solve_info> &info)
{
    const int n = w.n;
    const size_t m = d.m;
    if (!d.warm) {
        HIPCHK(launch_copy(P64, n * m, d.bvec, w.r, c->st));
        HIPCHK(launch_zero(P64, n * m, d.x, c->st));
        return WCL_OK;
    }
    if (d.eo) {
        for (int k = 0; k < n; k++)
            HIPCHK(hipMemcpyAsync((char *)d.x + k * half_bytes(P64, c->Vh), (char *)w.x + k * full_bytes(P64, c->Vh),
                                  half_bytes(P64, c->Vh), hipMemcpyDeviceToDevice, c->st));
    }
    std::vector<double> rel(n, 0.0);
    CHK(check_true(c, d, w, bnorm2, rel));
    for (int k = 0; k < n; k++) {
        if (final_[k]) continue;
        info[k].true_relres = rel[k];
        if (rel[k] <= o.tol) { final_[k] = 1; info[k].status = WCL_OK; }
    }
    CHK(apply_A(c, d, w, d.x, w.t, nullptr));
    HIPCHK(launch_copy(P64, n * m, d.bvec, w.r, c->st));
    HIPCHK(launch_axpby(P64, n * m, make_double2(-1.0, 0.0), w.t, make_double2(1.0, 0.0), w.r, c->st));
    return WCL_OK;
}

int bicgstab_driver(wcl_ctx *c, const Driver &d, const wcl_solve_opts &o, const InnerCfg *cfg, SolveWs &w,
                    const std::vector<double> &bnorm2, std::vector<int> &final_, std::vector<wcl_solve_info> &info)
{
    const int n = w.n;
    const size_t m = d.m;
    Scalars *sc = SO(c);
    CHK(initial_residual(c, d, o, w, bnorm2, final_, info));
    CHK(write_final(c, final_));
    CHK(restart(c, d, w, -1, o.tol, bnorm2));
    for (int k = 0; k < n; k++)
        if (!final_[k] && HO(c)[k].b2 == 0.0) { final_[k] = 1; info[k].status = WCL_OK; }
    std::vector<int> it_inner(n, 0);
    std::vector<int> restarts(n, 0);
    std::vector<int> broke(n, 0);   // the last stop of the recurrence was a breakdown
    for (int k = 0; k < n; k++) info[k].outer_iters = 0;
    int iter = 0;
    const int every = d.flex ? 1 : std::max(1, o.check_every);
    while (iter < o.max_outer) {
        bool any_active = false;
        for (int k = 0; k < n; k++) any_active = any_active || !final_[k];
        if (!any_active) break;
        const int chunk = std::min(every, o.max_outer - iter);
        std::vector<size_t> rec_mark;
        for (int q = 0; q < chunk; q++) {
            rec_mark.push_back(c->recs.size());
            HIPCHK(launch_bicg_p(P64, m, w.r, w.p, w.v, sc, c->st, n, m));
            void *ph = w.p, *sh = w.s;
            if (d.flex) {
                CHK(inner_solve(c, *cfg, w, w.p, w.ph, n, it_inner));
                for (int k = 0; k < n; k++) info[k].inner_iters_total += final_[k] ? 0 : it_inner[k];
                ph = w.ph;
            }
            // on the even/odd system the reductions ride in the Schur operator's
            // second half and the x/r update, as in the inner solver
            const bool fused = d.eo && (c->hop_rhs == 1 || n == 1);
            int np = 0;
            if (fused) {
                CHK(schur_dot(c, P64, P64, ph, w.v, w.o, sc, n, 1, w.rt, &np));
                HIPCHK(launch_finalize(BICG_ALPHA, 2, c->partials, sc, c->st, n, nullptr, c->pstride, np));
            } else {
                CHK(apply_A(c, d, w, ph, w.v, sc));
                const void *a[1] = {w.rt}, *b[1] = {w.v};
                HIPCHK(launch_dots(P64, m, 1, a, b, c->partials, sc, c->st, n, m, c->pstride));
                HIPCHK(launch_finalize(BICG_ALPHA, 2, c->partials, sc, c->st, n, nullptr, c->pstride));
            }
            HIPCHK(launch_bicg_s(P64, m, w.r, w.v, w.s, sc, c->st, n, m));
            if (d.flex) {
                CHK(inner_solve(c, *cfg, w, w.s, w.sh, n, it_inner));
                for (int k = 0; k < n; k++) info[k].inner_iters_total += final_[k] ? 0 : it_inner[k];
                sh = w.sh;
            }
            if (fused) {
                CHK(schur_dot(c, P64, P64, sh, w.t, w.o, sc, n, 2, w.s, &np));
                HIPCHK(launch_finalize(BICG_OMEGA, 4, c->partials, sc, c->st, n, nullptr, c->pstride, np));
                HIPCHK(launch_bicg_xr_dots(P64, m, d.x, ph, sh, w.r, w.s, w.t, w.rt, sc, c->st, n, m, c->partials,
                                           c->pstride, &np));
                HIPCHK(launch_finalize(BICG_RHO, 4, c->partials, sc, c->st, n, nullptr, c->pstride, np));
            } else {
                CHK(apply_A(c, d, w, sh, w.t, sc));
                {
                    const void *a[2] = {w.t, w.t}, *b[2] = {w.s, w.t};
                    HIPCHK(launch_dots(P64, m, 2, a, b, c->partials, sc, c->st, n, m, c->pstride));
                    HIPCHK(launch_finalize(BICG_OMEGA, 4, c->partials, sc, c->st, n, nullptr, c->pstride));
                }
                HIPCHK(launch_bicg_xr(P64, m, d.x, ph, sh, w.r, w.s, w.t, sc, c->st, n, m));
                {
                    const void *a[2] = {w.rt, w.r}, *b[2] = {w.r, w.r};
                    HIPCHK(launch_dots(P64, m, 2, a, b, c->partials, sc, c->st, n, m, c->pstride));
                    HIPCHK(launch_finalize(BICG_RHO, 4, c->partials, sc, c->st, n, nullptr, c->pstride));
                }
            }
        }
        iter += chunk;
        CHK(read_sc(c, HO(c), sc, n));
        bool candidates = false;
        int exec = 0;  // iterations of this chunk that did work for some right-hand side
        for (int k = 0; k < n; k++) {
            if (final_[k]) continue;
            exec = std::max(exec, HO(c)[k].iter - info[k].outer_iters);
            info[k].outer_iters = HO(c)[k].iter;
            if (!std::isfinite(HO(c)[k].r2)) { final_[k] = 1; info[k].status = WCL_ENAN; continue; }
            broke[k] = HO(c)[k].done == 2;
            if (HO(c)[k].done) candidates = true;
        }
        for (size_t q = (size_t)std::max(exec, 0); q < rec_mark.size(); q++) {  // queued after convergence
            const size_t end = (q + 1 < rec_mark.size()) ? rec_mark[q + 1] : c->recs.size();
            for (size_t r = rec_mark[q]; r < end; r++) c->recs[r].bytes = c->recs[r].flops = 0.0;
        }
        if (!candidates) continue;
        std::vector<double> rel(n, 0.0);
        CHK(check_true(c, d, w, bnorm2, rel));
        bool any_restart = false;
        for (int k = 0; k < n; k++) {
            if (final_[k] || !HO(c)[k].done) continue;
            info[k].true_relres = rel[k];
            if (rel[k] <= o.tol) { final_[k] = 1; info[k].status = WCL_OK; continue; }
            if (restarts[k] >= 8) { final_[k] = 1; info[k].status = broke[k] ? WCL_EBREAKDOWN : WCL_ENOCONV; continue; }
            restarts[k]++;
            any_restart = true;
        }
        CHK(write_final(c, final_));
        if (any_restart) {
            // residual replacement: r = b - A x for the restarted right-hand sides
            CHK(apply_A(c, d, w, d.x, w.t, nullptr));
            for (int k = 0; k < n; k++) {
                if (final_[k] || !HO(c)[k].done) continue;
                const size_t off = (size_t)k * m * 16;
                HIPCHK(launch_copy(P64, m, (char *)d.bvec + off, (char *)w.r + off, c->st));
                HIPCHK(launch_axpby(P64, m, make_double2(-1.0, 0.0), (char *)w.t + off, make_double2(1.0, 0.0),
                                    (char *)w.r + off, c->st));
                const int it_done = HO(c)[k].iter;
                CHK(restart(c, d, w, k, o.tol, bnorm2));
                HO(c)[k].iter = it_done;  // keep counting this right-hand side's iterations
                CHK(write_sc(c, SO(c) + k, HO(c) + k, 1));
            }
        }
    }
    // out of iterations: a recurrence that ended in a breakdown reports it
    for (int k = 0; k < n; k++)
        if (!final_[k]) info[k].status = broke[k] ? WCL_EBREAKDOWN : WCL_ENOCONV;
    return WCL_OK;
}

// Defect correction: x_e += K(r), r = bhat - Dhat x_e in FP64, per right-hand side.
int outer_dc(wcl_ctx *c, const wcl_solve_opts &o, const InnerCfg &cfg, SolveWs &w, const std::vector<double> &bnorm2,
             std::vector<int> &final_, std::vector<wcl_solve_info> &info)
{
    const int n = w.n;
    const size_t m = 12 * (size_t)c->Vh;
    std::vector<int> it(n, 0);
    Driver d{true, true, m, w.xe, w.bh, o.x0_dev != nullptr};
    CHK(initial_residual(c, d, o, w, bnorm2, final_, info));
    for (int outer = 0; outer < o.max_outer; outer++) {
        bool any_active = false;
        for (int k = 0; k < n; k++) any_active = any_active || !final_[k];
        if (!any_active) break;
        CHK(write_final(c, final_));
        CHK(inner_solve(c, cfg, w, w.r, w.ph, n, it));
        for (int k = 0; k < n; k++)
            if (!final_[k]) { info[k].inner_iters_total += it[k]; info[k].outer_iters++; }
        // final right-hand sides got K = 0 from the gated inner solve
        HIPCHK(launch_axpby(P64, n * m, make_double2(1.0, 0.0), w.ph, make_double2(1.0, 0.0), w.xe, c->st));
        CHK(schur(c, P64, P64, w.xe, w.r, w.o, nullptr, n));
        HIPCHK(launch_axpby(P64, n * m, make_double2(1.0, 0.0), w.bh, make_double2(-1.0, 0.0), w.r, c->st));
        std::vector<double> r2(n);
        CHK(norms_host(c, P64, m, w.r, m, n, r2.data()));
        bool check = false;
        for (int k = 0; k < n; k++) {
            if (final_[k]) continue;
            if (!std::isfinite(r2[k])) { final_[k] = 1; info[k].status = WCL_ENAN; continue; }
            if (r2[k] <= o.tol * o.tol * bnorm2[k]) check = true;
        }
        if (!check) continue;
        std::vector<double> rel(n, 0.0);
        CHK(check_true(c, d, w, bnorm2, rel));
        for (int k = 0; k < n; k++) {
            if (final_[k]) continue;
            info[k].true_relres = rel[k];
            if (rel[k] <= o.tol) { final_[k] = 1; info[k].status = WCL_OK; }
        }
    }
    for (int k = 0; k < n; k++)
        if (!final_[k]) info[k].status = WCL_ENOCONV;
    return WCL_OK;
}

}  // namespace

extern "C" int wcl_solve(wcl_ctx *c, const double *b, double *x, int nrhs, const wcl_solve_opts *opts,
                         wcl_solve_info *infos)
{
    if (!c || !b || !x) return fail(WCL_EINVAL, "null argument");
    if (!c->have_params) return fail(WCL_ESTATE, "wcl_solve before wcl_set_gauge and wcl_set_params");
    if (nrhs < 1) return fail(WCL_EINVAL, "nrhs must be >= 1");
    wcl_solve_opts o;
    if (opts) o = *opts;
    else wcl_default_opts(&o);
    if (!(o.tol > 0) || o.max_outer < 1 || o.max_inner < 1 || !(o.inner_tol > 0))
        return fail(WCL_EINVAL, "tol, inner_tol > 0 and iteration limits >= 1 required");
    if (o.outer < 0 || o.outer > WCL_OUTER_PLAIN64_EO) return fail(WCL_EINVAL, "unknown outer solver");
    if (o.inner_prec != 32 && o.inner_prec != 16) return fail(WCL_EINVAL, "inner_prec must be 32 or 16");
    if (o.inner_vec_prec != 32 && o.inner_vec_prec != 16) return fail(WCL_EINVAL, "inner_vec_prec must be 32 or 16");
    if (o.inner_vec_prec == 16 && o.inner_prec != 16)
        return fail(WCL_EINVAL, "FP16 inner vectors need the FP16 links and clover (inner_prec 16)");
    if (o.check_every < 1) o.check_every = 8;
    if (o.persistent) {
        if (o.outer != WCL_OUTER_FBICGSTAB && o.outer != WCL_OUTER_DC)
            return fail(WCL_EINVAL, "the persistent inner solve belongs to the FBICGSTAB and DC solvers");
        if (o.use_graph) return fail(WCL_EINVAL, "persistent and use_graph are exclusive");
        if (nrhs > PMAX_RHS) return fail(WCL_EINVAL, "the persistent inner solve takes at most 16 right-hand sides");
    }
    const bool plain = o.outer == WCL_OUTER_PLAIN64;
    const bool plain_eo = o.outer == WCL_OUTER_PLAIN64_EO;
    const bool inner = !plain && !plain_eo;
    if (o.use_ras && inner) {
        CHK(wcl_set_ras(c, o.ras_overlap, o.ras_iters, o.ras_solver, o.ras_mult));
        if (o.ras_block[0] || o.ras_block[1] || o.ras_block[2] || o.ras_block[3]) CHK(wcl_set_ras_cores(c, o.ras_block));
    }
    if (o.persistent && o.use_ras && (ras_generic(c) || c->ras_mult || c->ras_solver != WCL_RAS_MR))
        return fail(WCL_EINVAL, "the persistent inner solve runs the additive Schwarz with minimal-residual "
                                "blocks of the fused kernel (tile cores, at most 648 sites per parity)");
    const int n = nrhs;
    CHK(ensure_batch(c, n));
    SolveWs w;
    CHK(get_ws(c, w, inner, plain, n));
    hipGraphExec_t graph_exec = nullptr;
    hipStream_t cap_stream = nullptr;
    if (o.use_graph && inner) HIPCHK(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
    struct GraphGuard {
        hipGraphExec_t *e;
        hipStream_t *s;
        ~GraphGuard()
        {
            if (*e) (void)hipGraphExecDestroy(*e);
            if (*s) (void)hipStreamDestroy(*s);
        }
    } guard{&graph_exec, &cap_stream};
    InnerCfg cfg{o.inner_prec, o.inner_vec_prec, o.inner_tol, o.max_inner, o.use_ras != 0, o.check_every,
                 o.use_graph != 0 && inner, &graph_exec, cap_stream, o.persistent != 0 && inner};
    // the inner stopping threshold is fixed for the whole solve
    for (int k = 0; k < n; k++) {
        HI(c)[k] = Scalars{};
        HI(c)[k].stop2 = o.inner_tol * o.inner_tol;
    }
    CHK(write_sc(c, SI(c), HI(c), n));
    HIPCHK(hipStreamSynchronize(c->st));
    const auto t0 = std::chrono::steady_clock::now();
    const size_t fb = full_bytes(P64, c->Vh);
    for (int k = 0; k < n; k++)
        HIPCHK(launch_pack_spinor(c->g, b + (size_t)k * c->V * 24, (char *)w.b + k * fb, c->st));
    if (o.adjoint) HIPCHK(launch_gamma5(2 * (size_t)n, c->Vh, w.b, c->st));  // D^dag = g5 D g5
    // initial guess (may alias x): the solve of D x' = g5 b starts from g5 x0
    // when adjoint
    const bool warm = o.x0_dev != nullptr;
    if (warm) {
        for (int k = 0; k < n; k++)
            HIPCHK(launch_pack_spinor(c->g, o.x0_dev + (size_t)k * c->V * 24, (char *)w.x + k * fb, c->st));
        if (o.adjoint) HIPCHK(launch_gamma5(2 * (size_t)n, c->Vh, w.x, c->st));
    }
    std::vector<double> bnorm2(n);
    CHK(norms_host(c, P64, 24 * (size_t)c->Vh, w.b, 24 * (size_t)c->Vh, n, bnorm2.data()));
    std::vector<wcl_solve_info> info(n);
    std::vector<int> final_(n, 0);
    for (int k = 0; k < n; k++) {
        memset(&info[k], 0, sizeof(wcl_solve_info));
        if (!std::isfinite(bnorm2[k])) { final_[k] = 1; info[k].status = WCL_ENAN; }
        else if (bnorm2[k] == 0.0) { final_[k] = 1; info[k].status = WCL_OK; }
    }
    if (plain) {
        Driver d{false, false, 24 * (size_t)c->Vh, w.x, w.b, warm};
        CHK(bicgstab_driver(c, d, o, nullptr, w, bnorm2, final_, info));
    } else {
        CHK(schur_rhs64(c, w.b, w.bh, w.o, w.s, n));
        if (plain_eo) {
            Driver d{true, false, 12 * (size_t)c->Vh, w.xe, w.bh, warm};
            CHK(bicgstab_driver(c, d, o, nullptr, w, bnorm2, final_, info));
        } else if (o.outer == WCL_OUTER_FBICGSTAB) {
            Driver d{true, true, 12 * (size_t)c->Vh, w.xe, w.bh, warm};
            CHK(bicgstab_driver(c, d, o, &cfg, w, bnorm2, final_, info));
        } else {
            CHK(outer_dc(c, o, cfg, w, bnorm2, final_, info));
        }
        HIPCHK(launch_zero(P64, n * 24 * (size_t)c->Vh, w.x, c->st));
        for (int k = 0; k < n; k++)
            HIPCHK(hipMemcpyAsync((char *)w.x + k * fb, (char *)w.xe + k * half_bytes(P64, c->Vh),
                                  half_bytes(P64, c->Vh), hipMemcpyDeviceToDevice, c->st));
        CHK(reconstruct64(c, w.b, w.x, w.o, n));
    }
    // NaN right-hand sides return x = 0
    for (int k = 0; k < n; k++)
        if (info[k].status == WCL_ENAN || bnorm2[k] == 0.0)
            HIPCHK(launch_zero(P64, 24 * (size_t)c->Vh, (char *)w.x + k * fb, c->st));
    std::vector<double> rel(n, 0.0);
    CHK(true_residuals(c, w, bnorm2, rel));
    for (int k = 0; k < n; k++) {
        if (info[k].status == WCL_ENAN || bnorm2[k] == 0.0) continue;
        info[k].true_relres = rel[k];
        if (!std::isfinite(rel[k])) info[k].status = WCL_ENAN;
        else if (info[k].status == WCL_OK && rel[k] > o.tol) info[k].status = WCL_ENOCONV;
    }
    if (o.adjoint) HIPCHK(launch_gamma5(2 * (size_t)n, c->Vh, w.x, c->st));
    for (int k = 0; k < n; k++)
        HIPCHK(launch_unpack_spinor(c->g, (char *)w.x + k * fb, x + (size_t)k * c->V * 24, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    int worst = WCL_OK;
    for (int k = 0; k < n; k++) {
        info[k].seconds = secs;
        if (infos) infos[k] = info[k];
        // worst status: NaN, then breakdown, then no convergence
        const int rank_new = info[k].status == WCL_ENAN ? 3 : info[k].status == WCL_EBREAKDOWN ? 2
                             : info[k].status != WCL_OK ? 1 : 0;
        const int rank_old = worst == WCL_ENAN ? 3 : worst == WCL_EBREAKDOWN ? 2 : worst != WCL_OK ? 1 : 0;
        if (rank_new > rank_old) worst = info[k].status;
    }
    if (worst != WCL_OK) {
        const char *what = worst == WCL_ENOCONV ? "solver did not reach the tolerance"
                           : worst == WCL_EBREAKDOWN ? "BiCGStab breakdown"
                                                     : "NaN or Inf in the data";
        return fail(worst, what);
    }
    return WCL_OK;
}

// ===========================================================================
namespace {
// Mean event time of `reps` launches (after 10 warm-ups) rotating over copies.
template <typename F>
int time_launches(wcl_ctx *c, int reps, int copies, F launch, double *ms)
{
    for (int i = 0; i < 10; i++) CHK(launch(i % copies));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, c->st));
    for (int i = 0; i < reps; i++) CHK(launch(i % copies));
    HIPCHK(hipEventRecord(e1, c->st));
    HIPCHK(hipEventSynchronize(e1));
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = (double)t / reps;
    return WCL_OK;
}

int bench_args(wcl_ctx *c, int prec, int reps, int copies, const double *ms, bool need_params, const char *what)
{
    if (!c || !ms) return fail(WCL_EINVAL, "null argument");
    if (!(need_params ? c->have_params : c->have_gauge))
        return fail(WCL_ESTATE, std::string(what) + (need_params ? " before wcl_set_params" : " before wcl_set_gauge"));
    if (prec != 32 && prec != 16) return fail(WCL_EINVAL, "bench prec must be 32 or 16");
    if (reps < 1 || copies < 1 || copies > 32) return fail(WCL_EINVAL, "reps >= 1 and 1 <= copies <= 32 required");
    return WCL_OK;
}
}  // namespace

extern "C" int wcl_bench_hop(wcl_ctx *c, int prec, int nrhs, int reps, int copies, double *ms)
{
    CHK(bench_args(c, prec, reps, copies, ms, false, "wcl_bench_hop"));
    if (nrhs < 1 || nrhs > 64) return fail(WCL_EINVAL, "wcl_bench_hop: 1 <= nrhs <= 64 required");
    const size_t Vh = c->Vh;
    const int lb = prec_bytes(prec), ep = eff_lprec(c, prec);
    const size_t lbytes = ep == prec ? link_bytes(lb, Vh) : link_bytes_c(ep, Vh), sbytes = spinor_bytes(4, Vh);
    std::vector<void *> lk(copies), in(copies), out(copies);
    for (int k = 0; k < copies; k++) {
        if (k == 0) lk[k] = links_for(c, ep);
        else {
            CHK(wsget(c, S_BENCH + 3 * k, lbytes, &lk[k]));
            HIPCHK(hipMemcpyAsync(lk[k], lk[0], lbytes, hipMemcpyDeviceToDevice, c->st));
        }
        CHK(wsget(c, S_BENCH + 3 * k + 1, sbytes * nrhs, &in[k]));
        CHK(wsget(c, S_BENCH + 3 * k + 2, sbytes * nrhs, &out[k]));
        // deterministic, non-trivial input: copy the FP32 links' first reals
        for (int r = 0; r < nrhs; r++)
            HIPCHK(hipMemcpyAsync((char *)in[k] + r * sbytes, (const char *)c->U32 + r * 64, sbytes,
                                  hipMemcpyDeviceToDevice, c->st));
    }
    return time_launches(c, reps, copies, [&](int k) -> int {
        HopLaunch L = hop_base(c, prec, P32);
        L.links = lk[k];
        L.mode = HOP;
        L.p = 0;
        L.in = in[k];
        L.out = out[k];
        L.nrhs = nrhs;
        L.in_stride = L.out_stride = sbytes;
        HIPCHK(launch_hop(L, c->st));
        return WCL_OK;
    }, ms);
}

extern "C" int wcl_bench_clover(wcl_ctx *c, int prec, int reps, int copies, double *ms)
{
    CHK(bench_args(c, prec, reps, copies, ms, true, "wcl_bench_clover"));
    const size_t Vh = c->Vh;
    const size_t cbytes = clover_bytes(prec_bytes(prec), Vh), sbytes = spinor_bytes(4, Vh);
    std::vector<void *> cl(copies), in(copies), out(copies);
    for (int k = 0; k < copies; k++) {
        if (k == 0) cl[k] = clovinv_for(c, prec);
        else {
            CHK(wsget(c, S_BENCH + 3 * k, cbytes, &cl[k]));
            HIPCHK(hipMemcpyAsync(cl[k], cl[0], cbytes, hipMemcpyDeviceToDevice, c->st));
        }
        CHK(wsget(c, S_BENCH + 3 * k + 1, sbytes, &in[k]));
        CHK(wsget(c, S_BENCH + 3 * k + 2, sbytes, &out[k]));
        HIPCHK(hipMemcpyAsync(in[k], c->U32, sbytes, hipMemcpyDeviceToDevice, c->st));
    }
    return time_launches(c, reps, copies, [&](int k) -> int {
        HIPCHK(launch_clover(c->g, prec, P32, 0, cl[k], in[k], out[k], c->st));
        return WCL_OK;
    }, ms);
}

extern "C" int wcl_bench_stream(wcl_ctx *c, double mib, int reps, double *read_gbs, double *copy_gbs)
{
    if (!c || !read_gbs || !copy_gbs) return fail(WCL_EINVAL, "null argument");
    if (!(mib >= 1.0 && mib <= 65536.0) || reps < 1) return fail(WCL_EINVAL, "1 <= mib <= 65536 and reps >= 1 required");
    const size_t bytes = ((size_t)(mib * 1048576.0) / 16) * 16, n16 = bytes / 16;
    const int blocks = 4 * std::max(c->num_cus, 1);
    void *a, *b, *out;
    CHK(wsget(c, S_BENCH, bytes, &a));
    CHK(wsget(c, S_BENCH + 1, bytes, &b));
    CHK(wsget(c, S_BENCH + 2, (size_t)blocks * 256 * sizeof(float), &out));
    HIPCHK(launch_zero(P32, bytes / 8, a, c->st));
    double ms[2];
    for (int copy = 0; copy < 2; copy++) {
        CHK(time_launches(c, reps, 1, [&](int) -> int {
            HIPCHK(launch_stream(copy, a, b, n16, (float *)out, blocks, c->st));
            return WCL_OK;
        }, &ms[copy]));
    }
    *read_gbs = bytes / (ms[0] * 1e-3) / 1e9;
    *copy_gbs = 2.0 * bytes / (ms[1] * 1e-3) / 1e9;
    return WCL_OK;
}

extern "C" int wcl_grad(wcl_ctx *c, const double *x, const double *y, double *gU, double *gk)
{
    if (!c || !x || !y || !gU || !gk) return fail(WCL_EINVAL, "null argument");
    if (!c->have_params) return fail(WCL_ESTATE, "wcl_grad before wcl_set_gauge and wcl_set_params");
    const size_t Vh = c->Vh;
    const size_t f64 = 2 * spinor_bytes(8, Vh);
    void *X, *Y, *K, *G, *HX, *CX;
    CHK(wsget(c, S_GX, f64, &X));
    CHK(wsget(c, S_GY, f64, &Y));
    CHK(wsget(c, S_GK, 2 * 6 * 9 * 16 * Vh, &K));
    CHK(wsget(c, S_GG, link_bytes(8, Vh), &G));
    CHK(wsget(c, S_GHX, f64, &HX));
    CHK(wsget(c, S_GCX, f64, &CX));
    HIPCHK(launch_pack_spinor(c->g, x, X, c->st));
    HIPCHK(launch_pack_spinor(c->g, y, Y, c->st));
    HIPCHK(launch_grad(c->g, c->U64, X, Y, K, c->kappa, c->csw, G, c->st));
    HIPCHK(launch_export_links(c->g, G, gU, c->st));
    // dL/dkappa = Re<y, H x> + c_sw Re<y, C x>
    for (int p = 0; p < 2; p++) {
        HopLaunch L = hop_base(c, P64, P64);
        L.mode = HOP;
        L.p = p;
        L.in = par(X, P64, Vh, 1 - p);
        L.out = par(HX, P64, Vh, p);
        CHK(run_hop(c, L));
    }
    HIPCHK(launch_sigmaF(c->g, c->U64, X, CX, c->st));
    const void *a[2] = {Y, Y}, *b[2] = {HX, CX};
    HIPCHK(launch_dots(P64, 24 * Vh, 2, a, b, c->partials, nullptr, c->st, 1, 0, c->pstride));
    double part[2][RED_BLOCKS];   // the real parts of <y, Hx> and <y, Cx> (terms 0 and 2)
    HIPCHK(hipMemcpyAsync(part[0], c->partials, sizeof(part[0]), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipMemcpyAsync(part[1], c->partials + 2 * (size_t)c->pstride, sizeof(part[1]), hipMemcpyDeviceToHost,
                          c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    double yhx = 0.0, ycx = 0.0;
    for (int j = 0; j < RED_BLOCKS; j++) {
        yhx += part[0][j];
        ycx += part[1][j];
    }
    *gk = yhx + c->csw * ycx;
    return WCL_OK;
}

// ===========================================================================
extern "C" int wcl_profile(wcl_ctx *c, int enable)
{
    if (!c) return fail(WCL_EINVAL, "null context");
    HIPCHK(hipStreamSynchronize(c->st));
    for (auto &r : c->recs) {
        if (r.e0) c->pool.push_back(r.e0);
        if (r.e1) c->pool.push_back(r.e1);
    }
    c->recs.clear();
    memset(c->stats, 0, sizeof(c->stats));
    c->prof = enable != 0;
    return WCL_OK;
}

extern "C" int wcl_profile_mask(wcl_ctx *c, int mask)
{
    if (!c) return fail(WCL_EINVAL, "null context");
    if (mask < 0 || mask >= (1 << WCL_K_COUNT)) return fail(WCL_EINVAL, "mask holds bits of WCL_K_* classes only");
    c->prof_mask = mask;
    return WCL_OK;
}

extern "C" int wcl_profile_read(wcl_ctx *c, int kclass, wcl_kstat *out)
{
    if (!c || !out || kclass < 0 || kclass >= WCL_K_COUNT) return fail(WCL_EINVAL, "bad argument");
    HIPCHK(hipStreamSynchronize(c->st));
    for (auto &r : c->recs) {
        float ms = 0.f;
        if (r.e0) HIPCHK(hipEventElapsedTime(&ms, r.e0, r.e1));
        wcl_kstat &k = c->stats[r.kclass];
        if (r.flops > 0.0) {  // launches that did work (not no-ops queued past convergence)
            k.launches += 1;
            k.ms += ms;
            k.bytes += r.bytes;
            k.flops += r.flops;
        } else {
            k.idle_launches += 1;
            k.idle_ms += ms;
        }
        if (r.e0) c->pool.push_back(r.e0);
        if (r.e1) c->pool.push_back(r.e1);
    }
    c->recs.clear();
    *out = c->stats[kclass];
    return WCL_OK;
}

extern "C" int wcl_set_tuning(wcl_ctx *c, int hop_block, int hop_depth, int hop_xcd, int hop_nontemporal)
{
    if (!c) return fail(WCL_EINVAL, "null context");
    if (hop_block != 64 && hop_block != 128 && hop_block != 256) return fail(WCL_EINVAL, "hop_block must be 64, 128 or 256");
    if (hop_depth < 2 || hop_depth > 3) return fail(WCL_EINVAL, "hop_depth must be 2 or 3");
    c->hop_block = hop_block;
    c->hop_depth = hop_depth;
    c->hop_xcd = hop_xcd ? 1 : 0;
    c->hop_nt = hop_nontemporal ? 1 : 0;
    return WCL_OK;
}

extern "C" int wcl_set_hop_tiles(wcl_ctx *c, int tiles)
{
    if (!c) return fail(WCL_EINVAL, "null context");
    if (tiles != 1 && tiles != 2 && tiles != 4 && tiles != 8) return fail(WCL_EINVAL, "tiles must be 1, 2, 4 or 8");
    c->hop_tpw = tiles;
    return WCL_OK;
}

extern "C" int wcl_set_hop_staging(wcl_ctx *c, int enable)
{
    if (!c) return fail(WCL_EINVAL, "null context");
    c->hop_lds = enable ? 1 : 0;
    return WCL_OK;
}

extern "C" int wcl_set_batch_tuning(wcl_ctx *c, int rhs_per_thread)
{
    if (!c) return fail(WCL_EINVAL, "null context");
    if (rhs_per_thread != 1 && rhs_per_thread != 2 && rhs_per_thread != 4)
        return fail(WCL_EINVAL, "rhs_per_thread must be 1, 2 or 4");
    c->hop_rhs = rhs_per_thread;
    return WCL_OK;
}

namespace {
struct TuneKey {
    int L[4], B[4], tbc, prec, compress, nrhs, flags, device, nt, stage;
    bool operator<(const TuneKey &o) const { return memcmp(this, &o, sizeof(TuneKey)) < 0; }
};
std::mutex g_tune_mu;
std::map<TuneKey, wcl_tuning> g_tune_cache;
}  // namespace

extern "C" int wcl_autotune(wcl_ctx *c, int prec, int nrhs, const double *b, const wcl_solve_opts *opts, int flags,
                            wcl_tuning *out)
{
    if (!c || !out) return fail(WCL_EINVAL, "null argument");
    if (prec != 32 && prec != 16) return fail(WCL_EINVAL, "autotune prec must be 32 or 16");
    if (nrhs < 1 || nrhs > 64) return fail(WCL_EINVAL, "autotune nrhs must be 1 .. 64");
    if (flags <= 0 || flags > (WCL_TUNE_HOP | WCL_TUNE_BATCH | WCL_TUNE_SCHWARZ))
        return fail(WCL_EINVAL, "unknown autotune flags");
    if ((flags & WCL_TUNE_SCHWARZ) && (!b || !opts)) return fail(WCL_EINVAL, "Schwarz tuning needs b_dev and opts");
    TuneKey key;
    memset(&key, 0, sizeof(key));
    for (int mu = 0; mu < 4; mu++) { key.L[mu] = c->g.L[mu]; key.B[mu] = c->g.B[mu]; }
    key.tbc = c->g.tbc; key.prec = prec; key.compress = c->compress; key.nrhs = nrhs; key.flags = flags;
    key.device = c->device;
    key.nt = c->hop_nt;              // candidates are timed with the caller's load policy
    key.stage = c->hop_lds;
    wcl_tuning t;
    memset(&t, 0, sizeof(t));
    t.hop_block = c->hop_block; t.hop_depth = c->hop_depth; t.hop_xcd = c->hop_xcd; t.hop_tiles = c->hop_tpw;
    t.rhs_per_thread = c->hop_rhs;
    t.use_ras = opts ? opts->use_ras : 1;
    t.ras_overlap = opts ? opts->ras_overlap : c->ras_overlap;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            t = it->second;
            t.cached = 1;
        }
    }
    if (t.cached) {
        CHK(wcl_set_tuning(c, t.hop_block, t.hop_depth, t.hop_xcd, c->hop_nt));
        CHK(wcl_set_hop_tiles(c, t.hop_tiles));
        CHK(wcl_set_batch_tuning(c, t.rhs_per_thread));
        *out = t;
        return WCL_OK;
    }
    if (flags & WCL_TUNE_HOP) {
        const int blocks[3] = {64, 128, 256}, depths[2] = {2, 3}, tiles[2] = {1, 2};
        double best = 1e30;
        for (int xcd = 0; xcd < 2; xcd++)
            for (int ib = 0; ib < 3; ib++)
                for (int io = 0; io < 2; io++)
                    for (int it = 0; it < 2; it++) {
                        CHK(wcl_set_tuning(c, blocks[ib], depths[io], xcd, c->hop_nt));
                        CHK(wcl_set_hop_tiles(c, tiles[it]));
                        // the best of three timings: one slow sample (clock ramp,
                        // another process) must not decide
                        double ms = 1e30;
                        for (int rep = 0; rep < 3; rep++) {
                            double m;
                            CHK(wcl_bench_hop(c, prec, nrhs, 20, 4, &m));
                            ms = std::min(ms, m);
                        }
                        if (ms < best) {
                            best = ms;
                            t.hop_block = blocks[ib]; t.hop_depth = depths[io]; t.hop_xcd = xcd; t.hop_tiles = tiles[it];
                        }
                    }
        CHK(wcl_set_tuning(c, t.hop_block, t.hop_depth, t.hop_xcd, c->hop_nt));
        CHK(wcl_set_hop_tiles(c, t.hop_tiles));
        t.hop_ms = best;
    }
    if ((flags & WCL_TUNE_BATCH) && nrhs > 1) {
        const int rpt[3] = {1, 2, 4};
        double best = 1e30;
        for (int k = 0; k < 3; k++) {
            CHK(wcl_set_batch_tuning(c, rpt[k]));
            double ms = 1e30;
            for (int rep = 0; rep < 3; rep++) {
                double m;
                CHK(wcl_bench_hop(c, prec, nrhs, 20, 4, &m));
                ms = std::min(ms, m);
            }
            if (ms < best) { best = ms; t.rhs_per_thread = rpt[k]; }
        }
        CHK(wcl_set_batch_tuning(c, t.rhs_per_thread));
        if (!(flags & WCL_TUNE_HOP)) t.hop_ms = best;
    }
    if (flags & WCL_TUNE_SCHWARZ) {
        // candidates: the given recipe, the same without overlap, no Schwarz;
        // each solve once untimed (workspace, clover caches), then timed
        const size_t bytes = (size_t)nrhs * c->V * 24 * sizeof(double);
        void *x = nullptr;
        CHK(alloc(&x, bytes));
        struct Free { void *p; ~Free() { if (p) (void)hipFree(p); } } guard{x};
        std::vector<wcl_solve_info> info(nrhs);
        const int cand_ras[3] = {1, 1, 0}, cand_ov[3] = {opts->ras_overlap, 0, opts->ras_overlap};
        double best = 1e30;
        for (int k = 0; k < 3; k++) {
            if (k == 1 && opts->ras_overlap == 0) continue;
            wcl_solve_opts o = *opts;
            o.use_ras = cand_ras[k];
            o.ras_overlap = cand_ov[k];
            o.x0_dev = nullptr;
            const int rc0 = wcl_solve(c, b, (double *)x, nrhs, &o, info.data());
            if (rc0 != WCL_OK) continue;   // a recipe that does not converge is not a candidate
            HIPCHK(hipStreamSynchronize(c->st));
            const auto t0 = std::chrono::steady_clock::now();
            const int rc = wcl_solve(c, b, (double *)x, nrhs, &o, info.data());
            HIPCHK(hipStreamSynchronize(c->st));
            const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (rc == WCL_OK && ms < best) { best = ms; t.use_ras = o.use_ras; t.ras_overlap = o.ras_overlap; }
        }
        if (best == 1e30) return fail(WCL_ENOCONV, "autotune: no Schwarz candidate solved the system");
        t.solve_ms = best;
        // leave the context's Schwarz settings as the caller's opts had them
        if (opts->use_ras) CHK(wcl_set_ras(c, opts->ras_overlap, opts->ras_iters, opts->ras_solver, opts->ras_mult));
    }
    t.cached = 0;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune_cache[key] = t;
    }
    *out = t;
    return WCL_OK;
}

extern "C" int wcl_autotune_hop(wcl_ctx *c, int prec, int copies, int *best)
{
    if (!c) return fail(WCL_EINVAL, "null context");
    const int blocks[3] = {64, 128, 256}, depths[2] = {2, 3};
    double best_ms = 1e30;
    int bb = c->hop_block, bo = c->hop_depth, bx = c->hop_xcd;
    for (int xcd = 0; xcd < 2; xcd++)
        for (int ib = 0; ib < 3; ib++)
            for (int io = 0; io < 2; io++) {
                CHK(wcl_set_tuning(c, blocks[ib], depths[io], xcd, c->hop_nt));
                double ms;
                CHK(wcl_bench_hop(c, prec, 1, 50, copies, &ms));
                if (ms < best_ms) { best_ms = ms; bb = blocks[ib]; bo = depths[io]; bx = xcd; }
            }
    CHK(wcl_set_tuning(c, bb, bo, bx, c->hop_nt));
    if (best) { best[0] = bb; best[1] = bo; best[2] = bx; }
    return WCL_OK;
}
