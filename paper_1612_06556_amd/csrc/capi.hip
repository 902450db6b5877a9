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
#include <string>
#include <vector>

#include "../../include/wcl.h"
#include "wcl_launch.h"

using namespace wcl;

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
    void *T64 = nullptr, *Ti64 = nullptr, *T32 = nullptr, *Ti32 = nullptr, *T16 = nullptr, *Ti16 = nullptr;
    int *info = nullptr;
    double kappa = 0, csw = 0;
    bool have_gauge = false, have_params = false;
    int ras_overlap = 1, ras_iters = 4;
    std::vector<Buf> ws;        // workspace, indexed by slot
    double *partials = nullptr; // [6][RED_BLOCKS]
    Scalars *sc = nullptr;      // [2]: outer, inner
    Scalars *sc_host = nullptr; // pinned mirror
    // hopping-kernel launch configuration (set by wcl_set_tuning / wcl_autotune_hop)
    int hop_block = 256, hop_depth = 2, hop_xcd = 1;
    // event profiling of kernel classes
    struct Rec {
        int kclass;
        hipEvent_t e0, e1;
        double bytes, flops;
    };
    bool prof = false;
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

void *links_for(wcl_ctx *c, int prec) { return prec == P64 ? c->U64 : prec == P32 ? c->U32 : c->U16; }
void *clov_for(wcl_ctx *c, int prec) { return prec == P64 ? c->T64 : prec == P32 ? c->T32 : c->T16; }
void *clovinv_for(wcl_ctx *c, int prec) { return prec == P64 ? c->Ti64 : prec == P32 ? c->Ti32 : c->Ti16; }

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
    L.link_prec = lprec;
    L.spin_prec = sprec;
    L.links = links_for(c, lprec);
    L.nrhs = 1;
    L.xcd = c->hop_xcd;
    L.block = c->hop_block;
    L.depth = c->hop_depth;
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
    if (c->prof) {
        e0 = take_event(c);
        e1 = take_event(c);
        if (!e0 || !e1) return fail(WCL_EHIP, "hipEventCreate failed");
        HIPCHK(hipEventRecord(e0, c->st));
    }
    HIPCHK(launch());
    if (c->prof) {
        HIPCHK(hipEventRecord(e1, c->st));
        c->recs.push_back({kclass, e0, e1, bytes, flops});
    }
    return WCL_OK;
}

int run_hop(wcl_ctx *c, const HopLaunch &L)
{
    double b = 0, f = 0;
    if (c->prof) hop_work(L, &b, &f);
    return profiled(c, WCL_K_HOP, b, f, [&] { return launch_hop(L, c->st); });
}

int run_ras(wcl_ctx *c, const RasLaunch &R)
{
    double b = 0, f = 0;
    if (c->prof) ras_work(R, &b, &f);
    return profiled(c, WCL_K_RAS, b, f, [&] { return launch_ras(R, c->st); });
}

int run_clover(wcl_ctx *c, int lp, int sp, int p, const void *clov, const void *in, void *out)
{
    const double sb = sp == P64 ? 192.0 : sp == P32 ? 96.0 : 48.0;
    const double cb = lp == P64 ? 576.0 : lp == P32 ? 288.0 : 144.0;
    return profiled(c, WCL_K_CLOVER, (2 * sb + cb) * c->Vh, 504.0 * c->Vh,
                    [&] { return launch_clover(c->g, lp, sp, p, clov, in, out, c->st); });
}

// One parity of the full operator: out_p = A_pp x_p + coef H in_{1-p}
int full_D_parity(wcl_ctx *c, int lprec, int sprec, int p, const void *field_in, void *field_out, int dagger,
                  const Scalars *sc)
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
    CHK(run_hop(c, L));
    return WCL_OK;
}

int full_D(wcl_ctx *c, int lprec, int sprec, const void *in, void *out, int dagger, const Scalars *sc = nullptr)
{
    CHK(full_D_parity(c, lprec, sprec, 0, in, out, dagger, sc));
    CHK(full_D_parity(c, lprec, sprec, 1, in, out, dagger, sc));
    return WCL_OK;
}

// Schur operator on even fields: tmp_o = A_oo^-1 H_oe in_e ; out_e = in_e - k^2 A_ee^-1 H_eo tmp_o
int schur(wcl_ctx *c, int lprec, int sprec, const void *in_e, void *out_e, void *tmp_o, const Scalars *sc)
{
    HopLaunch L = hop_base(c, lprec, sprec);
    L.clov = clovinv_for(c, lprec);
    L.sc = sc;
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

// bhat_e = A_ee^-1 (b_e + k H_eo A_oo^-1 b_o)  (field b: both parities, FP64)
int schur_rhs64(wcl_ctx *c, const void *b, void *bhat_e, void *tmp_o, void *tmp_e)
{
    CHK(run_clover(c, P64, P64, 1, c->Ti64, par(b, P64, c->Vh, 1), tmp_o));
    CHK(run_clover(c, P64, P64, 0, c->Ti64, par(b, P64, c->Vh, 0), tmp_e));
    HopLaunch L = hop_base(c, P64, P64);
    L.mode = XPAY;
    L.p = 0;
    L.in = tmp_o;
    L.x = tmp_e;
    L.out = bhat_e;
    L.clov = c->Ti64;
    L.coef = c->kappa;
    CHK(run_hop(c, L));
    return WCL_OK;
}

// x_o = A_oo^-1 (b_o + k H_oe x_e) into the odd half of field x (even half = x_e already)
int reconstruct64(wcl_ctx *c, const void *b, void *x, void *tmp_o)
{
    CHK(run_clover(c, P64, P64, 1, c->Ti64, par(b, P64, c->Vh, 1), tmp_o));
    HopLaunch L = hop_base(c, P64, P64);
    L.mode = XPAY;
    L.p = 1;
    L.in = par(x, P64, c->Vh, 0);
    L.x = tmp_o;
    L.out = par(x, P64, c->Vh, 1);
    L.clov = c->Ti64;
    L.coef = c->kappa;
    CHK(run_hop(c, L));
    return WCL_OK;
}

int check_prec(int prec) { return (prec == 64 || prec == 32 || prec == 16) ? WCL_OK : fail(WCL_EINVAL, "prec must be 64, 32 or 16"); }

int read_scalars(wcl_ctx *c, int which)
{
    HIPCHK(hipMemcpyAsync(c->sc_host + which, c->sc + which, sizeof(Scalars), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    return WCL_OK;
}

int write_scalars(wcl_ctx *c, int which)
{
    HIPCHK(hipMemcpyAsync(c->sc + which, c->sc_host + which, sizeof(Scalars), hipMemcpyHostToDevice, c->st));
    return WCL_OK;
}

// |v|^2 of n complex numbers into sc[which].t[0] (device)
int norm2_dev(wcl_ctx *c, int prec, size_t n, const void *v, int which)
{
    const void *a[1] = {v}, *b[1] = {v};
    HIPCHK(launch_dots(prec, n, 1, a, b, c->partials, nullptr, c->st));
    HIPCHK(launch_finalize(NORM_ONLY, 2, c->partials, c->sc + which, c->st));
    return WCL_OK;
}

int norm2_host(wcl_ctx *c, int prec, size_t n, const void *v, double *out)
{
    CHK(norm2_dev(c, prec, n, v, 1));
    CHK(read_scalars(c, 1));
    *out = c->sc_host[1].t[0];
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
    // bench copies start here
    S_BENCH = 64,
};

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
    if (V > (1ll << 30)) return fail(WCL_EINVAL, "lattice too large");
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
    c->st = (hipStream_t)hip_stream;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return fail(WCL_EHIP, "no HIP device");
    }
    int rc = WCL_OK;
    if ((rc = alloc((void **)&c->partials, sizeof(double) * 6 * RED_BLOCKS)) != WCL_OK ||
        (rc = alloc((void **)&c->sc, sizeof(Scalars) * 2)) != WCL_OK ||
        (rc = alloc((void **)&c->info, sizeof(int))) != WCL_OK) {
        wcl_destroy(c);
        return rc;
    }
    if (hipHostMalloc((void **)&c->sc_host, sizeof(Scalars) * 2, hipHostMallocDefault) != hipSuccess) {
        wcl_destroy(c);
        return fail(WCL_ENOMEM, "hipHostMalloc failed");
    }
    memset(c->sc_host, 0, sizeof(Scalars) * 2);
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
    void *ptrs[] = {c->U64, c->U32, c->U16, c->T64, c->Ti64, c->T32, c->Ti32, c->T16, c->Ti16, c->info,
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
    if (!c->U64) {
        CHK(alloc(&c->U64, link_bytes(8, Vh)));
        CHK(alloc(&c->U32, link_bytes(4, Vh)));
        CHK(alloc(&c->U16, link_bytes(2, Vh)));
    }
    HIPCHK(launch_ingest_gauge(c->g, U, c->U64, c->U32, c->U16, c->st));
    c->have_gauge = true;
    c->have_params = false;
    return WCL_OK;
}

int wcl_set_params(wcl_ctx *c, double kappa, double csw)
{
    if (!c) return fail(WCL_EINVAL, "null context");
    if (!c->have_gauge) return fail(WCL_ESTATE, "wcl_set_params before wcl_set_gauge");
    if (!std::isfinite(kappa) || !std::isfinite(csw)) return fail(WCL_EINVAL, "kappa and csw must be finite");
    const size_t Vh = c->Vh;
    if (!c->T64) {
        CHK(alloc(&c->T64, clover_bytes(8, Vh)));
        CHK(alloc(&c->Ti64, clover_bytes(8, Vh)));
        CHK(alloc(&c->T32, clover_bytes(4, Vh)));
        CHK(alloc(&c->Ti32, clover_bytes(4, Vh)));
        CHK(alloc(&c->T16, clover_bytes(2, Vh)));
        CHK(alloc(&c->Ti16, clover_bytes(2, Vh)));
    }
    c->kappa = kappa;
    c->csw = csw;
    int zero = 0, bad = 0;
    HIPCHK(hipMemcpyAsync(c->info, &zero, sizeof(int), hipMemcpyHostToDevice, c->st));
    HIPCHK(launch_clover_build(c->g, c->U64, csw * kappa, c->T64, c->Ti64, c->T32, c->Ti32, c->T16, c->Ti16,
                               c->info, c->st));
    HIPCHK(hipMemcpyAsync(&bad, c->info, sizeof(int), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    if (bad) return fail(WCL_ENAN, std::to_string(bad) + " clover blocks are not positive definite");
    c->have_params = true;
    return WCL_OK;
}

int wcl_set_ras(wcl_ctx *c, int overlap, int iters)
{
    if (!c) return fail(WCL_EINVAL, "null context");
    if (overlap < 0 || iters < 1) return fail(WCL_EINVAL, "overlap >= 0 and iters >= 1 required");
    for (int mu = 0; mu < 4; mu++)
        if (overlap > c->g.B[mu] || c->g.L[mu] < c->g.B[mu] + 2 * overlap)
            return fail(WCL_EINVAL, "RAS extended block does not fit the lattice");
    if (ras_threads(c->g, overlap) > 1024) return fail(WCL_EINVAL, "RAS extended block too large for one workgroup");
    c->ras_overlap = overlap;
    c->ras_iters = iters;
    return WCL_OK;
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
            RasLaunch R;
            R.g = &c->g;
            R.overlap = c->ras_overlap;
            R.iters = c->ras_iters;
            R.link_prec = lp;
            R.in = par(a, sp, Vh, 0);
            R.out = par(b, sp, Vh, 0);
            R.links = links_for(c, lp);
            R.clov_inv = clovinv_for(c, lp);
            R.kappa2 = (float)(c->kappa * c->kappa);
            R.sc = nullptr;
            CHK(run_ras(c, R));
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
    o->inner_prec = 32;
    o->use_graph = 0;
    o->check_every = 8;
}

}  // extern "C"

// ===========================================================================
// Solvers.
namespace {

struct SolveWs {
    // FP64 full fields (both parities)
    void *b, *x, *res;
    // FP64 even vectors
    void *bh, *xe, *r, *rt, *p, *v, *s, *t, *ph, *sh, *o;
    // FP32 even vectors
    void *rhs, *x32, *r32, *rt32, *p32, *v32, *s32, *t32, *ph32, *sh32, *o32;
};

int get_ws(wcl_ctx *c, SolveWs &w, bool inner)
{
    const size_t Vh = c->Vh;
    const size_t e64 = spinor_bytes(8, Vh), e32 = spinor_bytes(4, Vh);
    CHK(wsget(c, S_B64, 2 * e64, &w.b));
    CHK(wsget(c, S_X64, 2 * e64, &w.x));
    CHK(wsget(c, S_R64F, 2 * e64, &w.res));
    void **ev[] = {&w.bh, &w.xe, &w.r, &w.rt, &w.p, &w.v, &w.s, &w.t, &w.ph, &w.sh, &w.o};
    for (int k = 0; k < 11; k++) CHK(wsget(c, S_BH + k, e64, ev[k]));
    if (inner) {
        void **fv[] = {&w.rhs, &w.x32, &w.r32, &w.rt32, &w.p32, &w.v32, &w.s32, &w.t32, &w.ph32, &w.sh32, &w.o32};
        for (int k = 0; k < 11; k++) CHK(wsget(c, S_RHS32 + k, e32, fv[k]));
    }
    return WCL_OK;
}

struct InnerCfg {
    int lprec;
    double tol;
    int maxit;
    bool ras;
    int check_every;
};

// One BiCGStab iteration (right preconditioned by RAS when enabled) on the
// FP32 Schur system, all scalars in sc (device).
int inner_iteration(wcl_ctx *c, const InnerCfg &cfg, SolveWs &w, Scalars *sc)
{
    const size_t n = 12 * (size_t)c->Vh;
    const int lp = cfg.lprec;
    HIPCHK(launch_bicg_p(P32, n, w.r32, w.p32, w.v32, sc, c->st));
    void *ph = w.p32, *sh = w.s32;
    RasLaunch R;
    if (cfg.ras) {
        R.g = &c->g;
        R.overlap = c->ras_overlap;
        R.iters = c->ras_iters;
        R.link_prec = lp;
        R.links = links_for(c, lp);
        R.clov_inv = clovinv_for(c, lp);
        R.kappa2 = (float)(c->kappa * c->kappa);
        R.sc = sc;
        R.in = w.p32;
        R.out = w.ph32;
        CHK(run_ras(c, R));
        ph = w.ph32;
    }
    CHK(schur(c, lp, P32, ph, w.v32, w.o32, sc));
    {
        const void *a[1] = {w.rt32}, *b[1] = {w.v32};
        HIPCHK(launch_dots(P32, n, 1, a, b, c->partials, sc, c->st));
        HIPCHK(launch_finalize(BICG_ALPHA, 2, c->partials, sc, c->st));
    }
    HIPCHK(launch_bicg_s(P32, n, w.r32, w.v32, w.s32, sc, c->st));
    if (cfg.ras) {
        R.in = w.s32;
        R.out = w.sh32;
        CHK(run_ras(c, R));
        sh = w.sh32;
    }
    CHK(schur(c, lp, P32, sh, w.t32, w.o32, sc));
    {
        const void *a[2] = {w.t32, w.t32}, *b[2] = {w.s32, w.t32};
        HIPCHK(launch_dots(P32, n, 2, a, b, c->partials, sc, c->st));
        HIPCHK(launch_finalize(BICG_OMEGA, 4, c->partials, sc, c->st));
    }
    HIPCHK(launch_bicg_xr(P32, n, w.x32, ph, sh, w.r32, w.s32, w.t32, sc, c->st));
    {
        const void *a[2] = {w.rt32, w.r32}, *b[2] = {w.r32, w.r32};
        HIPCHK(launch_dots(P32, n, 2, a, b, c->partials, sc, c->st));
        HIPCHK(launch_finalize(BICG_RHO, 4, c->partials, sc, c->st));
    }
    return WCL_OK;
}

// out64 = ||in64|| * K(in64 / ||in64||): the single-precision inner solve.
int inner_solve(wcl_ctx *c, const InnerCfg &cfg, SolveWs &w, const void *in64, void *out64, int *iters)
{
    const size_t n = 12 * (size_t)c->Vh;
    const size_t Vh = c->Vh;
    Scalars *sc = c->sc + 1;
    CHK(norm2_dev(c, P64, n, in64, 1));
    HIPCHK(launch_convert(P64, P32, Vh, Vh, Vh, in64, w.r32, &sc->t[0], 1, 1.0, c->st));
    HIPCHK(launch_copy(P32, n, w.r32, w.rt32, c->st));
    HIPCHK(launch_zero(P32, n, w.x32, c->st));
    HIPCHK(launch_zero(P32, n, w.p32, c->st));
    HIPCHK(launch_zero(P32, n, w.v32, c->st));
    {
        const void *a[2] = {w.rt32, w.r32}, *b[2] = {w.r32, w.r32};
        HIPCHK(launch_dots(P32, n, 2, a, b, c->partials, nullptr, c->st));
        HIPCHK(launch_finalize(BICG_INIT_RHO, 4, c->partials, sc, c->st));
    }
    // Iterations are queued in chunks; every kernel of an iteration queued
    // after convergence is a no-op.  The chunk length follows the observed
    // convergence rate so that few such iterations are queued.
    int launched = 0;
    int chunk = std::min(cfg.check_every, 4);
    double r2_prev = 1.0;  // |r0|^2 of the normalised right-hand side
    int it_prev = 0;
    std::vector<size_t> rec_mark;  // profile records at the start of each queued iteration
    while (launched < cfg.maxit) {
        chunk = std::max(1, std::min(chunk, cfg.maxit - launched));
        for (int k = 0; k < chunk; k++) {
            rec_mark.push_back(c->recs.size());
            CHK(inner_iteration(c, cfg, w, sc));
        }
        launched += chunk;
        CHK(read_scalars(c, 1));
        const Scalars &h = c->sc_host[1];
        if (h.done) break;
        // predicted iterations to reach the target at the rate seen so far
        const int di = h.iter - it_prev;
        if (di > 0 && h.r2 > 0.0 && h.r2 < r2_prev) {
            const double rate = std::log(h.r2 / r2_prev) / di;
            const double need = std::log(h.stop2 * h.b2 / h.r2) / rate;
            chunk = (int)std::min(16.0, std::max(1.0, std::floor(need)));
        } else {
            chunk = std::min(cfg.check_every, 4);
        }
        r2_prev = h.r2;
        it_prev = h.iter;
    }
    *iters = c->sc_host[1].iter;
    // launches of iterations past the converged one did no work
    for (size_t k = (size_t)*iters; k < rec_mark.size(); k++) {
        const size_t end = (k + 1 < rec_mark.size()) ? rec_mark[k + 1] : c->recs.size();
        for (size_t r = rec_mark[k]; r < end; r++) c->recs[r].bytes = c->recs[r].flops = 0.0;
    }
    HIPCHK(launch_convert(P32, P64, Vh, Vh, Vh, w.x32, out64, &sc->t[0], 2, 1.0, c->st));
    return WCL_OK;
}

// true relative residual of the full system: ||b - D x|| / ||b|| (FP64)
int true_residual(wcl_ctx *c, SolveWs &w, double bnorm2, double *rel)
{
    const size_t n = 24 * (size_t)c->Vh;
    CHK(full_D(c, P64, P64, w.x, w.res, 0));
    HIPCHK(launch_axpby(P64, n, make_double2(1.0, 0.0), w.b, make_double2(-1.0, 0.0), w.res, c->st));
    double r2;
    CHK(norm2_host(c, P64, n, w.res, &r2));
    *rel = std::sqrt(r2 / bnorm2);
    return WCL_OK;
}

int set_outer_stop(wcl_ctx *c, double stop2)
{
    CHK(read_scalars(c, 0));
    c->sc_host[0].stop2 = stop2;
    c->sc_host[0].done = 0;
    CHK(write_scalars(c, 0));
    return WCL_OK;
}

// FP64 (flexible) BiCGStab on the Schur system with preconditioner K.
int outer_fbicgstab(wcl_ctx *c, const wcl_solve_opts &o, const InnerCfg &cfg, SolveWs &w, double bnorm2,
                    wcl_solve_info &info)
{
    const size_t n = 12 * (size_t)c->Vh;
    Scalars *sc = c->sc;
    double bh2;
    CHK(norm2_host(c, P64, n, w.bh, &bh2));
    HIPCHK(launch_copy(P64, n, w.bh, w.r, c->st));
    HIPCHK(launch_zero(P64, n, w.xe, c->st));
    int inner_total = 0;
    int status = WCL_ENOCONV;
    for (int restart = 0; restart < 8 && status == WCL_ENOCONV; restart++) {
        // (re)start the recurrence from the current residual r
        HIPCHK(launch_copy(P64, n, w.r, w.rt, c->st));
        HIPCHK(launch_zero(P64, n, w.p, c->st));
        HIPCHK(launch_zero(P64, n, w.v, c->st));
        {
            const void *a[2] = {w.rt, w.r}, *b[2] = {w.r, w.r};
            HIPCHK(launch_dots(P64, n, 2, a, b, c->partials, nullptr, c->st));
            HIPCHK(launch_finalize(BICG_INIT_RHO, 4, c->partials, sc, c->st));
        }
        CHK(read_scalars(c, 0));
        // stop when |r|^2 <= tol^2 |b|^2 (b2 holds |r0|^2 after the init)
        const double r02 = c->sc_host[0].b2;
        if (r02 == 0.0) { status = WCL_OK; break; }
        CHK(set_outer_stop(c, o.tol * o.tol * bnorm2 / r02));
        bool restart_now = false;
        while (info.outer_iters < o.max_outer) {
            HIPCHK(launch_bicg_p(P64, n, w.r, w.p, w.v, sc, c->st));
            int it;
            CHK(inner_solve(c, cfg, w, w.p, w.ph, &it));
            inner_total += it;
            CHK(schur(c, P64, P64, w.ph, w.v, w.o, sc));
            {
                const void *a[1] = {w.rt}, *b[1] = {w.v};
                HIPCHK(launch_dots(P64, n, 1, a, b, c->partials, sc, c->st));
                HIPCHK(launch_finalize(BICG_ALPHA, 2, c->partials, sc, c->st));
            }
            HIPCHK(launch_bicg_s(P64, n, w.r, w.v, w.s, sc, c->st));
            CHK(inner_solve(c, cfg, w, w.s, w.sh, &it));
            inner_total += it;
            CHK(schur(c, P64, P64, w.sh, w.t, w.o, sc));
            {
                const void *a[2] = {w.t, w.t}, *b[2] = {w.s, w.t};
                HIPCHK(launch_dots(P64, n, 2, a, b, c->partials, sc, c->st));
                HIPCHK(launch_finalize(BICG_OMEGA, 4, c->partials, sc, c->st));
            }
            HIPCHK(launch_bicg_xr(P64, n, w.xe, w.ph, w.sh, w.r, w.s, w.t, sc, c->st));
            {
                const void *a[2] = {w.rt, w.r}, *b[2] = {w.r, w.r};
                HIPCHK(launch_dots(P64, n, 2, a, b, c->partials, sc, c->st));
                HIPCHK(launch_finalize(BICG_RHO, 4, c->partials, sc, c->st));
            }
            info.outer_iters++;
            CHK(read_scalars(c, 0));
            const Scalars &h = c->sc_host[0];
            if (!std::isfinite(h.r2)) { status = WCL_ENAN; break; }
            if (h.done == 1 || h.done == 2) {
                // true residual decides; otherwise replace r and restart
                HIPCHK(launch_copy(P64, n, w.xe, w.x, c->st));
                CHK(reconstruct64(c, w.b, w.x, w.o));
                double rel;
                CHK(true_residual(c, w, bnorm2, &rel));
                info.true_relres = rel;
                if (rel <= o.tol) { status = WCL_OK; break; }
                CHK(schur(c, P64, P64, w.xe, w.r, w.o, nullptr));
                HIPCHK(launch_axpby(P64, n, make_double2(1.0, 0.0), w.bh, make_double2(-1.0, 0.0), w.r, c->st));
                restart_now = true;
                break;
            }
        }
        if (!restart_now) break;
    }
    info.inner_iters_total = inner_total;
    if (status == WCL_ENOCONV && info.outer_iters >= o.max_outer) status = WCL_ENOCONV;
    info.status = status;
    return WCL_OK;
}

// Defect correction: x_e += K(r), r = bhat - Dhat x_e in FP64.
int outer_dc(wcl_ctx *c, const wcl_solve_opts &o, const InnerCfg &cfg, SolveWs &w, double bnorm2,
             wcl_solve_info &info)
{
    const size_t n = 12 * (size_t)c->Vh;
    HIPCHK(launch_copy(P64, n, w.bh, w.r, c->st));
    HIPCHK(launch_zero(P64, n, w.xe, c->st));
    int inner_total = 0;
    info.status = WCL_ENOCONV;
    while (info.outer_iters < o.max_outer) {
        int it;
        CHK(inner_solve(c, cfg, w, w.r, w.ph, &it));
        inner_total += it;
        HIPCHK(launch_axpby(P64, n, make_double2(1.0, 0.0), w.ph, make_double2(1.0, 0.0), w.xe, c->st));
        CHK(schur(c, P64, P64, w.xe, w.r, w.o, nullptr));
        HIPCHK(launch_axpby(P64, n, make_double2(1.0, 0.0), w.bh, make_double2(-1.0, 0.0), w.r, c->st));
        info.outer_iters++;
        double r2;
        CHK(norm2_host(c, P64, n, w.r, &r2));
        if (!std::isfinite(r2)) { info.status = WCL_ENAN; break; }
        if (r2 <= o.tol * o.tol * bnorm2) {
            HIPCHK(launch_copy(P64, n, w.xe, w.x, c->st));
            CHK(reconstruct64(c, w.b, w.x, w.o));
            double rel;
            CHK(true_residual(c, w, bnorm2, &rel));
            info.true_relres = rel;
            if (rel <= o.tol) { info.status = WCL_OK; break; }
        }
    }
    info.inner_iters_total = inner_total;
    return WCL_OK;
}

// Plain FP64 BiCGStab on the full D, no preconditioner.
int plain64(wcl_ctx *c, const wcl_solve_opts &o, SolveWs &w, double bnorm2, wcl_solve_info &info)
{
    const size_t n = 24 * (size_t)c->Vh;
    const size_t e64 = spinor_bytes(8, c->Vh);
    void *r, *rt, *p, *v, *s, *t;
    CHK(wsget(c, S_PR, 2 * e64, &r));
    CHK(wsget(c, S_PRT, 2 * e64, &rt));
    CHK(wsget(c, S_PP, 2 * e64, &p));
    CHK(wsget(c, S_PV, 2 * e64, &v));
    CHK(wsget(c, S_PS, 2 * e64, &s));
    CHK(wsget(c, S_PT, 2 * e64, &t));
    Scalars *sc = c->sc;
    HIPCHK(launch_zero(P64, n, w.x, c->st));
    HIPCHK(launch_copy(P64, n, w.b, r, c->st));
    info.status = WCL_ENOCONV;
    const int every = o.check_every > 0 ? o.check_every : 8;
    for (int restart = 0; restart < 8; restart++) {
        HIPCHK(launch_copy(P64, n, r, rt, c->st));
        HIPCHK(launch_zero(P64, n, p, c->st));
        HIPCHK(launch_zero(P64, n, v, c->st));
        {
            const void *a[2] = {rt, r}, *b[2] = {r, r};
            HIPCHK(launch_dots(P64, n, 2, a, b, c->partials, nullptr, c->st));
            HIPCHK(launch_finalize(BICG_INIT_RHO, 4, c->partials, sc, c->st));
        }
        CHK(read_scalars(c, 0));
        const double r02 = c->sc_host[0].b2;
        if (r02 == 0.0) { info.status = WCL_OK; break; }
        CHK(set_outer_stop(c, o.tol * o.tol * bnorm2 / r02));
        const int it0 = info.outer_iters;
        bool stop = false;
        std::vector<size_t> rec_mark;  // profile records at the start of each queued iteration
        int queued = 0;
        while (info.outer_iters < o.max_outer) {
            const int chunk = std::min(every, o.max_outer - it0 - queued);
            if (chunk <= 0) break;
            queued += chunk;
            for (int k = 0; k < chunk; k++) {
                rec_mark.push_back(c->recs.size());
                HIPCHK(launch_bicg_p(P64, n, r, p, v, sc, c->st));
                CHK(full_D(c, P64, P64, p, v, 0, sc));
                {
                    const void *a[1] = {rt}, *b[1] = {v};
                    HIPCHK(launch_dots(P64, n, 1, a, b, c->partials, sc, c->st));
                    HIPCHK(launch_finalize(BICG_ALPHA, 2, c->partials, sc, c->st));
                }
                HIPCHK(launch_bicg_s(P64, n, r, v, s, sc, c->st));
                CHK(full_D(c, P64, P64, s, t, 0, sc));
                {
                    const void *a[2] = {t, t}, *b[2] = {s, t};
                    HIPCHK(launch_dots(P64, n, 2, a, b, c->partials, sc, c->st));
                    HIPCHK(launch_finalize(BICG_OMEGA, 4, c->partials, sc, c->st));
                }
                HIPCHK(launch_bicg_xr(P64, n, w.x, p, s, r, s, t, sc, c->st));
                {
                    const void *a[2] = {rt, r}, *b[2] = {r, r};
                    HIPCHK(launch_dots(P64, n, 2, a, b, c->partials, sc, c->st));
                    HIPCHK(launch_finalize(BICG_RHO, 4, c->partials, sc, c->st));
                }
            }
            CHK(read_scalars(c, 0));
            const Scalars &h = c->sc_host[0];
            info.outer_iters = it0 + h.iter;
            for (size_t k = (size_t)h.iter; k < rec_mark.size(); k++) {  // no-op launches
                const size_t end = (k + 1 < rec_mark.size()) ? rec_mark[k + 1] : c->recs.size();
                for (size_t q = rec_mark[k]; q < end; q++) c->recs[q].bytes = c->recs[q].flops = 0.0;
            }
            if (!std::isfinite(h.r2)) { info.status = WCL_ENAN; stop = true; break; }
            if (h.done) {
                double rel;
                CHK(true_residual(c, w, bnorm2, &rel));
                info.true_relres = rel;
                if (rel <= o.tol) { info.status = WCL_OK; stop = true; }
                else HIPCHK(launch_copy(P64, n, w.res, r, c->st));  // residual replacement
                break;
            }
        }
        if (stop || info.outer_iters >= o.max_outer) break;
    }
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
    if (o.outer < 0 || o.outer > WCL_OUTER_PLAIN64) return fail(WCL_EINVAL, "unknown outer solver");
    if (o.inner_prec != 32 && o.inner_prec != 16) return fail(WCL_EINVAL, "inner_prec must be 32 or 16");
    if (o.check_every < 1) o.check_every = 8;
    if (o.use_ras && o.outer != WCL_OUTER_PLAIN64) CHK(wcl_set_ras(c, o.ras_overlap, o.ras_iters));
    SolveWs w;
    CHK(get_ws(c, w, o.outer != WCL_OUTER_PLAIN64));
    InnerCfg cfg{o.inner_prec, o.inner_tol, o.max_inner, o.use_ras != 0, o.check_every};
    // the inner stopping threshold is fixed for the whole solve
    {
        CHK(read_scalars(c, 1));
        c->sc_host[1].stop2 = o.inner_tol * o.inner_tol;
        CHK(write_scalars(c, 1));
    }
    int worst = WCL_OK;
    for (int k = 0; k < nrhs; k++) {
        wcl_solve_info info;
        memset(&info, 0, sizeof(info));
        HIPCHK(hipStreamSynchronize(c->st));
        const auto t0 = std::chrono::steady_clock::now();
        const double *bk = b + (size_t)k * c->V * 24;
        double *xk = x + (size_t)k * c->V * 24;
        HIPCHK(launch_pack_spinor(c->g, bk, w.b, c->st));
        if (o.adjoint) HIPCHK(launch_gamma5(2, c->Vh, w.b, c->st));  // D^dag = g5 D g5
        double bnorm2;
        CHK(norm2_host(c, P64, 24 * (size_t)c->Vh, w.b, &bnorm2));
        if (!std::isfinite(bnorm2)) {
            info.status = WCL_ENAN;
        } else if (bnorm2 == 0.0) {
            HIPCHK(launch_zero(P64, 24 * (size_t)c->Vh, w.x, c->st));
            info.status = WCL_OK;
        } else if (o.outer == WCL_OUTER_PLAIN64) {
            CHK(plain64(c, o, w, bnorm2, info));
        } else {
            CHK(schur_rhs64(c, w.b, w.bh, w.o, w.s));
            if (o.outer == WCL_OUTER_FBICGSTAB) CHK(outer_fbicgstab(c, o, cfg, w, bnorm2, info));
            else CHK(outer_dc(c, o, cfg, w, bnorm2, info));
            HIPCHK(launch_copy(P64, 12 * (size_t)c->Vh, w.xe, w.x, c->st));
            CHK(reconstruct64(c, w.b, w.x, w.o));
        }
        if (info.status != WCL_ENAN && bnorm2 > 0.0) {
            double rel;
            CHK(true_residual(c, w, bnorm2, &rel));
            info.true_relres = rel;
            if (info.status == WCL_OK && rel > o.tol) info.status = WCL_ENOCONV;
            if (!std::isfinite(rel)) info.status = WCL_ENAN;
        }
        if (o.adjoint) HIPCHK(launch_gamma5(2, c->Vh, w.x, c->st));
        HIPCHK(launch_unpack_spinor(c->g, w.x, xk, c->st));
        HIPCHK(hipStreamSynchronize(c->st));
        info.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (infos) infos[k] = info;
        if (info.status != WCL_OK && (worst == WCL_OK || info.status == WCL_ENAN)) worst = info.status;
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
extern "C" int wcl_bench_hop(wcl_ctx *c, int prec, int reps, int copies, double *ms)
{
    if (!c || !ms) return fail(WCL_EINVAL, "null argument");
    if (!c->have_gauge) return fail(WCL_ESTATE, "wcl_bench_hop before wcl_set_gauge");
    if (prec != 32 && prec != 16) return fail(WCL_EINVAL, "bench prec must be 32 or 16");
    if (reps < 1 || copies < 1 || copies > 32) return fail(WCL_EINVAL, "reps >= 1 and 1 <= copies <= 32 required");
    const size_t Vh = c->Vh;
    const int lb = prec_bytes(prec);
    const size_t lbytes = link_bytes(lb, Vh), sbytes = spinor_bytes(4, Vh);
    std::vector<void *> lk(copies), in(copies), out(copies);
    for (int k = 0; k < copies; k++) {
        if (k == 0) lk[k] = links_for(c, prec);
        else {
            CHK(wsget(c, S_BENCH + 3 * k, lbytes, &lk[k]));
            HIPCHK(hipMemcpyAsync(lk[k], lk[0], lbytes, hipMemcpyDeviceToDevice, c->st));
        }
        CHK(wsget(c, S_BENCH + 3 * k + 1, sbytes, &in[k]));
        CHK(wsget(c, S_BENCH + 3 * k + 2, sbytes, &out[k]));
        // deterministic, non-trivial input: copy the FP32 links' first reals
        HIPCHK(hipMemcpyAsync(in[k], c->U32, sbytes, hipMemcpyDeviceToDevice, c->st));
    }
    auto launch = [&](int k) -> int {
        HopLaunch L = hop_base(c, prec, P32);
        L.links = lk[k];
        L.mode = HOP;
        L.p = 0;
        L.in = in[k];
        L.out = out[k];
        HIPCHK(launch_hop(L, c->st));
        return WCL_OK;
    };
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
    HIPCHK(launch_dots(P64, 24 * Vh, 2, a, b, c->partials, nullptr, c->st));
    double part[4 * RED_BLOCKS];
    HIPCHK(hipMemcpyAsync(part, c->partials, sizeof(part), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    double yhx = 0.0, ycx = 0.0;
    for (int j = 0; j < RED_BLOCKS; j++) {
        yhx += part[0 * RED_BLOCKS + j];
        ycx += part[2 * RED_BLOCKS + j];
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
        c->pool.push_back(r.e0);
        c->pool.push_back(r.e1);
    }
    c->recs.clear();
    memset(c->stats, 0, sizeof(c->stats));
    c->prof = enable != 0;
    return WCL_OK;
}

extern "C" int wcl_profile_read(wcl_ctx *c, int kclass, wcl_kstat *out)
{
    if (!c || !out || kclass < 0 || kclass >= WCL_K_COUNT) return fail(WCL_EINVAL, "bad argument");
    HIPCHK(hipStreamSynchronize(c->st));
    for (auto &r : c->recs) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, r.e0, r.e1));
        wcl_kstat &k = c->stats[r.kclass];
        k.launches += 1;
        k.ms += ms;
        k.bytes += r.bytes;
        k.flops += r.flops;
        c->pool.push_back(r.e0);
        c->pool.push_back(r.e1);
    }
    c->recs.clear();
    *out = c->stats[kclass];
    return WCL_OK;
}

extern "C" int wcl_set_tuning(wcl_ctx *c, int hop_block, int hop_depth, int hop_xcd)
{
    if (!c) return fail(WCL_EINVAL, "null context");
    if (hop_block != 64 && hop_block != 128 && hop_block != 256) return fail(WCL_EINVAL, "hop_block must be 64, 128 or 256");
    if (hop_depth < 2 || hop_depth > 4) return fail(WCL_EINVAL, "hop_depth must be 2, 3 or 4");
    c->hop_block = hop_block;
    c->hop_depth = hop_depth;
    c->hop_xcd = hop_xcd ? 1 : 0;
    return WCL_OK;
}

extern "C" int wcl_autotune_hop(wcl_ctx *c, int prec, int copies, int *best)
{
    if (!c) return fail(WCL_EINVAL, "null context");
    const int blocks[3] = {64, 128, 256}, depths[3] = {2, 3, 4};
    double best_ms = 1e30;
    int bb = c->hop_block, bo = c->hop_depth, bx = c->hop_xcd;
    for (int xcd = 0; xcd < 2; xcd++)
        for (int ib = 0; ib < 3; ib++)
            for (int io = 0; io < 3; io++) {
                CHK(wcl_set_tuning(c, blocks[ib], depths[io], xcd));
                double ms;
                CHK(wcl_bench_hop(c, prec, 50, copies, &ms));
                if (ms < best_ms) { best_ms = ms; bb = blocks[ib]; bo = depths[io]; bx = xcd; }
            }
    CHK(wcl_set_tuning(c, bb, bo, bx));
    if (best) { best[0] = bb; best[1] = bo; best[2] = bx; }
    return WCL_OK;
}
