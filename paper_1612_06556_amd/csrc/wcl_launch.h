// wcl_launch.h -- host-side launchers of the library's kernels (internal).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <vector>

#include "wcl_common.h"

namespace wcl {

// Start / stop events of a timed launch.  ext_launch puts them into the
// kernel's own dispatch packet (no extra queue packets between kernels, the
// duration is the kernel's alone); null events launch untimed.
struct LaunchEvents {
    hipEvent_t start, stop;
};
template <typename... Params, typename... Args>
inline void ext_launch(void (*k)(Params...), dim3 grid, dim3 block, uint32_t shm, hipStream_t st,
                       const LaunchEvents &ev, Args... args)
{
    hipExtLaunchKernelGGL(k, grid, block, shm, st, ev.start, ev.stop, 0u, args...);
}

// Storage precision codes.  P32C / P16C: links as two rows (12 reals) in
// FP32 / FP16, clover in FP32 / FP16; spinors never use these codes.
enum Prec { P64 = 64, P32 = 32, P16 = 16, P32C = 33, P16C = 17 };

inline int prec_bytes(int prec) { return prec == P64 ? 8 : (prec == P32 || prec == P32C) ? 4 : 2; }
// bytes of one compressed link field (both parities, 4 directions)
inline size_t link_bytes_c(int prec, size_t Vh) { return prec == P32C ? 24 * 16 * Vh : (8 * 16 + 8 * 8) * Vh; }

// Epilogues of the hopping kernel; acc = H_{p,1-p} in (projectors swapped
// when dagger):
//   HOP      out = acc
//   CLOV_H   out = A acc                 (A = packed clover field, parity p)
//   XPAY     out = x + coef * A acc      (Schur second half)
//   CLOVX    out = A x + coef * acc      (one parity of the full operator)
enum HopMode { HOP = 0, CLOV_H = 1, XPAY = 2, CLOVX = 3 };

struct HopLaunch {
    const Geom *g;
    int link_prec;      // storage of links and clover
    int spin_prec;      // storage of in / out / x
    int mode;
    int dagger;
    int p;              // output parity
    const void *in;     // parity 1-p
    void *out;          // parity p
    const void *links;
    const void *clov;   // parity-major clover field (mode != HOP)
    const void *x;      // parity p (XPAY, CLOVX)
    double coef;
    int nrhs;           // right-hand sides, fields strided by *_stride bytes
    size_t in_stride, out_stride, x_stride;
    int xcd;            // XCD-aware workgroup order
    int block;          // threads per workgroup (64..256)
    int depth;          // hops whose operands are in flight per thread (2, 3)
    int nontemporal;    // links / clover loaded non-temporally (single right-hand side only)
    int lds_stage;      // 1: stage each 128-site tile's input spinors in LDS (block 128, 4^4 tiles)
    int tpw;            // consecutive site blocks per workgroup (0 or 1: one; at most 64)
    int rhs_per_thread; // 2 or 4: batched launches keep that many right-hand sides per thread
                        // (FP32 spinors, modes HOP / CLOV_H / XPAY); else one per workgroup
    const struct Scalars *sc;  // if non-null, the launch is a no-op once sc->done
    LaunchEvents ev;           // timing events of the launch (null: untimed)
    // fused reductions (mode XPAY, FP64 / FP32 / FP16 spinors, one right-hand side per
    // workgroup): ndot 1 writes the partials of <dotw, out> (terms 0, 1);
    // ndot 2 those of <out, dotw> (terms 0, 1) and <out, out> (term 2), per
    // workgroup at partials[rhs][term][block] (stride pstride)
    int ndot;
    const void *dotw;
    double *partials;
    int pstride;
};

hipError_t launch_hop(const HopLaunch &a, hipStream_t st);
// workgroups per right-hand side of a hop launch (the partials of a fused reduction)
int hop_parts(const HopLaunch &a);

// Algorithmic HBM bytes and flops of one hop launch (per the operator's
// definition: every link, the input spinor, the clover site and the output
// once; 1320 flop per hop site, 504 per clover site, 48 per fused axpy).
void hop_work(const HopLaunch &a, double *bytes, double *flops);
// Same for one RAS application (bytes: links and clover inverse of both
// parities, input and output once per even site; flops: the block hops,
// clover multiplications and minimal-residual vector work actually done).
void ras_work(const struct RasLaunch &a, double *bytes, double *flops);

// out = A in on parity p (A = clover field).
hipError_t launch_clover(const Geom &g, int link_prec, int spin_prec, int p, const void *clov,
                         const void *in, void *out, hipStream_t st, int nrhs = 1, size_t in_stride = 0,
                         size_t out_stride = 0, LaunchEvents ev = {});

// Canonical complex128 [V][4][3] <-> e/o FP64 field [2][12][Vh] double2.
hipError_t launch_pack_spinor(const Geom &g, const double *canon, void *eo, hipStream_t st);
hipError_t launch_unpack_spinor(const Geom &g, const void *eo, double *canon, hipStream_t st);
// Canonical U [V][4][3][3] -> internal link fields (any null pointer skipped).
hipError_t launch_ingest_gauge(const Geom &g, const double *canon, void *u64, void *u32, void *u16,
                               hipStream_t st);
// FP64 links -> two-row FP32 (P32C) and FP16 (P16C) link fields, and the
// per-site copy of the two-row FP32 links read by the fused Schwarz kernel.
hipError_t launch_compress_links(const Geom &g, const void *u64, void *u32c, void *u16c, void *u32s,
                                 hipStream_t st);
// Per-workgroup maxima of the SU(3) defect of the FP64 links (|row2 -
// conj(row0 x row1)|, |row norm - 1|, |<row0, row1>|) into partial[nblocks].
hipError_t launch_su3_check(const Geom &g, const void *u64, double *partial, int nblocks, hipStream_t st);
// Streaming probes over n16 float4 elements: copy = 0 reads a into one float
// per thread of out[blocks * 256]; copy = 1 copies a to b.
hipError_t launch_stream(int copy, const void *a, void *b, size_t n16, float *out, int blocks, hipStream_t st);
// Clover T and T^-1 (FP64 arithmetic) from the FP64 links, written in all
// three precisions.  info_dev[0] counts sites whose 6x6 block lost positive
// definiteness during inversion (a zero or negative pivot).
// fbuf: scratch of 6 * 9 * 2 Vh doubles (the field strength planes).
hipError_t launch_clover_build(const Geom &g, const void *u64, double csw_kappa, void *t64, void *ti64,
                               void *t32, void *ti32, void *t16, void *ti16, int *info_dev, double *fbuf,
                               hipStream_t st);

// Spinor precision conversion of nsites sites in sections of Vh sites (both
// layouts hold 12 complex per site): out = scale * in.  mode 0: scale =
// scale_host; mode 1: scale_host / sqrt(v); mode 2: scale_host * sqrt(v), with
// v = scale_dev[(section / sec_per_scale) * sdev_stride].
hipError_t launch_convert(int in_prec, int out_prec, size_t nsites, size_t Vh_in, size_t Vh_out,
                          const void *in, void *out, const double *scale_dev, int mode,
                          double scale_host, hipStream_t st, int sec_per_scale = 1, int sdev_stride = 0);

// ---------------------------------------------------------------------------
// Reductions and BLAS-1 on flat complex arrays (length n complex numbers).
// Partials are written per workgroup in double; finalisers combine them in
// a fixed order (bitwise reproducible).
constexpr int RED_BLOCKS = 512;
constexpr int RED_THREADS = 256;

// Solver scalars on the device (per right-hand side, FP64).
struct Scalars {
    double rho[2], rho_old[2], alpha[2], omega[2];
    double r2, b2, stop2;        // |r|^2, |b|^2 of the current right-hand side, stop threshold^2
    double scale;                // normalisation of the inner right-hand side
    double t[8];                 // spare scalars for reductions
    int done;                    // 1 converged, 2 breakdown
    int iter;
    int pad[2];
};

// dot partials: for each (a_k, b_k) pair listed, sum conj(a_k) b_k, per
// right-hand side (slices `stride` complex numbers apart); partials hold
// [nrhs][6][RED_BLOCKS] doubles.
hipError_t launch_dots(int prec, size_t n, int npairs, const void *const *a, const void *const *b,
                       double *partials, const Scalars *sc, hipStream_t st, int nrhs = 1, size_t stride = 0,
                       int pstride = RED_BLOCKS);

// BiCGStab building blocks (complex scalars taken from Scalars).
enum BicgStep {
    BICG_INIT_RHO = 0,   // rho = <rt, r>, r2 = |r|^2, b2 = r2, rho_old = alpha = omega = 1, iter = 0
    BICG_ALPHA = 1,      // alpha = rho / <rt, v>
    BICG_OMEGA = 2,      // omega = <t, s> / <t, t>
    BICG_RHO = 3,        // rho_old = rho; rho = <rt, r>; r2 = |r|^2; done if r2 <= stop2 b2
    NORM_ONLY = 4,       // t[0] = |v|^2
};
// pstride: doubles between the terms of one right-hand side's partials (6
// terms per right-hand side); nparts: partials per term to add.
hipError_t launch_finalize(int step, int nterms, const double *partials, Scalars *sc, hipStream_t st,
                           int nrhs = 1, const Scalars *gate = nullptr, int pstride = RED_BLOCKS,
                           int nparts = RED_BLOCKS);

// p = r + beta (p - omega v), beta = (rho/rho_old)(alpha/omega)
hipError_t launch_bicg_p(int prec, size_t n, const void *r, void *p, const void *v, const Scalars *sc,
                         hipStream_t st, int nrhs = 1, size_t stride = 0);
// s = r - alpha v
hipError_t launch_bicg_s(int prec, size_t n, const void *r, const void *v, void *s, const Scalars *sc,
                         hipStream_t st, int nrhs = 1, size_t stride = 0);
// x += alpha ph + omega sh ; r = s - omega t
hipError_t launch_bicg_xr(int prec, size_t n, void *x, const void *ph, const void *sh, void *r,
                          const void *s, const void *t, const Scalars *sc, hipStream_t st, int nrhs = 1,
                          size_t stride = 0);

// the same with the partials of <rt, r>, <r, r> of the new r per workgroup
// (terms 0..3 as for BICG_RHO); *nparts receives the workgroup count.
hipError_t launch_bicg_xr_dots(int prec, size_t n, void *x, const void *ph, const void *sh, void *r,
                               const void *s, const void *t, const void *rt, const Scalars *sc, hipStream_t st,
                               int nrhs, size_t stride, double *partials, int pstride, int *nparts);

// Generic complex axpby: y = a x + b y, a and b host constants.
hipError_t launch_axpby(int prec, size_t n, double2 a, const void *x, double2 b, void *y, hipStream_t st);
hipError_t launch_copy(int prec, size_t n, const void *x, void *y, hipStream_t st);
hipError_t launch_zero(int prec, size_t n, void *y, hipStream_t st);

// Overlapped RAS block solve: out_e = M in_e (FP32 arithmetic).
struct RasLaunch {
    const Geom *g;
    int overlap;
    int iters;
    int link_prec;
    const void *in;      // even field, FP32 (or FP16 when vec_prec == P16)
    void *out;           // even field, same storage
    const void *links;
    const void *links_site;   // two-row FP32 links per site (P32C, fused kernel), else unused
    const void *clov_inv;
    float kappa2;
    const Scalars *sc;   // may be null; per right-hand side, skips when done
    int nrhs;            // right-hand sides, fields `stride` bytes apart
    size_t stride;
    bool jacobi;         // block solver: false = minimal residual, true = z += r, r -= Dhat_B r
    int vec_prec;        // storage of in / out: 0 or P32, or P16 (with FP16 links and clover)
    int colour;          // 0: every block; k + 1: the blocks of colour k only (bit mu = parity of
                         // the block coordinate in direction mu)
    bool accumulate;     // add the restricted block results to out (else write them)
    LaunchEvents ev;     // timing events of the launch (null: untimed)
};
hipError_t launch_ras(const RasLaunch &a, hipStream_t st);

// The inner single-precision BiCGStab (right preconditioned by the fused
// additive RAS, minimal-residual blocks, or unpreconditioned) as one
// persistent cooperative launch: every iteration until each right-hand side
// has converged (scalars sc, initialised as after BICG_INIT_RHO with stop2
// set) or maxit iterations have run.  One workgroup per CU; partials holds
// PMAX_WG x PMAX_RHS x 4 doubles; bar (2 unsigned) and err (1 int) are the
// grid barrier's counters and time-out flag (reset by the launch).
constexpr int PMAX_WG = 1024;
constexpr int PMAX_RHS = 16;
struct PersistLaunch {
    const Geom *g;
    int link_prec, vec_prec;
    const void *links, *clov_inv;
    const void *links_site;   // per-site two-row FP32 links of the Schwarz phases (P32C)
    double kappa2;
    int use_ras, overlap, iters;
    bool jacobi;
    void *x, *r, *rt, *p, *v, *s, *t, *ph, *sh, *o;   // [nrhs] even fields, stride bytes apart
    size_t stride;
    Scalars *sc;
    double *partials;
    unsigned *bar;
    int *err;
    int nrhs, maxit, num_cus;
};
hipError_t launch_persist(const PersistLaunch &L, hipStream_t st);

// Schwarz block solves with the block vectors in global memory (any core
// size and overlap that fit the lattice; block solver 0 minimal residual,
// 1 Jacobi, 2 BiCGStab).  A plan holds the geometry tables and the block
// fields; the caller owns the device buffers (tables, vectors, state).
struct GrasPlan {
    int cores[4], overlap;
    int nblk, ne, nep;          // blocks; sites per parity of an extended block; ne padded to 64
    int nvec;                   // block fields held (4 for minimal residual / Jacobi, 8 for BiCGStab)
    const uint32_t *gm;         // [2][nblk][nep] global half index | t-boundary bits
    const uint32_t *nb;         // [2][nep][4] local neighbour indices (0xffff: outside)
    const uint8_t *core;        // [nep] even local site in the core
    float2 *vec[8];             // block fields [nblk][12][nep] FP32
    void *state;                // per-block solver state
};
int gras_fields(int solver);
// Whether the fused LDS kernel can hold the extended block of tile cores.
bool gras_fits_fused(const Geom &g, int overlap);
// Geometry of a plan (validates the cores) and the host image of its tables.
hipError_t gras_tables(const Geom &g, const int cores[4], int overlap, GrasPlan *P, std::vector<uint32_t> &host);
// Point the plan at its device buffers (tables as uploaded from the host image).
void gras_bind(GrasPlan *P, void *tables, void *vectors, void *state);
size_t gras_vector_bytes(const GrasPlan &P);
size_t gras_state_bytes(const GrasPlan &P);
// One Schwarz application out_e = M in_e over every right-hand side of L
// (additive only: L.colour == 0, L.accumulate false).
hipError_t launch_gras(const GrasPlan &P, const RasLaunch &L, int solver, hipStream_t st);
void gras_work(const GrasPlan &P, const RasLaunch &L, int solver, double *bytes, double *flops);

// Gradient (FP64): K field [2][6][9][Vh] double2 scratch, G = link field.
hipError_t launch_grad(const Geom &g, const void *u64, const void *X, const void *Y, void *K, double kappa,
                       double csw, void *G, hipStream_t st);
// out = sum_{mu<nu} sigma_{mu nu} F_{mu nu} X (both parities, FP64, from the links)
hipError_t launch_sigmaF(const Geom &g, const void *u64, const void *X, void *out, hipStream_t st);
hipError_t launch_export_links(const Geom &g, const void *G, double *canon, hipStream_t st);
// gamma5 on nsec FP64 e/o sections of Vh sites (in place)
hipError_t launch_gamma5(size_t nsec, size_t Vh, void *f, hipStream_t st);
int ras_threads(const Geom &g, int overlap);

}  // namespace wcl
