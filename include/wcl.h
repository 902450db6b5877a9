/*
 * wcl.h -- C ABI of the MI355X Wilson-Clover library (libwcl.so).
 *
 * What it computes (Boku et al., "A performance evaluation of CCS QCD
 * Benchmark on the COMA system", LATTICE2016):
 *   - the Wilson-Clover quark matrix D = T - kappa H, whose hopping matrix
 *     multiplication H is the measured kernel (Sec. 3) and whose inverse on a
 *     source is the quark propagator (Sec. 1);
 *   - its solution D x = b by an FP64 flexible BiCGStab preconditioned with a
 *     single-precision BiCGStab, itself preconditioned by even/odd sites and
 *     overlapped Restricted Additive Schwarz (Sec. 2); the paper's offload
 *     entry point takes kappa, a stopping tolerance, an in/out iteration count,
 *     a read-only source and a written solution (Sec. 2, Fig. "Offloading part
 *     in the host CPU code") -- the same roles as wcl_solve's arguments here.
 *
 * Conventions
 *   Lattice  dims = {Lx, Ly, Lz, Lt}, every extent even and >= 4; site
 *            n = x + Lx*(y + Ly*(z + Lz*t)); parity (x+y+z+t) mod 2.
 *   Gauge    U: complex128 [V][4][3][3]; U[n][mu] is the link from site n in
 *            direction mu (x, y, z, t), a row-major 3x3 matrix.  The caller
 *            passes the physical links; the t boundary condition is applied by
 *            the library as a sign on the hops that cross t = Lt-1 <-> 0.
 *   Spinor   complex128 [nrhs][V][4][3] ([spin][colour]), chiral gamma basis:
 *            gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] (k = x, y, z),
 *            gamma_t = [[0, 1], [1, 0]], gamma_5 = diag(1, 1, -1, -1).
 *   Operator (H psi)(x) = sum_mu (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                               + (1 + gamma_mu) U_mu(x-mu)^dag psi(x-mu),
 *            T = 1 - c_sw kappa sum_{mu<nu} sigma_{mu nu} F_{mu nu},
 *            sigma_{mu nu} = (i/2)[gamma_mu, gamma_nu], F = (Q - Q^dag)/(8i)
 *            made traceless, Q the four plaquette leaves; D^dag = g5 D g5.
 *   Pointers marked _dev are device pointers (HIP) on the context's device;
 *            every user buffer stays owned by the caller and is not retained
 *            after the call returns.  All work is ordered on the context's
 *            stream; calls return once the results are complete on that
 *            stream (wcl_apply / wcl_apply_op / wcl_set_* do not block the host;
 *            wcl_solve synchronises for its convergence tests).
 *   Errors   every call returns WCL_OK (0) or a negative code; the message of
 *            the last failure on the calling thread is wcl_last_error().
 */
#ifndef WCL_H
#define WCL_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wcl_ctx wcl_ctx;

enum {
    WCL_OK = 0,
    WCL_EINVAL = -1,      /* bad argument (shape, pointer, option)               */
    WCL_ENOMEM = -2,      /* device allocation failed                            */
    WCL_EHIP = -3,        /* a HIP runtime call or kernel launch failed          */
    WCL_ENOCONV = -4,     /* solver hit its iteration limit; x holds the iterate */
    WCL_EBREAKDOWN = -5,  /* BiCGStab breakdown (vanishing rho, <r~,v> or omega)  */
    WCL_ENAN = -6,        /* NaN / Inf in the data                               */
    WCL_ESTATE = -7       /* apply / solve before wcl_set_gauge + wcl_set_params */
};

/* Storage precision of links, clover and vectors in wcl_apply / wcl_apply_op. */
enum { WCL_PREC64 = 64, WCL_PREC32 = 32, WCL_PREC16 = 16 };

/* Create a context for one lattice on the current HIP device (the paper's
 * solver holds its gauge and clover fields resident on the card between
 * calls, Sec. 2; here that state is explicit and owned by the context).
 * tile: extents of the internal blocked layout and of the Schwarz cores
 * (each even and dividing dims[mu]); NULL picks 4^4 when it divides the
 * lattice, else 2^4.  Not in the paper (layout): 4^4 suits the fused
 * Schwarz kernel and repeated (cache-resident) hops; tiles spanning whole
 * x-rows (e.g. 24x4x8x4 on 24^3x32) make single-use hops faster, and a
 * Schwarz solve on them needs explicit cores (wcl_set_ras_cores).  t_bc = +1 periodic, -1 antiperiodic in time.
 * hip_stream: a hipStream_t (NULL = the null stream).  *out receives the
 * context, owned by the caller until wcl_destroy.  Errors: WCL_EINVAL
 * (also for more than 7,456,540 sites: fields are addressed with 32-bit byte
 * offsets, and the FP64 links take 576 bytes a site); WCL_ENOMEM / WCL_EHIP
 * when the context's first device buffers fail. */
int wcl_create(const int dims[4], int t_bc, const int tile[4], void *hip_stream, wcl_ctx **out);
/* Switch the stream every later call of this context is ordered on. */
int wcl_set_stream(wcl_ctx *ctx, void *hip_stream);
/* Copy and convert the gauge field U (the links of the Wilson-Clover matrix,
 * Sec. 1) into the context's FP64, FP32 and FP16 copies in the blocked
 * even/odd layout; the caller's buffer is read on the stream and not kept.
 * Invalidates kappa / c_sw (call wcl_set_params again).  Errors:
 * WCL_EINVAL (null), WCL_ENOMEM, WCL_EHIP, and with two-row storage on the
 * SU(3) check below. */
int wcl_set_gauge(wcl_ctx *ctx, const double *U_dev);
/* Set kappa and c_sw of the Wilson-Clover matrix (Sec. 1; kappa is also an
 * argument of the paper's offloaded solver, Sec. 2); (re)builds the clover
 * term T and T^-1 per site in FP64 (then stored in FP64, FP32 and FP16), the
 * blocks the even/odd preconditioning divides by.  Synchronises the stream.
 * WCL_ESTATE before wcl_set_gauge; WCL_EINVAL for non-finite values;
 * WCL_ENAN if a clover block is not positive definite. */
int wcl_set_params(wcl_ctx *ctx, double kappa, double csw);

/* Two-row (12-real) link storage for the FP32 and FP16 tiers (enable 1) or
 * full 3x3 links (0, the default): the SU(3) reconstruction the paper's
 * single-precision solver uses (Sec. 2; it keeps two columns, here two
 * rows).  An SU(3) matrix is fixed by its first two rows (row 2 =
 * conj(row0 x row1)), so the hopping and Schwarz kernels read 48 (FP32) or
 * 24 (FP16) bytes per link instead of 72 / 36 and rebuild the third row in
 * registers; FP64 work always uses the full links.  The context then holds
 * the FP32 two-row links twice (field-major for the hopping kernels, per site
 * for the Schwarz block solves: 384 bytes a site each) and the FP16 ones
 * once.  Enabling
 * checks, on the current and every later wcl_set_gauge, that each link is
 * SU(3) to 1e-7 (row norms, row orthogonality, row 2 against the cross
 * product); otherwise the call fails with WCL_EINVAL and, in wcl_set_gauge,
 * the context has no gauge field until the next successful call.  With
 * compression on, wcl_set_gauge synchronises the stream for that check. */
int wcl_set_compression(wcl_ctx *ctx, int enable);

/* out = D in (dagger = 0) or D^dag in (dagger = 1) on nrhs full-lattice
 * spinors: the Wilson-Clover quark matrix whose hopping part is the paper's
 * measured "MULT" kernel (Sec. 2, Sec. 3).  Computed with links, clover and
 * vectors stored in prec (64; 32: FP32 storage and arithmetic; 16: FP16
 * storage, FP32 arithmetic).  in_dev / out_dev: complex128
 * [nrhs][V][4][3] device buffers owned by the caller; they must not
 * overlap.  WCL_ESTATE before wcl_set_params; WCL_EINVAL for nrhs < 1, an
 * unknown prec or a null pointer; WCL_ENOMEM when the context's workspace
 * cannot grow (it is allocated on first use and kept). */
int wcl_apply(wcl_ctx *ctx, const double *in_dev, double *out_dev, int nrhs, int dagger, int prec);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): wcl_apply
 * without any allocation.  Same arguments, layouts, ownership, results and
 * errors as wcl_apply (the same kernels run in the same order), but its
 * temporaries live in a fixed scratch array of 64 MiB per GPU that the
 * library holds until the process ends, and it records no profiling events:
 * lattices of at most 174762 sites (e.g. 8^4, 16^3x32) -- larger ones fail
 * with WCL_EINVAL; right-hand sides are processed one after another.  Every
 * call on one GPU uses that GPU's one scratch array, so calls that overlap on
 * one GPU (other streams or host threads) race and must be serialised by
 * the caller.  The context's resident fields come from wcl_set_gauge and
 * wcl_set_params, which do allocate. */
int wcl_apply_noalloc(wcl_ctx *ctx, const double *in_dev, double *out_dev, int nrhs, int dagger, int prec);

/* One step of the hot path on canonical FP64 vectors, for per-step checks of
 * the even/odd preconditioned matrix and its RAS preconditioner (Sec. 2);
 * same buffer rules and errors as wcl_apply, and WCL_EINVAL for an unknown
 * op, RAS at prec 64 and SCHUR_RHS below prec 64:
 *   WCL_OP_HOP        out = H in                      (both parities)
 *   WCL_OP_CLOVER     out = T in
 *   WCL_OP_CLOVER_INV out = T^-1 in
 *   WCL_OP_SCHUR      out_e = Dhat in_e, out_o = 0, Dhat = 1 - k^2 T_ee^-1 H_eo T_oo^-1 H_oe
 *   WCL_OP_SCHUR_RHS  out_e = T_ee^-1 (in_e + k H_eo T_oo^-1 in_o), out_o = 0
 *   WCL_OP_RAS        out_e = M in_e, out_o = 0   (one RAS application; prec 32 or 16,
 *                     overlap, iterations and block solver from the last wcl_set_ras,
 *                     default 1, 4 and minimal residual)
 *   WCL_OP_D / WCL_OP_DDAG as wcl_apply.                                   */
enum { WCL_OP_HOP = 0, WCL_OP_CLOVER = 1, WCL_OP_CLOVER_INV = 2, WCL_OP_SCHUR = 3,
       WCL_OP_SCHUR_RHS = 4, WCL_OP_RAS = 5, WCL_OP_D = 6, WCL_OP_DDAG = 7 };
int wcl_apply_op(wcl_ctx *ctx, int op, const double *in_dev, double *out_dev, int nrhs, int prec);
/* Schwarz settings of WCL_OP_RAS (a solve sets them from its options):
 * overlap (extension of the cores on every side), iters (block steps), the
 * block solver -- WCL_RAS_MR, minimal residual from zero (the default),
 * WCL_RAS_JACOBI, the linear alternative z <- z + (r_B - Dhat_B z), or
 * WCL_RAS_BICGSTAB, `iters` BiCGStab iterations (two block applications
 * each) from zero -- and the scheme: multiplicative = 0 is the additive
 * (restricted) Schwarz of the paper; 1 runs the 16 block colours (parities
 * of the block coordinates) in turn, each on the residual in - Dhat z left by
 * the colours before it (the paper leaves the Schwarz variant open, Sec. 2).
 * The cores are the layout's tiles unless wcl_set_ras_cores set others.
 * Tile cores with MR or Jacobi and an extended block of at most 648 sites
 * per parity run as one fused kernel (block vectors in LDS); every other
 * setting runs the block solves with the block vectors in device memory
 * (the context allocates them here: 8 or 4 FP32 fields of the extended
 * blocks' size, with BiCGStab or not).  WCL_EINVAL when the extended block
 * does not fit the lattice, for an unknown solver, and for multiplicative
 * Schwarz outside the fused kernel's settings; the settings then stay. */
enum { WCL_RAS_MR = 0, WCL_RAS_JACOBI = 1, WCL_RAS_BICGSTAB = 2 };
int wcl_set_ras(wcl_ctx *ctx, int overlap, int iters, int solver, int multiplicative);
/* Schwarz cores (paper Sec. 2 leaves their size open): cores[mu] even,
 * dividing L[mu], with L[mu] >= cores[mu] + 2 overlap; cores = NULL or all
 * zero restores the tiles.  Explicit cores, even equal to the tiles, select
 * the device-memory block path (additive Schwarz only).  WCL_EINVAL
 * otherwise, leaving the cores as they were. */
int wcl_set_ras_cores(wcl_ctx *ctx, const int cores[4]);

/* Solver options. */
/* FBICGSTAB: FP64 flexible BiCGStab on the even/odd system, preconditioned
 * by the inner single-precision solve (Sec. 2); DC: defect correction with the
 * same inner solve; PLAIN64: unpreconditioned FP64 BiCGStab on the full D;
 * PLAIN64_EO: unpreconditioned FP64 BiCGStab on the even/odd system. */
enum { WCL_OUTER_FBICGSTAB = 0, WCL_OUTER_DC = 1, WCL_OUTER_PLAIN64 = 2, WCL_OUTER_PLAIN64_EO = 3 };
typedef struct {
    double tol;          /* stop when ||b - D x|| / ||b|| <= tol (true FP64 residual) */
    int max_outer;       /* outer iterations (PLAIN64*: BiCGStab iterations)         */
    int max_inner;       /* inner iterations per preconditioner call                 */
    double inner_tol;    /* inner relative residual                                  */
    int outer;           /* WCL_OUTER_*                                              */
    int use_ras;         /* RAS preconditioning of the inner solver                  */
    int ras_overlap;     /* extension of the cores (the tile) on every side          */
    int ras_iters;       /* minimal-residual steps per block solve                   */
    int inner_prec;      /* 32: FP32 links/clover; 16: FP16 links/clover (FP32 math) */
    int use_graph;       /* replay the inner iteration as a captured hipGraph        */
    int check_every;     /* inner iterations between host convergence checks         */
    int adjoint;         /* 1: solve D^dag x = b instead, as x = g5 D^-1 (g5 b)      */
    int ras_solver;      /* WCL_RAS_MR, WCL_RAS_JACOBI or WCL_RAS_BICGSTAB (RAS block solver) */
    int inner_vec_prec;  /* 32, or 16: the inner solver's vectors stored in FP16 (FP32
                          * arithmetic; needs inner_prec 16)                        */
    int ras_mult;        /* 1: multiplicative Schwarz (colour sweeps), see wcl_set_ras */
    int persistent;      /* 1: each inner solve runs as one persistent cooperative kernel
                          * (every inner iteration, reductions and convergence test on
                          * the device; FBICGSTAB / DC, additive Schwarz on the fused
                          * kernel or no Schwarz, one or more right-hand sides)      */
    const double *x0_dev; /* NULL: zero start.  Else an initial guess, complex128
                          * [nrhs][V][4][3] on the device (the paper's solver takes the
                          * solution vector in and out, Sec. 2); its even sites start
                          * the even/odd solvers, the whole field the full-D solver */
    int ras_block[4];    /* Schwarz cores (with use_ras): all 0 keeps the context's
                          * (the tiles, or wcl_set_ras_cores); else set as by
                          * wcl_set_ras_cores for this and later solves           */
} wcl_solve_opts;

typedef struct {
    int outer_iters;       /* outer iterations (PLAIN64: BiCGStab iterations) */
    int inner_iters_total; /* inner BiCGStab iterations over all calls        */
    int status;            /* WCL_OK / WCL_ENOCONV / WCL_EBREAKDOWN / WCL_ENAN */
    int pad;
    double true_relres;    /* ||b - D x|| / ||b|| in FP64 at return           */
    double seconds;        /* wall time of the solve                          */
} wcl_solve_info;

/* Fill opts with the defaults: tol 1e-10, FBICGSTAB, RAS on (overlap 1,
 * 4 iterations, minimal residual), inner_tol 1e-2, FP32 inner links and
 * vectors, 100 outer, 500 inner, zero start, launch-per-kernel inner solve. */
void wcl_default_opts(wcl_solve_opts *opts);

/* Solve D x = b (the quark propagator, Sec. 1) for nrhs right-hand sides by
 * the paper's FP64 flexible BiCGStab over the single-precision BiCGStab with
 * even/odd and overlapped RAS preconditioning (Sec. 2), or by the variants
 * selected in opts.  All right-hand sides advance in lockstep through the
 * same launches (per-rhs scalars; a converged right-hand side is masked out).
 * b_dev, x_dev: complex128 [nrhs][V][4][3], caller-owned, must not overlap;
 * x_dev is written; opts->x0_dev (may alias x_dev) is the initial guess or
 * NULL for zero.  info (nrhs entries, may be NULL) receives per-rhs results.
 * Returns the worst status: WCL_ENOCONV (x holds the best iterate),
 * WCL_EBREAKDOWN (BiCGStab broke down on the last restart allowed), WCL_ENAN,
 * WCL_EINVAL for bad options, WCL_ESTATE before wcl_set_params. */
int wcl_solve(wcl_ctx *ctx, const double *b_dev, double *x_dev, int nrhs, const wcl_solve_opts *opts,
              wcl_solve_info *info);

/* Not in the paper: the differentiation workload this library adds around
 * the solve.  Gradient of L = Re<eta, D^-1 b> from x = D^-1 b and
 * y = D^-dag eta (both canonical FP64 device spinors, caller-owned):
 * gU_dev[V][4][3][3] complex128 receives 2 dL/d conj(U) (PyTorch's
 * convention), *gkappa_host dL/dkappa.  Synchronises the stream.
 * WCL_ESTATE before wcl_set_params; WCL_EINVAL for null pointers. */
int wcl_grad(wcl_ctx *ctx, const double *x_dev, const double *y_dev, double *gU_dev, double *gkappa_host);

/* Time the standalone even/odd hopping kernel H_eo, the paper's measured
 * "MULT" (Sec. 3), on nrhs right-hand sides per launch (FP32 or FP16 links,
 * two-row when compression is on; FP32 spinors; nrhs > 1 uses the batched
 * launch shape of wcl_set_batch_tuning): `reps` launches after 10 warm-ups,
 * rotating over `copies` independent sets of links and spinors (1 <= copies
 * <= 32; more copies defeat the 256 MB Infinity Cache).  *ms_per_call
 * receives the mean launch time from HIP events.  Buffers come from the
 * context's workspace.  WCL_ESTATE before wcl_set_gauge; WCL_EINVAL for
 * other precisions, nrhs outside 1..64 or bad counts. */
int wcl_bench_hop(wcl_ctx *ctx, int prec, int nrhs, int reps, int copies, double *ms_per_call);
/* Time the standalone clover apply out_e = T_ee^-1 in_e (FP32 or FP16
 * clover, FP32 spinors), the 504-flop-per-site part of the even/odd
 * preconditioned matrix (Sec. 2), with the protocol of wcl_bench_hop for
 * one right-hand side.  WCL_ESTATE before wcl_set_params. */
int wcl_bench_clover(wcl_ctx *ctx, int prec, int reps, int copies, double *ms_per_call);

/* Not in the paper (measurement): streaming ceilings of the device, for the
 * roofline: the mean rate of a
 * read-only pass and of a copy over two buffers of `mib` MiB each (context
 * workspace; `reps` launches after 10 warm-ups).  *read_gbs = bytes read per
 * second, *copy_gbs = bytes read + written per second, in GB/s. */
int wcl_bench_stream(wcl_ctx *ctx, double mib, int reps, double *read_gbs, double *copy_gbs);

/* Not in the paper (measurement): kernel-class profiling on the context's
 * stream: with profiling enabled,
 * every launch of the classes below is timed by HIP events (carried in the
 * kernel's dispatch packet for the single-kernel hop, RAS and clover
 * launches; recorded around multi-kernel launches) and its
 * algorithmic HBM bytes and flops are recorded (1320 flop per hop site,
 * 504 per clover site; bytes = each link, clover site and vector once).
 * WCL_K_INNER holds the persistent inner-solve launches (opts.persistent),
 * timed by events around the launch, with the work of the iterations they
 * ran (their Schur, Schwarz and vector work by the rules above).
 * wcl_profile(ctx, 1) clears and starts, (ctx, 0) stops; wcl_profile_read
 * synchronises the stream and returns the totals of one class. */
enum { WCL_K_HOP = 0, WCL_K_RAS = 1, WCL_K_CLOVER = 2, WCL_K_INNER = 3, WCL_K_COUNT = 4 };
typedef struct {
    int launches;        /* launches that did work                            */
    int idle_launches;   /* launches queued after convergence (no-ops)        */
    double ms;           /* summed event time of the working launches         */
    double bytes;        /* summed algorithmic HBM bytes                      */
    double flops;        /* summed flops (conventions above)                  */
    double idle_ms;      /* summed event time of the no-op launches           */
} wcl_kstat;
int wcl_profile(wcl_ctx *ctx, int enable);
int wcl_profile_read(wcl_ctx *ctx, int kclass, wcl_kstat *out);
/* Classes whose launches carry timing events while profiling (bit k = class
 * WCL_K_k; default all).  Every profiled launch costs a few microseconds of
 * queue time for its events; launches of the other classes are still counted
 * (launches, bytes, flops) with ms = 0.  WCL_EINVAL for other bits. */
int wcl_profile_mask(wcl_ctx *ctx, int mask);

/* Not in the paper (tuning; the paper tunes its KNC kernel by loop blocking
 * and prefetching, Sec. 2).  Launch configuration of the hopping kernel:
 * threads per workgroup (64, 128,
 * 256), pipeline depth (2, 3: hops of a site whose neighbour spinor and
 * link are in flight while an earlier hop is computed), XCD-aware workgroup
 * order (0/1) and non-temporal link/clover loads (0/1; single right-hand
 * side only).  wcl_autotune_hop times every block/depth/xcd combination with
 * wcl_bench_hop (prec, `copies` field sets) and keeps the fastest; best[3]
 * (may be NULL) receives {block, depth, xcd}. */
int wcl_set_tuning(wcl_ctx *ctx, int hop_block, int hop_depth, int hop_xcd, int hop_nontemporal);
int wcl_autotune_hop(wcl_ctx *ctx, int prec, int copies, int *best);
/* Staged input of the hopping kernel (default on): each workgroup first
 * copies the input spinors of its own half-sites into LDS and reads the
 * neighbours that fall in that range from there (in the blocked layout most
 * of a tile's hops stay inside the tile), the rest from global memory.
 * Applies to depth-2, non-dagger launches (temporal or non-temporal operator
 * loads); results are bitwise those of the unstaged kernel.  enable = 0 switches it off. */
int wcl_set_hop_staging(wcl_ctx *ctx, int enable);
/* Not in the paper (tuning).  The project autotuner: picks, by measurement,
 *   (flags & WCL_TUNE_HOP)    the hopping kernel's launch shape -- threads per
 *                             workgroup 64/128/256, pipeline depth 2/3, XCD
 *                             order 0/1, site blocks per workgroup 1/2 -- timed
 *                             with wcl_bench_hop at `prec` on nrhs right-hand
 *                             sides (4 field copies);
 *   (flags & WCL_TUNE_BATCH)  right-hand sides per thread 1/2/4 of the batched
 *                             launches (nrhs > 1);
 *   (flags & WCL_TUNE_SCHWARZ) the Schwarz choice of the solve opts describes
 *                             -- its own overlap, overlap 0, or no Schwarz --
 *                             by the measured time of wcl_solve(b_dev, opts)
 *                             (b_dev: nrhs canonical sources; needs opts);
 * every candidate being a shape the library's parity tests cover.  The
 * chosen launch shapes are set in the context; the Schwarz choice is
 * returned in *out (use_ras, ras_overlap) for the caller's opts.  Results
 * are cached per process, keyed by lattice, boundary condition, tiles,
 * precision, link storage, nrhs, flags and the hop's load policy (non-temporal
 * loads, LDS staging: candidates are timed with the context's current ones)
 * (out->cached = 1 on a hit, the
 * shapes are then set without timing).  WCL_EINVAL for bad arguments. */
enum { WCL_TUNE_HOP = 1, WCL_TUNE_BATCH = 2, WCL_TUNE_SCHWARZ = 4 };
typedef struct {
    int hop_block;        /* hopping launch shape: threads per workgroup        */
    int hop_depth;        /*   pipeline depth                                   */
    int hop_xcd;          /*   XCD-aware workgroup order                        */
    int hop_tiles;        /*   site blocks per workgroup                        */
    int rhs_per_thread;   /* batched launches                                   */
    int use_ras;          /* Schwarz choice: on / off                           */
    int ras_overlap;      /*   extension of the cores                          */
    int cached;           /* 1: the result came from the cache                  */
    double hop_ms;        /* launch time of the chosen hop shape (ms)          */
    double solve_ms;      /* time of the solve with the chosen Schwarz (ms)    */
} wcl_tuning;
int wcl_autotune(wcl_ctx *ctx, int prec, int nrhs, const double *b_dev, const wcl_solve_opts *opts, int flags,
                 wcl_tuning *out);
/* Consecutive site blocks (of the workgroup size) each hop workgroup takes
 * in turn (1, 2, 4 or 8; default 1): fewer, longer-lived workgroups, each
 * sweeping one contiguous range of every field.  Results are bitwise those
 * of one block per workgroup.  WCL_EINVAL for other values. */
int wcl_set_hop_tiles(wcl_ctx *ctx, int tiles);
/* Batched launches (nrhs > 1) of the FP32-vector hopping kernels (the inner
 * solver's Schur halves): rhs_per_thread = 1 gives each right-hand side its
 * own workgroups (links shared through L2); 2 or 4 keep that many right-hand
 * sides in one thread's registers, so every link and clover block loaded
 * serves all of them.  WCL_EINVAL for other values. */
int wcl_set_batch_tuning(wcl_ctx *ctx, int rhs_per_thread);

/* Message of the last failure on the calling thread (never NULL; owned by
 * the library, valid until the thread's next failing call). */
const char *wcl_last_error(void);
/* Synchronise the context's stream and free every device buffer it owns;
 * NULL is accepted.  Always WCL_OK. */
int wcl_destroy(wcl_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
