"""Thin ctypes binding of ``libwcl.so`` (the C ABI declared in ``include/wcl.h``).

Argument marshalling only: every step of the path runs in the HIP kernels of
the library.  PyTorch provides the device memory (complex128 CUDA tensors) and
the stream.  The module-level functions carry the C names; ``Lattice`` is a
convenience wrapper around one context.

The library must be built (``paper_1612_06556_amd/build.py``); there is no
fallback: loading fails loudly when ``libwcl.so`` is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwcl.so")

WCL_OK, WCL_EINVAL, WCL_ENOMEM, WCL_EHIP, WCL_ENOCONV, WCL_EBREAKDOWN, WCL_ENAN, WCL_ESTATE = (
    0, -1, -2, -3, -4, -5, -6, -7)
OP_HOP, OP_CLOVER, OP_CLOVER_INV, OP_SCHUR, OP_SCHUR_RHS, OP_RAS, OP_D, OP_DDAG = range(8)
OUTER_FBICGSTAB, OUTER_DC, OUTER_PLAIN64, OUTER_PLAIN64_EO = 0, 1, 2, 3
RAS_MR, RAS_JACOBI, RAS_BICGSTAB = 0, 1, 2


class WclError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"wcl error {code}: {msg}")
        self.code = code


class wcl_solve_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_outer", ctypes.c_int), ("max_inner", ctypes.c_int),
                ("inner_tol", ctypes.c_double), ("outer", ctypes.c_int), ("use_ras", ctypes.c_int),
                ("ras_overlap", ctypes.c_int), ("ras_iters", ctypes.c_int), ("inner_prec", ctypes.c_int),
                ("use_graph", ctypes.c_int), ("check_every", ctypes.c_int), ("adjoint", ctypes.c_int),
                ("ras_solver", ctypes.c_int), ("inner_vec_prec", ctypes.c_int), ("ras_mult", ctypes.c_int),
                ("persistent", ctypes.c_int), ("x0_dev", ctypes.c_void_p), ("ras_block", ctypes.c_int * 4)]


class wcl_solve_info(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int), ("inner_iters_total", ctypes.c_int),
                ("status", ctypes.c_int), ("pad", ctypes.c_int), ("true_relres", ctypes.c_double),
                ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


class wcl_tuning(ctypes.Structure):
    _fields_ = [("hop_block", ctypes.c_int), ("hop_depth", ctypes.c_int), ("hop_xcd", ctypes.c_int),
                ("hop_tiles", ctypes.c_int), ("rhs_per_thread", ctypes.c_int), ("use_ras", ctypes.c_int),
                ("ras_overlap", ctypes.c_int), ("cached", ctypes.c_int), ("hop_ms", ctypes.c_double),
                ("solve_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


TUNE_HOP, TUNE_BATCH, TUNE_SCHWARZ = 1, 2, 4


class wcl_kstat(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int), ("idle_launches", ctypes.c_int), ("ms", ctypes.c_double),
                ("bytes", ctypes.c_double), ("flops", ctypes.c_double), ("idle_ms", ctypes.c_double)]


K_HOP, K_RAS, K_CLOVER, K_INNER = 0, 1, 2, 3

_lib = None
_ip = ctypes.POINTER(ctypes.c_int)
_vp = ctypes.c_void_p


def load():
    """Load libwcl.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1612_06556_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    lib.wcl_last_error.restype = ctypes.c_char_p
    lib.wcl_create.argtypes = [_ip, ctypes.c_int, _ip, _vp, ctypes.POINTER(_vp)]
    lib.wcl_set_stream.argtypes = [_vp, _vp]
    lib.wcl_set_gauge.argtypes = [_vp, _vp]
    lib.wcl_set_params.argtypes = [_vp, ctypes.c_double, ctypes.c_double]
    lib.wcl_set_ras.argtypes = [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.wcl_set_ras_cores.argtypes = [_vp, _ip]
    lib.wcl_apply.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.wcl_apply_op.argtypes = [_vp, ctypes.c_int, _vp, _vp, ctypes.c_int, ctypes.c_int]
    lib.wcl_apply_noalloc.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.wcl_default_opts.argtypes = [ctypes.POINTER(wcl_solve_opts)]
    lib.wcl_default_opts.restype = None
    lib.wcl_solve.argtypes = [_vp, _vp, _vp, ctypes.c_int, ctypes.POINTER(wcl_solve_opts),
                              ctypes.POINTER(wcl_solve_info)]
    lib.wcl_grad.argtypes = [_vp, _vp, _vp, _vp, ctypes.POINTER(ctypes.c_double)]
    lib.wcl_bench_hop.argtypes = [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_double)]
    lib.wcl_bench_clover.argtypes = [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.wcl_destroy.argtypes = [_vp]
    lib.wcl_profile.argtypes = [_vp, ctypes.c_int]
    lib.wcl_profile_read.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(wcl_kstat)]
    lib.wcl_profile_mask.argtypes = [_vp, ctypes.c_int]
    lib.wcl_set_tuning.argtypes = [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.wcl_autotune_hop.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _ip]
    lib.wcl_set_hop_staging.argtypes = [_vp, ctypes.c_int]
    lib.wcl_set_hop_tiles.argtypes = [_vp, ctypes.c_int]
    lib.wcl_autotune.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.POINTER(wcl_solve_opts), ctypes.c_int,
                                 ctypes.POINTER(wcl_tuning)]
    lib.wcl_set_compression.argtypes = [_vp, ctypes.c_int]
    lib.wcl_set_batch_tuning.argtypes = [_vp, ctypes.c_int]
    lib.wcl_bench_stream.argtypes = [_vp, ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]
    _lib = lib
    return lib


def _check(rc):
    if rc != WCL_OK:
        raise WclError(rc, load().wcl_last_error().decode())
    return rc


def _ivec(v):
    return (ctypes.c_int * 4)(*[int(t) for t in v])


# --- C-named wrappers --------------------------------------------------------

def wcl_create(dims, t_bc=-1, tile=None, stream=None):
    h = _vp()
    _check(load().wcl_create(_ivec(dims), int(t_bc), _ivec(tile) if tile is not None else None,
                             _vp(stream or 0), ctypes.byref(h)))
    return h


def wcl_set_stream(h, stream):
    _check(load().wcl_set_stream(h, _vp(stream or 0)))


def wcl_set_gauge(h, U_ptr):
    _check(load().wcl_set_gauge(h, _vp(U_ptr)))


def wcl_set_compression(h, enable):
    _check(load().wcl_set_compression(h, int(enable)))


def wcl_set_params(h, kappa, csw):
    _check(load().wcl_set_params(h, float(kappa), float(csw)))


def wcl_set_ras(h, overlap, iters, solver=0, multiplicative=0):
    _check(load().wcl_set_ras(h, int(overlap), int(iters), int(solver), int(multiplicative)))


def wcl_set_ras_cores(h, cores):
    arr = None if cores is None else (ctypes.c_int * 4)(*[int(c) for c in cores])
    _check(load().wcl_set_ras_cores(h, arr))


def wcl_apply(h, in_ptr, out_ptr, nrhs, dagger, prec):
    _check(load().wcl_apply(h, _vp(in_ptr), _vp(out_ptr), int(nrhs), int(dagger), int(prec)))


def wcl_apply_noalloc(h, in_ptr, out_ptr, nrhs, dagger, prec):
    _check(load().wcl_apply_noalloc(h, _vp(in_ptr), _vp(out_ptr), int(nrhs), int(dagger), int(prec)))


def wcl_apply_op(h, op, in_ptr, out_ptr, nrhs, prec):
    _check(load().wcl_apply_op(h, int(op), _vp(in_ptr), _vp(out_ptr), int(nrhs), int(prec)))


def wcl_default_opts():
    o = wcl_solve_opts()
    load().wcl_default_opts(ctypes.byref(o))
    return o


def wcl_solve(h, b_ptr, x_ptr, nrhs, opts, raise_on_error=True):
    infos = (wcl_solve_info * nrhs)()
    rc = load().wcl_solve(h, _vp(b_ptr), _vp(x_ptr), int(nrhs), ctypes.byref(opts), infos)
    if raise_on_error and rc not in (WCL_OK,):
        _check(rc)
    return rc, [i.as_dict() for i in infos]


def wcl_grad(h, x_ptr, y_ptr, gU_ptr):
    gk = ctypes.c_double(0.0)
    _check(load().wcl_grad(h, _vp(x_ptr), _vp(y_ptr), _vp(gU_ptr), ctypes.byref(gk)))
    return gk.value


def wcl_bench_hop(h, prec, reps, copies, nrhs=1):
    ms = ctypes.c_double(0.0)
    _check(load().wcl_bench_hop(h, int(prec), int(nrhs), int(reps), int(copies), ctypes.byref(ms)))
    return ms.value


def wcl_bench_clover(h, prec, reps, copies):
    ms = ctypes.c_double(0.0)
    _check(load().wcl_bench_clover(h, int(prec), int(reps), int(copies), ctypes.byref(ms)))
    return ms.value


def wcl_bench_stream(h, mib, reps):
    r, c = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(load().wcl_bench_stream(h, float(mib), int(reps), ctypes.byref(r), ctypes.byref(c)))
    return r.value, c.value


def wcl_destroy(h):
    load().wcl_destroy(h)


def wcl_profile(h, enable):
    _check(load().wcl_profile(h, int(bool(enable))))


def wcl_profile_mask(h, mask):
    _check(load().wcl_profile_mask(h, int(mask)))


def wcl_profile_read(h, kclass):
    k = wcl_kstat()
    _check(load().wcl_profile_read(h, int(kclass), ctypes.byref(k)))
    return {"launches": k.launches, "ms": k.ms, "bytes": k.bytes, "flops": k.flops,
            "idle_launches": k.idle_launches, "idle_ms": k.idle_ms}


def wcl_set_tuning(h, hop_block, hop_depth, hop_xcd, hop_nontemporal=0):
    _check(load().wcl_set_tuning(h, int(hop_block), int(hop_depth), int(hop_xcd), int(hop_nontemporal)))


def wcl_set_batch_tuning(h, rhs_per_thread):
    _check(load().wcl_set_batch_tuning(h, int(rhs_per_thread)))


def wcl_autotune_hop(h, prec, copies):
    best = (ctypes.c_int * 3)()
    _check(load().wcl_autotune_hop(h, int(prec), int(copies), best))
    return {"hop_block": best[0], "hop_depth": best[1], "hop_xcd": best[2]}


def wcl_autotune(h, prec, nrhs, flags, b_ptr=None, opts=None):
    t = wcl_tuning()
    _check(load().wcl_autotune(h, int(prec), int(nrhs), _vp(b_ptr or 0),
                               ctypes.byref(opts) if opts is not None else None, int(flags), ctypes.byref(t)))
    return t.as_dict()


def wcl_set_hop_tiles(h, tiles):
    _check(load().wcl_set_hop_tiles(h, int(tiles)))


def wcl_set_hop_staging(h, enable):
    _check(load().wcl_set_hop_staging(h, int(enable)))


# --- convenience wrapper -----------------------------------------------------

class Lattice:
    """One lattice, one gauge field, one (kappa, c_sw) on the current device.

    Fields are torch complex128 CUDA tensors in the canonical layout:
    U ``[V,4,3,3]``, spinors ``[V,4,3]`` or ``[nrhs,V,4,3]``.
    """

    def __init__(self, dims, t_bc=-1, tile=None):
        import torch
        self.torch = torch
        self.dims = tuple(int(d) for d in dims)
        self.V = int(np.prod(self.dims))
        self.h = wcl_create(self.dims, t_bc, tile, torch.cuda.current_stream().cuda_stream)
        self.kappa = None
        self.csw = None

    def _sync_stream(self):
        wcl_set_stream(self.h, self.torch.cuda.current_stream().cuda_stream)

    def _dev(self, a, shape_tail):
        t = self.torch
        if isinstance(a, np.ndarray):
            a = t.from_numpy(np.ascontiguousarray(a, dtype=np.complex128))
        a = a.to(device="cuda", dtype=t.complex128).contiguous()
        if tuple(a.shape[-len(shape_tail):]) != shape_tail:
            raise ValueError(f"expected trailing shape {shape_tail}, got {tuple(a.shape)}")
        return a

    def set_gauge(self, U):
        self._U = self._dev(U, (self.V, 4, 3, 3))
        self._sync_stream()
        wcl_set_gauge(self.h, self._U.data_ptr())

    def set_compression(self, enable):
        """Two-row (12-real) FP32/FP16 link storage; the links must be SU(3)."""
        self._sync_stream()
        wcl_set_compression(self.h, int(bool(enable)))

    def set_params(self, kappa, csw):
        self._sync_stream()
        wcl_set_params(self.h, kappa, csw)
        self.kappa, self.csw = float(kappa), float(csw)

    def _spinors(self, psi):
        psi = self._dev(psi, (self.V, 4, 3))
        nrhs = 1 if psi.dim() == 3 else int(np.prod(psi.shape[:-3]))
        return psi, nrhs

    def apply(self, psi, dagger=False, prec=64):
        psi, nrhs = self._spinors(psi)
        out = self.torch.empty_like(psi)
        self._sync_stream()
        wcl_apply(self.h, psi.data_ptr(), out.data_ptr(), nrhs, int(bool(dagger)), prec)
        return out

    def apply_op(self, op, psi, prec=64):
        psi, nrhs = self._spinors(psi)
        out = self.torch.empty_like(psi)
        self._sync_stream()
        wcl_apply_op(self.h, op, psi.data_ptr(), out.data_ptr(), nrhs, prec)
        return out

    def set_ras(self, overlap=1, iters=4, solver=0, multiplicative=0):
        """Schwarz overlap, block steps, block solver (RAS_MR, RAS_JACOBI or
        RAS_BICGSTAB) and scheme (0 additive, 1 multiplicative colour sweeps)."""
        wcl_set_ras(self.h, overlap, iters, solver, multiplicative)

    def set_ras_cores(self, cores=None):
        """Schwarz cores (4 even extents dividing the lattice); None: the tiles."""
        wcl_set_ras_cores(self.h, cores)

    def solve(self, b, raise_on_error=True, x0=None, **kw):
        """Solve D x = b; ``x0`` (same shape as b) is an optional initial guess."""
        b, nrhs = self._spinors(b)
        x = self.torch.empty_like(b)
        o = wcl_default_opts()
        for k, v in kw.items():
            if not hasattr(o, k) or k == "x0_dev":
                raise KeyError(k)
            if k == "ras_block":
                v = (ctypes.c_int * 4)(*v)
            setattr(o, k, v)
        if x0 is not None:
            x0, n0 = self._spinors(x0)
            if n0 != nrhs:
                raise ValueError("x0 must hold one guess per right-hand side")
            o.x0_dev = x0.data_ptr()
        self._sync_stream()
        rc, infos = wcl_solve(self.h, b.data_ptr(), x.data_ptr(), nrhs, o, raise_on_error)
        return x, (infos[0] if nrhs == 1 and b.dim() == 3 else infos), rc

    def grad(self, x, y):
        x, _ = self._spinors(x)
        y, _ = self._spinors(y)
        gU = self.torch.empty((self.V, 4, 3, 3), dtype=self.torch.complex128, device="cuda")
        self._sync_stream()
        gk = wcl_grad(self.h, x.data_ptr(), y.data_ptr(), gU.data_ptr())
        return gU, gk

    def bench_hop(self, prec=32, reps=100, copies=1, nrhs=1):
        self._sync_stream()
        return wcl_bench_hop(self.h, prec, reps, copies, nrhs)

    def autotune(self, prec=32, nrhs=1, flags=TUNE_HOP, b=None, **opts):
        """The project autotuner (wcl_autotune); opts as for solve()."""
        o = None
        bp = None
        if b is not None:
            b, nrhs = self._spinors(b)
            bp = b.data_ptr()
            o = wcl_default_opts()
            for k, v in opts.items():
                setattr(o, k, v)
        self._sync_stream()
        return wcl_autotune(self.h, prec, nrhs, flags, bp, o)

    def bench_clover(self, prec=32, reps=100, copies=1):
        self._sync_stream()
        return wcl_bench_clover(self.h, prec, reps, copies)

    def close(self):
        if getattr(self, "h", None):
            wcl_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
