"""Plain FP64 CPU oracle for the Wilson-Clover hot path (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package.  It wraps ``wco.c`` (plain C, double
complex, whole spin and colour matrices, no blocking or fusion) through
ctypes and shares no code with the HIP library.

All fields are canonical host arrays (see ``wco.h``): gauge ``U[V][4][3][3]``
and spinors ``psi[V][4][3]``, complex128, C order, site
``n = x + Lx*(y + Ly*(z + Lz*t))``.

Every routine below is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py`` against closed forms, brute force and invariants;
the solver iteration counts are the one output with no external pin
("parity unpinned": they depend on rounding).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libwco.so")
_SOURCES = [os.path.join(_HERE, "wco.c")]
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def build_library(verbose: bool = False) -> str:
    """Compile ``libwco.so`` with gcc (plain C11 + OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-o", _LIB_PATH + ".tmp", *_SOURCES, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or any(
            os.path.getmtime(s) > os.path.getmtime(_LIB_PATH) for s in _SOURCES):
        build_library()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.wco_create.restype = ctypes.c_void_p
    lib.wco_create.argtypes = [_ip, ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp]
    lib.wco_destroy.argtypes = [ctypes.c_void_p]
    lib.wco_set_threads.argtypes = [ctypes.c_int]
    lib.wco_set_threads.restype = ctypes.c_int
    for name in ("wco_hop", "wco_clover", "wco_clover_inv", "wco_clover_C", "wco_schur",
                 "wco_schur_rhs"):
        getattr(lib, name).argtypes = [ctypes.c_void_p, _dp, _dp]
    lib.wco_D.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_int]
    lib.wco_reconstruct.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
    for name in ("wco_field_strength", "wco_clover_matrix", "wco_clover_inv_matrix"):
        getattr(lib, name).argtypes = [ctypes.c_void_p, _dp]
    lib.wco_ras.argtypes = [ctypes.c_void_p, _ip, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp]
    lib.wco_ras.restype = ctypes.c_int
    lib.wco_sap.argtypes = [ctypes.c_void_p, _ip, ctypes.c_int, ctypes.c_int, ctypes.c_int, _dp, _dp]
    lib.wco_sap.restype = ctypes.c_int
    for name in ("wco_bicgstab_full", "wco_bicgstab_eo"):
        f = getattr(lib, name)
        f.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_double, ctypes.c_int, _ip, _dp]
        f.restype = ctypes.c_int
    lib.wco_inner_bicgstab.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_double, ctypes.c_int,
                                       ctypes.c_int, _ip, ctypes.c_int, ctypes.c_int, _ip]
    lib.wco_inner_bicgstab.restype = ctypes.c_int
    lib.wco_fbicgstab.argtypes = [ctypes.c_void_p, _dp, _dp, ctypes.c_double, ctypes.c_int,
                                  ctypes.c_double, ctypes.c_int, ctypes.c_int, _ip, ctypes.c_int,
                                  ctypes.c_int, _ip, _ip, _dp]
    lib.wco_fbicgstab.restype = ctypes.c_int
    lib.wco_grad.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp]
    _lib = lib
    return lib


def set_threads(n: int = 0) -> int:
    """OpenMP threads for the oracle's site loops; returns the count in use."""
    return _load().wco_set_threads(int(n))


def _c(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def _p(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _ivec(v):
    return (ctypes.c_int * 4)(*[int(t) for t in v])


class SolveResult(tuple):
    pass


class Oracle:
    """FP64 Wilson-Clover operator on a fixed gauge field.

    ``D = T - kappa*H`` with ``T = 1 - csw*kappa*sum_{mu<nu} sigma_{mu nu} F_{mu nu}``.
    """

    def __init__(self, dims, tbc: int, kappa: float, csw: float, U: np.ndarray):
        lib = _load()
        self.dims = tuple(int(d) for d in dims)
        self.V = int(np.prod(self.dims))
        self.tbc, self.kappa, self.csw = int(tbc), float(kappa), float(csw)
        self._U = _c(U).reshape(self.V, 4, 3, 3)
        self._h = lib.wco_create(_ivec(self.dims), self.tbc, self.kappa, self.csw, _p(self._U))
        if not self._h:
            raise ValueError("oracle: bad arguments or singular clover term")
        self._lib = lib

    def close(self):
        if getattr(self, "_h", None):
            self._lib.wco_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- helpers ------------------------------------------------------------
    def _spinor(self, v):
        return _c(v).reshape(self.V, 4, 3)

    def _un(self, name, v):
        a = self._spinor(v)
        out = np.empty_like(a)
        getattr(self._lib, name)(self._h, _p(a), _p(out))
        return out

    def parity(self) -> np.ndarray:
        Lx, Ly, Lz, Lt = self.dims
        n = np.arange(self.V)
        x = n % Lx
        y = (n // Lx) % Ly
        z = (n // (Lx * Ly)) % Lz
        t = n // (Lx * Ly * Lz)
        return (x + y + z + t) & 1

    # --- operators ----------------------------------------------------------
    def hop(self, v):
        return self._un("wco_hop", v)

    def clover(self, v):
        return self._un("wco_clover", v)

    def clover_inv(self, v):
        return self._un("wco_clover_inv", v)

    def clover_C(self, v):
        return self._un("wco_clover_C", v)

    def D(self, v, dagger: bool = False):
        a = self._spinor(v)
        out = np.empty_like(a)
        self._lib.wco_D(self._h, _p(a), _p(out), int(bool(dagger)))
        return out

    def field_strength(self):
        F = np.empty((self.V, 6, 3, 3), dtype=np.complex128)
        self._lib.wco_field_strength(self._h, _p(F))
        return F

    def clover_matrix(self):
        T = np.empty((self.V, 12, 12), dtype=np.complex128)
        self._lib.wco_clover_matrix(self._h, _p(T))
        return T

    def clover_inv_matrix(self):
        T = np.empty((self.V, 12, 12), dtype=np.complex128)
        self._lib.wco_clover_inv_matrix(self._h, _p(T))
        return T

    def schur(self, xe):
        return self._un("wco_schur", xe)

    def schur_rhs(self, b):
        return self._un("wco_schur_rhs", b)

    def reconstruct(self, b, xe):
        bb, xx = self._spinor(b), self._spinor(xe)
        out = np.empty_like(bb)
        self._lib.wco_reconstruct(self._h, _p(bb), _p(xx), _p(out))
        return out

    def ras(self, v, block=(4, 4, 4, 4), overlap: int = 1, iters: int = 4, solver: int = 0):
        """One RAS application (solver 0: minimal residual, 1: block Jacobi,
        2: block BiCGStab)."""
        a = self._spinor(v)
        out = np.empty_like(a)
        rc = self._lib.wco_ras(self._h, _ivec(block), int(overlap), int(iters), int(solver), _p(a), _p(out))
        if rc != 0:
            raise ValueError("oracle RAS: block shape does not fit the lattice")
        return out

    def sap(self, v, block=(4, 4, 4, 4), overlap: int = 1, iters: int = 4, solver: int = 0):
        """One multiplicative Schwarz application (16 colours in turn)."""
        a = self._spinor(v)
        out = np.empty_like(a)
        rc = self._lib.wco_sap(self._h, _ivec(block), int(overlap), int(iters), int(solver), _p(a), _p(out))
        if rc != 0:
            raise ValueError("oracle SAP: block shape does not fit the lattice")
        return out

    # --- solvers ------------------------------------------------------------
    def _solve(self, name, b, tol, maxiter):
        bb = self._spinor(b)
        x = np.empty_like(bb)
        it = ctypes.c_int(0)
        rr = ctypes.c_double(0.0)
        st = getattr(self._lib, name)(self._h, _p(bb), _p(x), float(tol), int(maxiter),
                                       ctypes.byref(it), ctypes.byref(rr))
        return x, dict(status=st, iters=it.value, relres=rr.value)

    def bicgstab_full(self, b, tol=1e-10, maxiter=10000):
        """Plain BiCGStab on the full D (no preconditioner)."""
        return self._solve("wco_bicgstab_full", b, tol, maxiter)

    def bicgstab_eo(self, b, tol=1e-13, maxiter=10000):
        """BiCGStab on the even/odd Schur system, then odd reconstruction."""
        return self._solve("wco_bicgstab_eo", b, tol, maxiter)

    def inner_bicgstab(self, rhs, stol=1e-4, maxiter=200, use_ras=True, block=(4, 4, 4, 4),
                       overlap=1, ras_iters=4):
        r = self._spinor(rhs)
        x = np.empty_like(r)
        it = ctypes.c_int(0)
        st = self._lib.wco_inner_bicgstab(self._h, _p(r), _p(x), float(stol), int(maxiter),
                                          int(bool(use_ras)), _ivec(block), int(overlap),
                                          int(ras_iters), ctypes.byref(it))
        return x, dict(status=st, iters=it.value)

    def fbicgstab(self, b, tol=1e-10, max_outer=100, inner_tol=1e-4, max_inner=200,
                  use_ras=True, block=(4, 4, 4, 4), overlap=1, ras_iters=4):
        bb = self._spinor(b)
        x = np.empty_like(bb)
        no, ni = ctypes.c_int(0), ctypes.c_int(0)
        rr = ctypes.c_double(0.0)
        st = self._lib.wco_fbicgstab(self._h, _p(bb), _p(x), float(tol), int(max_outer),
                                     float(inner_tol), int(max_inner), int(bool(use_ras)),
                                     _ivec(block), int(overlap), int(ras_iters),
                                     ctypes.byref(no), ctypes.byref(ni), ctypes.byref(rr))
        return x, dict(status=st, outer=no.value, inner_total=ni.value, relres=rr.value)

    def grad(self, x, y):
        """Link and kappa gradient of L = Re<eta, D^-1 b> from x and y."""
        xx, yy = self._spinor(x), self._spinor(y)
        gU = np.empty((self.V, 4, 3, 3), dtype=np.complex128)
        gk = ctypes.c_double(0.0)
        self._lib.wco_grad(self._h, _p(xx), _p(yy), _p(gU), ctypes.byref(gk))
        return gU, gk.value
