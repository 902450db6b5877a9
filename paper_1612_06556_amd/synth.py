"""Seeded synthetic inputs shared by the HIP path, the oracle and the benches.

This module draws random numbers and nothing else: it holds none of the
Dirac-operator or solver arithmetic, so that neither side of a parity test can
borrow the other's mathematics through it.

Layouts (canonical, host, complex128, C order):

* gauge field  ``U[V][4][3][3]``   -- ``U[n, mu]`` is the link from site ``n``
  in direction ``mu`` (0..3 = x, y, z, t), a row-major 3x3 matrix;
* spinor field ``psi[V][4][3]``     -- ``[spin][colour]`` per site;
* site index   ``n = x + Lx*(y + Ly*(z + Lz*t))``.

The paper benchmarks on gauge configurations it does not describe; the
stand-in here is a field of near-unit SU(3) links, each the exponential of
``i*eps*H`` for a random Hermitian traceless ``H`` with complex Gaussian
entries, re-unitarised to det 1 to machine precision.
"""
from __future__ import annotations

import math

import numpy as np

_CHUNK_SITES = 1 << 16


def volume(dims) -> int:
    return int(np.prod([int(d) for d in dims]))


def _reunitarise(W: np.ndarray) -> np.ndarray:
    """Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1)."""
    r0 = W[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = W[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def su3_field(dims, seed: int, eps: float = 0.3) -> np.ndarray:
    """Random SU(3) links ``exp(i*eps*H)``, ``H`` Hermitian traceless Gaussian.

    Draw order: site-major, then direction, then the 3x3 entries of the complex
    Gaussian matrix ``A`` (real part, imaginary part); ``H = (A + A^dag)/2``
    minus its trace part.  ``numpy.random.default_rng(seed)`` (PCG64).
    """
    V = volume(dims)
    rng = np.random.default_rng(seed)
    U = np.empty((V, 4, 3, 3), dtype=np.complex128)
    for s0 in range(0, V, _CHUNK_SITES):
        s1 = min(V, s0 + _CHUNK_SITES)
        g = rng.standard_normal((s1 - s0, 4, 3, 3, 2))
        A = (g[..., 0] + 1j * g[..., 1]) / math.sqrt(2.0)
        H = 0.5 * (A + np.conj(np.swapaxes(A, -1, -2)))
        tr = np.trace(H, axis1=-2, axis2=-1) / 3.0
        H = H - tr[..., None, None] * np.eye(3)
        w, Q = np.linalg.eigh(H)
        E = np.exp(1j * eps * w)
        W = (Q * E[..., None, :]) @ np.conj(np.swapaxes(Q, -1, -2))
        U[s0:s1] = _reunitarise(W)
    return U


def unit_field(dims) -> np.ndarray:
    """The free field: every link is the identity."""
    V = volume(dims)
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    U[:, :, 0, 0] = U[:, :, 1, 1] = U[:, :, 2, 2] = 1.0
    return U


def gaussian_spinor(dims, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Complex Gaussian spinor(s), real and imaginary parts ~ N(0, 1/2)."""
    V = volume(dims)
    rng = np.random.default_rng(seed)
    shape = (V, 4, 3, 2) if nrhs is None else (nrhs, V, 4, 3, 2)
    g = rng.standard_normal(shape) * math.sqrt(0.5)
    return np.ascontiguousarray(g[..., 0] + 1j * g[..., 1])


def point_sources(dims, site: int = 0) -> np.ndarray:
    """The 12 spin-colour point sources at one site: ``b[(s,c)][n][s'][c']``."""
    V = volume(dims)
    b = np.zeros((12, V, 4, 3), dtype=np.complex128)
    for k in range(12):
        b[k, site, k // 3, k % 3] = 1.0
    return b


def random_su3_gauge_transform(dims, seed: int) -> np.ndarray:
    """One broad random SU(3) matrix per site, ``g[V][3][3]``."""
    V = volume(dims)
    U = su3_field((V, 1, 1, 1), seed, eps=2.0)
    return np.ascontiguousarray(U[:, 0])
