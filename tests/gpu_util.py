"""Shared set-up for the GPU parity tests: one seeded gauge field fed to both
the HIP library (through the C-ABI binding) and the FP64 oracle."""
import functools

import numpy as np

import oracle
from paper_1612_06556_amd import synth


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test run without a visible GPU")
    return torch


@functools.lru_cache(maxsize=8)
def setup(dims, tbc, kappa, csw, seed, tile=None):
    torch = require_gpu()
    from paper_1612_06556_amd import wcl
    U = synth.su3_field(dims, seed)
    lat = wcl.Lattice(dims, tbc, tile)
    lat.set_gauge(torch.from_numpy(U).cuda())
    lat.set_params(kappa, csw)
    orc = oracle.Oracle(dims, tbc, kappa, csw, U)
    return lat, orc, U


def to_gpu(a):
    torch = require_gpu()
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def even_mask(dims):
    Lx, Ly, Lz, Lt = dims
    n = np.arange(int(np.prod(dims)))
    x, y, z, t = n % Lx, (n // Lx) % Ly, (n // (Lx * Ly)) % Lz, n // (Lx * Ly * Lz)
    return ((x + y + z + t) & 1) == 0


def site_err(a, b):
    """Largest per-site error: max over sites x of |a(x) - b(x)| divided by the
    root-mean-square site norm of b over the sites where b is non-zero (so one
    wrong site shows up even when the norm-wise error is small)."""
    a = np.asarray(a).reshape(-1, 12)
    b = np.asarray(b).reshape(-1, 12)
    nb = np.linalg.norm(b, axis=1)
    live = nb > 0
    rms = float(np.sqrt(np.mean(nb[live] ** 2))) if live.any() else 1.0
    return float(np.linalg.norm(a - b, axis=1).max() / max(rms, 1e-300))
