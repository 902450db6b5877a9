"""Test-side helpers: an independent construction of the Dirac matrices from
Pauli blocks, lattice coordinates and plane waves.  Used to pin the oracle;
nothing here is shared with the oracle or the HIP library."""
import numpy as np

PAULI = [np.array([[0, 1], [1, 0]], dtype=complex),
         np.array([[0, -1j], [1j, 0]], dtype=complex),
         np.array([[1, 0], [0, -1]], dtype=complex)]
I2 = np.eye(2, dtype=complex)
Z2 = np.zeros((2, 2), dtype=complex)


def gammas():
    """Chiral basis: gamma_k = [[0, -i s_k], [i s_k, 0]], gamma_t = [[0, 1], [1, 0]]."""
    g = [np.block([[Z2, -1j * s], [1j * s, Z2]]) for s in PAULI]
    g.append(np.block([[Z2, I2], [I2, Z2]]))
    return g


def gamma5():
    g = gammas()
    return g[0] @ g[1] @ g[2] @ g[3]


PLANES = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


def sigma(mu, nu):
    g = gammas()
    return 0.5j * (g[mu] @ g[nu] - g[nu] @ g[mu])


def coords(dims):
    V = int(np.prod(dims))
    n = np.arange(V)
    Lx, Ly, Lz, Lt = dims
    return np.stack([n % Lx, (n // Lx) % Ly, (n // (Lx * Ly)) % Lz, n // (Lx * Ly * Lz)], axis=1)


def parity(dims):
    return coords(dims).sum(axis=1) & 1


def site(dims, x):
    Lx, Ly, Lz, Lt = dims
    return int(x[0] % Lx + Lx * (x[1] % Ly + Ly * (x[2] % Lz + Lz * (x[3] % Lt))))


def momenta(dims, nvec, tbc):
    """p_mu = 2 pi n_mu / L_mu, with (2 n_t + 1) pi / L_t when antiperiodic."""
    p = [2 * np.pi * nvec[mu] / dims[mu] for mu in range(3)]
    p.append((2 * nvec[3] + (1 if tbc == -1 else 0)) * np.pi / dims[3])
    return np.array(p)


def plane_wave(dims, p, u):
    """psi(x) = exp(i p.x) u  with u a 4x3 spin-colour vector."""
    X = coords(dims)
    ph = np.exp(1j * (X @ p))
    return ph[:, None, None] * u[None, :, :]


def free_D_p(p, kappa):
    """D(p) = 1 - 2 kappa sum cos p + 2 i kappa sum gamma sin p (4x4 spin)."""
    g = gammas()
    M = (1 - 2 * kappa * np.cos(p).sum()) * np.eye(4, dtype=complex)
    for mu in range(4):
        M = M + 2j * kappa * np.sin(p[mu]) * g[mu]
    return M


def spin_apply(M, psi):
    """Apply a 4x4 spin matrix to a field psi[V][4][3]."""
    return np.einsum("st,ntc->nsc", M, psi)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))
