"""Pins of the FP64 oracle's operator: Dirac algebra, free-field closed form,
delta-source stencil, gamma5-hermiticity, gauge covariance and the clover term.

The paper prints no worked example (its figures are not numeric); every pin
here is a closed form, an invariant or brute force, chosen so that a dropped
term, a wrong sign, a transposed link or a misplaced neighbour fails one.
"""
import numpy as np
import pytest

import oracle
from lattice_ref import (PLANES, coords, free_D_p, gamma5, gammas, momenta, parity, plane_wave,
                         rel, sigma, site, spin_apply)
from paper_1612_06556_amd import synth


def test_reference_gamma_algebra():
    g = gammas()
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        for nu in range(4):
            ac = g[mu] @ g[nu] + g[nu] @ g[mu]
            assert np.allclose(ac, 2 * (mu == nu) * np.eye(4))
    assert np.allclose(gamma5(), np.diag([1, 1, -1, -1]))
    for mu, nu in PLANES:
        s = sigma(mu, nu)
        assert np.allclose(s, s.conj().T)
        assert np.allclose(s @ gamma5(), gamma5() @ s)
        assert np.allclose(s[:2, 2:], 0) and np.allclose(s[2:, :2], 0)


@pytest.mark.parametrize("tbc", [1, -1])
@pytest.mark.parametrize("nvec", [(0, 0, 0, 0), (1, 0, 2, 1), (3, 1, 0, 2)])
def test_free_field_plane_wave(tbc, nvec):
    """U = 1: D exp(ipx) u = D(p) exp(ipx) u, clover vanishes."""
    dims = (4, 6, 4, 8)
    kappa = 0.13
    o = oracle.Oracle(dims, tbc, kappa, 1.7, synth.unit_field(dims))
    rng = np.random.default_rng(7)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    p = momenta(dims, nvec, tbc)
    psi = plane_wave(dims, p, u)
    expect = plane_wave(dims, p, free_D_p(p, kappa) @ u)
    assert rel(o.D(psi), expect) < 1e-14
    assert rel(o.clover(psi), psi) < 1e-15
    # H alone: D = 1 - kappa H at U = 1
    assert rel(o.hop(psi), (psi - expect) / kappa) < 1e-13


@pytest.mark.parametrize("tbc", [1, -1])
def test_delta_source_stencil(tbc):
    """D e_{x0,s,c}: T(x0) e on x0, -kappa (1 -/+ g_mu) U on the 8 neighbours."""
    dims = (4, 4, 6, 4)
    kappa, csw = 0.11, 1.3
    U = synth.su3_field(dims, 11)
    o = oracle.Oracle(dims, tbc, kappa, csw, U)
    g = gammas()
    V = int(np.prod(dims))
    for x0 in [(0, 0, 0, 0), (1, 2, 3, 3), (3, 3, 5, 0)]:
        n0 = site(dims, x0)
        s0, c0 = 2, 1
        e = np.zeros((V, 4, 3), complex)
        e[n0, s0, c0] = 1.0
        out = o.D(e)
        expect = np.zeros_like(out)
        T = o.clover_matrix()[n0]
        expect[n0] += T[:, s0 * 3 + c0].reshape(4, 3)
        for mu in range(4):
            # site x0 - mu hops forward onto x0 with U_mu(x0 - mu)
            xm = list(x0); xm[mu] -= 1
            nm = site(dims, xm)
            sgn = tbc if (mu == 3 and x0[3] == 0) else 1
            col = np.zeros((4, 3), complex)
            col[:, :] = np.outer(np.eye(4)[:, s0], U[nm, mu][:, c0])
            expect[nm] += -kappa * sgn * spin_apply(np.eye(4) - g[mu], col[None])[0]
            # site x0 + mu hops backward onto x0 with U_mu(x0)^dag
            xp = list(x0); xp[mu] += 1
            npl = site(dims, xp)
            sgn = tbc if (mu == 3 and x0[3] == dims[3] - 1) else 1
            col = np.outer(np.eye(4)[:, s0], U[n0, mu].conj().T[:, c0])
            expect[npl] += -kappa * sgn * spin_apply(np.eye(4) + g[mu], col[None])[0]
        assert np.abs(out - expect).max() < 1e-14


def test_kappa_zero_is_identity():
    dims = (4, 4, 4, 4)
    U = synth.su3_field(dims, 3)
    o = oracle.Oracle(dims, -1, 0.0, 1.0, U)
    psi = synth.gaussian_spinor(dims, 4)
    assert np.array_equal(o.D(psi), psi)


@pytest.mark.parametrize("tbc", [1, -1])
def test_gamma5_hermiticity_and_dagger(tbc):
    dims = (4, 4, 4, 6)
    o = oracle.Oracle(dims, tbc, 0.125, 1.0, synth.su3_field(dims, 21))
    phi = synth.gaussian_spinor(dims, 22)
    psi = synth.gaussian_spinor(dims, 23)
    g5 = gamma5()
    g5Dg5psi = spin_apply(g5, o.D(spin_apply(g5, psi)))
    lhs = np.vdot(phi, g5Dg5psi)
    rhs = np.vdot(o.D(phi), psi)
    assert abs(lhs - rhs) / abs(rhs) < 1e-13
    assert abs(np.vdot(phi, o.D(psi)) - np.vdot(o.D(phi, dagger=True), psi)) < 1e-13 * np.linalg.norm(psi) ** 2


def _gauge_transform(U, g, dims):
    """U_mu(x) -> g(x) U_mu(x) g(x+mu)^dag"""
    X = coords(dims)
    Up = np.empty_like(U)
    for mu in range(4):
        Xp = X.copy(); Xp[:, mu] = (Xp[:, mu] + 1) % dims[mu]
        npl = Xp[:, 0] + dims[0] * (Xp[:, 1] + dims[1] * (Xp[:, 2] + dims[2] * Xp[:, 3]))
        Up[:, mu] = g @ U[:, mu] @ np.conj(np.swapaxes(g[npl], -1, -2))
    return Up


@pytest.mark.parametrize("tbc", [1, -1])
def test_gauge_covariance(tbc):
    dims = (4, 4, 6, 4)
    kappa, csw = 0.12, 1.0
    U = synth.su3_field(dims, 31)
    g = synth.random_su3_gauge_transform(dims, 32)
    Up = _gauge_transform(U, g, dims)
    o, op = oracle.Oracle(dims, tbc, kappa, csw, U), oracle.Oracle(dims, tbc, kappa, csw, Up)
    psi = synth.gaussian_spinor(dims, 33)
    gpsi = np.einsum("nab,nsb->nsa", g, psi)
    for name in ("hop", "clover", "D"):
        lhs = getattr(op, name)(gpsi)
        rhs = np.einsum("nab,nsb->nsa", g, getattr(o, name)(psi))
        assert rel(lhs, rhs) < 1e-13, name
    # the field strength transforms in the adjoint
    F, Fp = o.field_strength(), op.field_strength()
    gF = np.einsum("nab,npbc,ndc->npad", g, F, g.conj())
    assert rel(Fp, gF) < 1e-13


def test_clover_unit_field_and_structure():
    dims = (4, 4, 4, 4)
    o1 = oracle.Oracle(dims, -1, 0.126, 1.0, synth.unit_field(dims))
    assert np.abs(o1.clover_matrix() - np.eye(12)).max() == 0.0
    o = oracle.Oracle(dims, -1, 0.126, 1.0, synth.su3_field(dims, 41))
    T = o.clover_matrix()
    assert np.abs(T - np.conj(np.swapaxes(T, 1, 2))).max() < 1e-15
    G5 = np.kron(gamma5(), np.eye(3))
    assert np.abs(T @ G5 - G5 @ T).max() < 1e-15
    Ti = o.clover_inv_matrix()
    assert np.abs(T @ Ti - np.eye(12)).max() < 1e-13
    ev = np.linalg.eigvalsh(T)
    assert ev.min() > 0.5 and ev.max() < 1.5
    # F is Hermitian and traceless
    F = o.field_strength()
    assert np.abs(F - np.conj(np.swapaxes(F, -1, -2))).max() < 1e-15
    assert np.abs(np.trace(F, axis1=-2, axis2=-1)).max() < 1e-15


def test_clover_ignores_boundary_link_sign():
    """A t-boundary sign flip of every U_t(t = Lt-1) leaves T unchanged."""
    dims = (4, 4, 4, 6)
    U = synth.su3_field(dims, 51)
    Uf = U.copy()
    X = coords(dims)
    Uf[X[:, 3] == dims[3] - 1, 3] *= -1
    T = oracle.Oracle(dims, -1, 0.126, 1.0, U).clover_matrix()
    Tf = oracle.Oracle(dims, -1, 0.126, 1.0, Uf).clover_matrix()
    assert np.abs(T - Tf).max() < 1e-14


@pytest.mark.parametrize("k", [1, 2])
def test_clover_constant_abelian_field(k):
    """SU(3)-embedded U(1) field with constant xy flux phi = 2 pi k / (Lx Ly):
    every xy plaquette is exp(i phi q), so F_xy = sin(phi) q exactly and
    T = 1 - csw kappa sigma_xy (x) sin(phi) q; the other planes vanish."""
    dims = (4, 6, 4, 4)
    Lx, Ly = dims[0], dims[1]
    kappa, csw = 0.12, 1.4
    q = np.array([1.0, -1.0, 0.0])
    phi = 2 * np.pi * k / (Lx * Ly)
    X = coords(dims)
    V = len(X)
    U = synth.unit_field(dims)
    for n in range(V):
        x0, x1 = X[n, 0], X[n, 1]
        U[n, 1] = np.diag(np.exp(1j * phi * x0 * q))
        if x0 == Lx - 1:
            U[n, 0] = np.diag(np.exp(-1j * phi * Lx * x1 * q))
    o = oracle.Oracle(dims, -1, kappa, csw, U)
    F = o.field_strength()
    expectF = np.zeros((V, 6, 3, 3), complex)
    expectF[:, 0] = np.diag(np.sin(phi) * q)
    assert np.abs(F - expectF).max() < 1e-14
    T = o.clover_matrix()
    expectT = np.eye(12) - csw * kappa * np.kron(sigma(0, 1), np.diag(np.sin(phi) * q))
    assert np.abs(T - expectT[None]).max() < 1e-14


def test_schur_identity():
    """x_o = T_oo^-1 kappa H_oe x_e  =>  D(x_e + x_o) = (T_ee Dhat x_e, 0)."""
    dims = (4, 4, 4, 4)
    o = oracle.Oracle(dims, -1, 0.125, 1.0, synth.su3_field(dims, 61))
    even = parity(dims) == 0
    xe = synth.gaussian_spinor(dims, 62)
    xe[~even] = 0
    x = o.reconstruct(np.zeros_like(xe), xe)
    assert np.array_equal(x[even], xe[even])
    Dx = o.D(x)
    assert np.abs(Dx[~even]).max() < 1e-14
    assert rel(Dx, o.clover(o.schur(xe))) < 1e-14
    # bhat: the e/o right-hand side of the full solution satisfies Dhat x_e = bhat
    b = synth.gaussian_spinor(dims, 63)
    xs, info = o.bicgstab_full(b, 1e-13, 2000)
    assert info["status"] == 0
    xs_e = xs.copy(); xs_e[~even] = 0
    assert rel(o.schur(xs_e), o.schur_rhs(b)) < 1e-12
    assert rel(o.reconstruct(b, xs_e), xs) < 1e-12
