"""Pins of the oracle's gradient of L = Re<eta, D^-1 b> against FP64 central
finite differences (4^4 and 6^4) and the kappa = 0 closed forms."""
import numpy as np
import pytest

import oracle
from lattice_ref import gamma5, rel, spin_apply
from paper_1612_06556_amd import synth


def _loss(dims, U, kappa, csw, b, eta):
    o = oracle.Oracle(dims, -1, kappa, csw, U)
    x, info = o.bicgstab_eo(b, 1e-14, 5000)
    assert info["status"] == 0
    return float(np.vdot(eta, x).real)


def _xy(o, b, eta):
    x, _ = o.bicgstab_eo(b, 1e-14, 5000)
    g5 = gamma5()
    y5, _ = o.bicgstab_eo(spin_apply(g5, eta), 1e-14, 5000)
    return x, spin_apply(g5, y5)


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 6, 6, 6)])
def test_grad_links_and_kappa_fd(dims):
    kappa, csw = 0.125, 1.0
    U = synth.su3_field(dims, 1005)
    b = synth.gaussian_spinor(dims, 2005)
    eta = synth.gaussian_spinor(dims, 3005)
    o = oracle.Oracle(dims, -1, kappa, csw, U)
    x, y = _xy(o, b, eta)
    gU, gk = o.grad(x, y)
    h = 1e-5
    rng = np.random.default_rng(9)
    # random unconstrained complex direction over all links
    for trial in range(2):
        E = rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape)
        fd = (_loss(dims, U + h * E, kappa, csw, b, eta) - _loss(dims, U - h * E, kappa, csw, b, eta)) / (2 * h)
        an = float(np.vdot(gU, E).real)
        assert abs(fd - an) <= 1e-5 * abs(an), (fd, an)
    # su(3) direction on a handful of single links: U -> exp(i h X) U
    for n, mu in [(0, 0), (5, 3), (len(U) - 1, 2)]:
        A = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
        X = 0.5 * (A + A.conj().T)
        X -= np.trace(X) / 3 * np.eye(3)
        w, Q = np.linalg.eigh(X)

        def rot(s):
            Up = U.copy()
            Up[n, mu] = (Q * np.exp(1j * s * w)) @ Q.conj().T @ U[n, mu]
            return Up
        fd = (_loss(dims, rot(h), kappa, csw, b, eta) - _loss(dims, rot(-h), kappa, csw, b, eta)) / (2 * h)
        an = float(np.vdot(gU[n, mu], 1j * X @ U[n, mu]).real)
        assert abs(fd - an) <= 1e-5 * max(abs(an), 1e-3), (fd, an)
    # kappa
    fd = (_loss(dims, U, kappa + h, csw, b, eta) - _loss(dims, U, kappa - h, csw, b, eta)) / (2 * h)
    assert abs(fd - gk) <= 1e-5 * abs(gk), (fd, gk)


def test_grad_kappa_zero_closed_form():
    """At kappa = 0: x = b, y = eta, grad_U = 0, dL/dkappa = Re<eta, H b> + csw Re<eta, C b>."""
    dims = (4, 4, 4, 4)
    U = synth.su3_field(dims, 1)
    b = synth.gaussian_spinor(dims, 2)
    eta = synth.gaussian_spinor(dims, 3)
    o = oracle.Oracle(dims, -1, 0.0, 1.3, U)
    gU, gk = o.grad(b, eta)
    assert np.abs(gU).max() == 0.0
    expect = np.vdot(eta, o.hop(b)).real + 1.3 * np.vdot(eta, o.clover_C(b)).real
    assert abs(gk - expect) <= 1e-14 * abs(expect)


def test_grad_b_is_adjoint_solution():
    """grad_b = y = D^-dag eta: L is linear in b with Re<y, db>."""
    dims = (4, 4, 4, 4)
    U = synth.su3_field(dims, 11)
    o = oracle.Oracle(dims, -1, 0.125, 1.0, U)
    b = synth.gaussian_spinor(dims, 12)
    eta = synth.gaussian_spinor(dims, 13)
    _, y = _xy(o, b, eta)
    db = synth.gaussian_spinor(dims, 14)
    x1, _ = o.bicgstab_eo(b + db, 1e-14, 5000)
    x0, _ = o.bicgstab_eo(b, 1e-14, 5000)
    assert abs(np.vdot(eta, x1 - x0).real - np.vdot(y, db).real) < 1e-11 * np.linalg.norm(db)
    assert rel(o.D(y, dagger=True), eta) < 1e-13
