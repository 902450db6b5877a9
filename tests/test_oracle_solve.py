"""Pins of the oracle's solvers and of its Schwarz preconditioner.

* dense brute force on 4^4: D assembled column by column, numpy solve;
* free-field inverse in momentum space;
* hopping-parameter (Neumann) series at small kappa;
* RAS against a brute-force block solve built from the (pinned) global hop
  with every link outside the block zeroed (the Dirichlet cut by definition);
* the inner/outer solvers reach the unique x = D^-1 b.
Iteration counts are reported, not pinned (they depend on rounding).
"""
import numpy as np
import pytest

import oracle
from lattice_ref import coords, free_D_p, gamma5, momenta, parity, plane_wave, rel, spin_apply
from paper_1612_06556_amd import synth

DIMS4 = (4, 4, 4, 4)


@pytest.fixture(scope="module")
def dense4():
    kappa, csw = 0.12, 1.0
    U = synth.su3_field(DIMS4, 1001)
    o = oracle.Oracle(DIMS4, -1, kappa, csw, U)
    V = 256
    N = V * 12
    D = np.empty((N, N), complex)
    e = np.zeros(N, complex)
    for j in range(N):
        e[:] = 0
        e[j] = 1
        D[:, j] = o.D(e.reshape(V, 4, 3)).reshape(N)
    return o, D


def test_dense_gamma5_hermiticity(dense4):
    o, D = dense4
    G5 = np.kron(np.eye(256), np.kron(gamma5(), np.eye(3)))
    assert np.abs(G5 @ D @ G5 - D.conj().T).max() < 1e-14


def test_dense_solve_matches_bicgstab(dense4):
    o, D = dense4
    b = synth.gaussian_spinor(DIMS4, 2001)
    xd = np.linalg.solve(D, b.reshape(-1)).reshape(b.shape)
    x1, i1 = o.bicgstab_full(b, 1e-13, 5000)
    x2, i2 = o.bicgstab_eo(b, 1e-13, 5000)
    assert i1["status"] == 0 and i2["status"] == 0
    assert i1["relres"] <= 1e-13 and i2["relres"] <= 1e-13
    assert rel(x1, xd) < 1e-12
    assert rel(x2, xd) < 1e-12
    # the dagger solve: D^dag y = eta equals gamma5 D^-1 gamma5 eta
    eta = synth.gaussian_spinor(DIMS4, 3001)
    yd = np.linalg.solve(D.conj().T, eta.reshape(-1)).reshape(eta.shape)
    g5 = gamma5()
    y, iy = o.bicgstab_eo(spin_apply(g5, eta), 1e-13, 5000)
    assert rel(spin_apply(g5, y), yd) < 1e-12


def test_dense_schur_and_clover_inverse(dense4):
    o, D = dense4
    Tinv = o.clover_inv_matrix()
    T = o.clover_matrix()
    for n in (0, 17, 255):
        blk = D[n * 12:(n + 1) * 12, n * 12:(n + 1) * 12]
        assert np.abs(blk - T[n]).max() < 1e-15
        assert np.abs(np.linalg.inv(blk) - Tinv[n]).max() < 1e-13


@pytest.mark.parametrize("tbc", [1, -1])
def test_free_field_inverse(tbc):
    dims = (4, 4, 6, 8)
    kappa = 0.124
    o = oracle.Oracle(dims, tbc, kappa, 1.0, synth.unit_field(dims))
    rng = np.random.default_rng(5)
    u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    p = momenta(dims, (1, 2, 1, 3), tbc)
    b = plane_wave(dims, p, u)
    x, info = o.bicgstab_eo(b, 1e-13, 5000)
    assert info["status"] == 0
    # closed form D(p)^-1 = [1 - 2k sum cos - 2ik sum gamma sin] / [(1 - 2k sum cos)^2 + 4k^2 sum sin^2]
    m = 1 - 2 * kappa * np.cos(p).sum()
    Dp = free_D_p(p, kappa)
    Dinv = (2 * m * np.eye(4) - Dp) / (m * m + 4 * kappa ** 2 * (np.sin(p) ** 2).sum())
    assert np.allclose(Dinv @ Dp, np.eye(4), atol=1e-14)
    assert rel(x, plane_wave(dims, p, Dinv @ u)) < 1e-12


def test_neumann_series_small_kappa():
    """D = 1 - kappa K with K = H + csw C: D^-1 b = sum_n (kappa K)^n b."""
    dims = (4, 4, 4, 6)
    kappa, csw = 0.05, 1.0
    o = oracle.Oracle(dims, -1, kappa, csw, synth.su3_field(dims, 71))
    b = synth.gaussian_spinor(dims, 72)
    term = b.copy()
    acc = b.copy()
    nb = np.linalg.norm(b)
    for _ in range(80):
        term = kappa * (o.hop(term) + csw * o.clover_C(term))
        acc += term
        if np.linalg.norm(term) < 1e-15 * nb:
            break
    else:
        pytest.fail("Neumann series did not converge")
    x, info = o.bicgstab_full(b, 1e-14, 2000)
    assert rel(x, acc) < 1e-12
    # and T = 1 - csw kappa C
    assert rel(o.clover(b), b - csw * kappa * o.clover_C(b)) < 1e-15


def _bicgstab_steps(A, b, iters):
    """`iters` BiCGStab iterations on A x = b from x = 0, shadow residual b
    (van der Vorst 1992); stops when rho or <rh, v> is exactly zero."""
    x = np.zeros_like(b)
    r = b.copy()
    rh = b.copy()
    p = np.zeros_like(b)
    v = np.zeros_like(b)
    rho_old = alpha = omega = 1.0
    for _ in range(iters):
        rho = np.vdot(rh, r)
        if rho == 0:
            break
        p = r + (rho / rho_old) * (alpha / omega) * (p - omega * v)
        v = A(p)
        rv = np.vdot(rh, v)
        if rv == 0:
            break
        alpha = rho / rv
        s_ = r - alpha * v
        t = A(s_)
        tt = np.vdot(t, t).real
        omega = np.vdot(t, s_) / tt if tt != 0 else 0.0
        x = x + alpha * p + omega * s_
        r = s_ - omega * t
        rho_old = rho
        if tt == 0:
            break
    return x


def _ras_bruteforce(o, dims, U, v, block, overlap, iters, solver=0, colour=None):
    """RAS from the pinned global operator: per block, a copy of the oracle on a
    gauge field that keeps only the links between locally adjacent sites of the
    extended block (all other links zero), so its hop is the Dirichlet block
    hop; minimal residual (solver 0), block Jacobi steps with alpha = 1
    (solver 1) or BiCGStab iterations (solver 2) in numpy; keep the even core
    sites."""
    V = len(v)
    X = coords(dims)
    even = parity(dims) == 0
    out = np.zeros_like(v)
    nbk = [dims[mu] // block[mu] for mu in range(4)]
    ext = [block[mu] + 2 * overlap for mu in range(4)]
    for bi in range(int(np.prod(nbk))):
        rem = bi
        org = []
        col = 0
        for mu in range(4):
            org.append((rem % nbk[mu]) * block[mu])
            col |= ((rem % nbk[mu]) & 1) << mu
            rem //= nbk[mu]
        if colour is not None and col != colour:
            continue
        # local coordinate of every site in the extended block, -1 if outside
        loc = np.full((V, 4), -1)
        inside = np.ones(V, bool)
        for mu in range(4):
            a = (X[:, mu] - (org[mu] - overlap)) % dims[mu]
            inside &= a < ext[mu]
            loc[:, mu] = a
        UB = np.zeros_like(U)
        for mu in range(4):
            Xp = X.copy(); Xp[:, mu] = (Xp[:, mu] + 1) % dims[mu]
            npl = Xp[:, 0] + dims[0] * (Xp[:, 1] + dims[1] * (Xp[:, 2] + dims[2] * Xp[:, 3]))
            keep = inside & inside[npl] & (loc[:, mu] + 1 < ext[mu])
            UB[keep, mu] = U[keep, mu]
        oB = oracle.Oracle(dims, o.tbc, o.kappa, o.csw, UB)
        mask_e = (inside & even)[:, None, None]
        mask_o = (inside & ~even)[:, None, None]

        def dhat(x):
            y = o.clover_inv(oB.hop(x) * mask_o) * mask_o
            return (x - o.kappa ** 2 * o.clover_inv(oB.hop(y) * mask_e)) * mask_e

        r = v * mask_e
        z = np.zeros_like(v)
        if solver == 2:
            z = _bicgstab_steps(dhat, r, iters)
        for _ in range(iters if solver != 2 else 0):
            q = dhat(r)
            alpha = np.vdot(q, r) / np.vdot(q, q).real if solver == 0 else 1.0
            z = z + alpha * r
            r = r - alpha * q
        core = inside & even
        for mu in range(4):
            core &= (loc[:, mu] >= overlap) & (loc[:, mu] < overlap + block[mu])
        out[core] = z[core]
    return out


@pytest.mark.parametrize("solver", [0, 1, 2])
@pytest.mark.parametrize("dims,block,overlap", [((4, 4, 4, 4), (2, 2, 2, 2), 1),
                                                ((8, 4, 4, 4), (4, 2, 2, 2), 1),
                                                ((4, 4, 4, 8), (2, 2, 2, 4), 0)])
def test_ras_bruteforce(dims, block, overlap, solver):
    U = synth.su3_field(dims, 81)
    o = oracle.Oracle(dims, -1, 0.125, 1.0, U)
    v = synth.gaussian_spinor(dims, 82)
    v[parity(dims) == 1] = 0
    got = o.ras(v, block, overlap, 4, solver)
    ref = _ras_bruteforce(o, dims, U, v, block, overlap, 4, solver)
    assert rel(got, ref) < 1e-13
    assert np.abs(got[parity(dims) == 1]).max() == 0.0


def test_ras_jacobi_one_and_two_steps():
    """Block Jacobi from z = 0: one step gives z = r_B, two give 2 r_B - Dhat_B r_B;
    on a vector supported deep inside one core, Dhat_B acts as the global Dhat
    (hops reaching the cut need two sites), so the core output is
    2 v - Dhat v there."""
    dims = (8, 8, 8, 8)
    o = oracle.Oracle(dims, -1, 0.124, 1.0, synth.su3_field(dims, 83))
    X = coords(dims)
    v = synth.gaussian_spinor(dims, 84)
    deep = np.all((X % 4 >= 1) & (X % 4 <= 2), axis=1) & np.all(X < 4, axis=1)
    v[~deep | (parity(dims) == 1)] = 0
    assert np.abs(v).max() > 0
    m1 = o.ras(v, (4, 4, 4, 4), 1, 1, 1)
    assert rel(m1, v) < 1e-15
    m2 = o.ras(v, (4, 4, 4, 4), 1, 2, 1)
    core0 = np.all(X < 4, axis=1) & (parity(dims) == 0)
    ref = 2 * v - o.schur(v)
    assert rel(m2[core0], ref[core0]) < 1e-13


def test_ras_rejects_bad_blocks():
    dims = (4, 4, 4, 4)
    o = oracle.Oracle(dims, -1, 0.125, 1.0, synth.su3_field(dims, 1))
    v = synth.gaussian_spinor(dims, 2)
    with pytest.raises(ValueError):
        o.ras(v, (4, 4, 4, 4), 1, 4)  # extended block larger than the lattice
    with pytest.raises(ValueError):
        o.ras(v, (3, 2, 2, 2), 0, 4)


def test_ras_approximates_inverse():
    """RAS is a preconditioner: ||1 - Dhat M|| well below ||1|| on a smooth field."""
    dims = (8, 8, 8, 8)
    o = oracle.Oracle(dims, -1, 0.12, 1.0, synth.su3_field(dims, 91))
    v = synth.gaussian_spinor(dims, 92)
    v[parity(dims) == 1] = 0
    Mv = o.ras(v, (4, 4, 4, 4), 1, 4)
    assert rel(o.schur(Mv), v) < 0.5


@pytest.mark.parametrize("use_ras", [False, True])
def test_mixed_structure_solvers_reach_the_solution(use_ras):
    dims = (8, 8, 8, 8)
    o = oracle.Oracle(dims, -1, 0.12, 1.0, synth.su3_field(dims, 1001))
    b = synth.gaussian_spinor(dims, 2001)
    xref, iref = o.bicgstab_eo(b, 1e-13, 5000)
    assert iref["status"] == 0
    x, info = o.fbicgstab(b, 1e-10, 50, 1e-3, 200, use_ras, (4, 4, 4, 4), 1, 4)
    assert info["status"] == 0 and info["relres"] <= 1e-10
    assert rel(x, xref) < 1e-8
    # inner solver: relative residual of the Schur system at stol
    even = parity(dims) == 0
    bh = o.schur_rhs(b)
    xi, ii = o.inner_bicgstab(bh / np.linalg.norm(bh), 1e-5, 500, use_ras, (4, 4, 4, 4), 1, 4)
    assert ii["status"] == 0
    assert rel(o.schur(xi), bh / np.linalg.norm(bh)) < 1e-5 * 1.0001
    assert np.abs(xi[~even]).max() == 0.0


def test_ras_rejects_unknown_block_solver():
    dims = (8, 8, 8, 8)
    o = oracle.Oracle(dims, -1, 0.125, 1.0, synth.su3_field(dims, 3))
    v = synth.gaussian_spinor(dims, 4)
    with pytest.raises(ValueError):
        o.ras(v, (4, 4, 4, 4), 1, 4, 3)


@pytest.mark.parametrize("dims,block,overlap", [((4, 4, 4, 8), (2, 2, 2, 2), 1), ((8, 4, 4, 4), (2, 2, 2, 2), 0)])
def test_sap_bruteforce(dims, block, overlap):
    """Multiplicative Schwarz: the 16 colours in turn, each block solve (the
    brute-force block operator above) on the residual v - Dhat z of the
    colours before it, Dhat from the pinned global Schur code."""
    U = synth.su3_field(dims, 85)
    o = oracle.Oracle(dims, -1, 0.125, 1.0, U)
    v = synth.gaussian_spinor(dims, 86)
    ev = parity(dims) == 0
    v[~ev] = 0
    z = np.zeros_like(v)
    for k in range(16):
        r = v - o.schur(z)
        r[~ev] = 0
        z = z + _ras_bruteforce(o, dims, U, r, block, overlap, 4, 0, colour=k)
    got = o.sap(v, block, overlap, 4)
    assert rel(got, z) < 1e-13
    # a better preconditioner than the additive one on the same blocks
    assert rel(o.schur(got), v) < rel(o.schur(o.ras(v, block, overlap, 4)), v)


def test_ras_block_solvers_reach_exact_block_solve(dense4):
    """With enough steps, the minimal-residual and BiCGStab block solvers both
    reach the exact block solution: Schwarz with 2^4 cores and no overlap on
    4^4, each block system solved densely from the assembled D restricted to
    the block (its even/odd Schur complement, T_ee^-1 form)."""
    o, D = dense4
    X = coords(DIMS4)
    even = parity(DIMS4) == 0
    v = synth.gaussian_spinor(DIMS4, 87)
    v[~even] = 0
    exact = np.zeros_like(v)
    k2 = o.kappa ** 2
    for bi in range(16):
        org = [((bi >> mu) & 1) * 2 for mu in range(4)]
        inside = np.all((X >= org) & (X < np.array(org) + 2), axis=1)
        ie = np.flatnonzero(inside & even)
        io = np.flatnonzero(inside & ~even)
        idx = lambda sites: (sites[:, None] * 12 + np.arange(12)).reshape(-1)
        E, O = idx(ie), idx(io)
        Dee, Deo, Doe, Doo = D[np.ix_(E, E)], D[np.ix_(E, O)], D[np.ix_(O, E)], D[np.ix_(O, O)]
        S = Dee - Deo @ np.linalg.solve(Doo, Doe)   # = T_ee - k^2 H_eo T_oo^-1 H_oe
        # Dhat_B z = r with Dhat = T_ee^-1 S  <=>  S z = T_ee r
        z = np.linalg.solve(S, Dee @ v.reshape(-1)[E])
        exact.reshape(-1)[E] = z
    assert np.abs(exact[~even]).max() == 0
    mr = o.ras(v, (2, 2, 2, 2), 0, 300, 0)
    assert rel(mr, exact) < 1e-10
    errs = [rel(o.ras(v, (2, 2, 2, 2), 0, it, 2), exact) for it in (1, 2, 4, 8, 12)]
    print("BiCGStab block-solve errors", errs)
    assert errs[0] > 1e-3 and errs[1] < errs[0] and min(errs) < 1e-12
