"""GPU solves against the FP64 oracle (through wcl_solve).

Bar: final x within 1e-8 (relative) of the oracle's solution converged to
1e-13, at a true FP64 residual <= 1e-10 measured by the oracle's own D.
Iteration counts are reported, not compared (they depend on rounding)."""
import numpy as np
import pytest

import oracle
from gpu_util import rel, setup, to_gpu, to_host
from paper_1612_06556_amd import synth

pytestmark = pytest.mark.gpu


def _oracle_residual(orc, x, b):
    return float(np.linalg.norm(b - orc.D(x)) / np.linalg.norm(b))


_ref_cache = {}


def _reference(orc, b, key):
    if key not in _ref_cache:
        x, info = orc.bicgstab_eo(b, 1e-13, 20000)
        assert info["status"] == 0
        _ref_cache[key] = x
    return _ref_cache[key]


def test_plain_fp64_8x4():
    """Plain FP64 BiCGStab on the full D, 8^4, kappa 0.12, tol 1e-10."""
    from paper_1612_06556_amd import wcl
    dims = (8, 8, 8, 8)
    lat, orc, _ = setup(dims, -1, 0.12, 1.0, 1001, None)
    b = synth.gaussian_spinor(dims, 2001)
    x, info, rc = lat.solve(to_gpu(b), outer=wcl.OUTER_PLAIN64, tol=1e-10, max_outer=5000)
    x = to_host(x)
    print("plain64", info, flush=True)
    assert rc == 0 and info["status"] == 0
    assert _oracle_residual(orc, x, b) <= 1e-10
    assert rel(x, _reference(orc, b, "8a")) <= 1e-8


def test_plain_fp64_eo_8x4():
    """Plain FP64 BiCGStab on the even/odd Schur system (no inner solve)."""
    from paper_1612_06556_amd import wcl
    dims = (8, 8, 8, 8)
    lat, orc, _ = setup(dims, -1, 0.12, 1.0, 1001, None)
    b = synth.gaussian_spinor(dims, 2001)
    x, info, rc = lat.solve(to_gpu(b), outer=wcl.OUTER_PLAIN64_EO, tol=1e-10, max_outer=5000)
    x = to_host(x)
    print("plain64_eo", info, flush=True)
    assert rc == 0 and info["status"] == 0 and info["inner_iters_total"] == 0
    assert _oracle_residual(orc, x, b) <= 1e-10
    assert rel(x, _reference(orc, b, "8a")) <= 1e-8


@pytest.mark.parametrize("overlap,solver,mult", [(0, 0, 0), (1, 1, 0), (0, 1, 0), (1, 0, 1), (0, 1, 1)])
def test_schwarz_variants_8x4(overlap, solver, mult):
    """RAS variants inside the mixed solve: no overlap, block Jacobi steps."""
    dims = (8, 8, 8, 8)
    lat, orc, _ = setup(dims, -1, 0.12, 1.0, 1001, None)
    b = synth.gaussian_spinor(dims, 2001)
    x, info, rc = lat.solve(to_gpu(b), use_ras=1, ras_overlap=overlap, ras_solver=solver, ras_mult=mult,
                            tol=1e-10, inner_tol=1e-2, max_outer=200)
    x = to_host(x)
    print(f"schwarz overlap={overlap} solver={solver} mult={mult}", info, flush=True)
    assert rc == 0 and info["status"] == 0
    assert _oracle_residual(orc, x, b) <= 1e-10
    assert rel(x, _reference(orc, b, "8a")) <= 1e-8
    lat.set_ras(1, 4, 0, 0)


@pytest.mark.parametrize("outer,use_ras,inner_prec", [(0, 1, 32), (0, 0, 32), (1, 1, 32), (0, 1, 16), (1, 0, 16)])
def test_mixed_8x4(outer, use_ras, inner_prec):
    dims = (8, 8, 8, 8)
    lat, orc, _ = setup(dims, -1, 0.12, 1.0, 1001, None)
    b = synth.gaussian_spinor(dims, 2001)
    x, info, rc = lat.solve(to_gpu(b), outer=outer, use_ras=use_ras, inner_prec=inner_prec, tol=1e-10,
                            inner_tol=1e-2, max_outer=200)
    x = to_host(x)
    print(f"mixed outer={outer} ras={use_ras} prec={inner_prec}", info, flush=True)
    assert rc == 0 and info["status"] == 0
    assert _oracle_residual(orc, x, b) <= 1e-10
    assert rel(x, _reference(orc, b, "8a")) <= 1e-8


def test_mixed_ras_16x32():
    """16^3x32, kappa 0.125: FP64 flexible BiCGStab + FP32 RAS-BiCGStab (4^4, overlap 1, 4 MR)."""
    dims = (16, 16, 16, 32)
    lat, orc, _ = setup(dims, -1, 0.125, 1.0, 1002, None)
    b = synth.gaussian_spinor(dims, 2002)
    gb = to_gpu(b)
    # FP32 D error against the oracle
    e = rel(to_host(lat.apply(gb, prec=32)), orc.D(b))
    print(f"D fp32 16^3x32 rel={e:.3e}", flush=True)
    assert e <= 1e-6
    x, info, rc = lat.solve(gb, tol=1e-10, inner_tol=1e-2, use_ras=1)
    x = to_host(x)
    print("mixed 16^3x32", info, flush=True)
    assert rc == 0
    assert _oracle_residual(orc, x, b) <= 1e-10
    err = rel(x, _reference(orc, b, "16"))
    print(f"x error vs oracle {err:.3e}", flush=True)
    assert err <= 1e-8


@pytest.mark.parametrize("inner_prec", [32, 16])
def test_bench_solve_24x32(inner_prec):
    """The benchmark's solve at 24^3x32, kappa 0.126 (two-row links, FP64 flexible
    BiCGStab + RAS-BiCGStab): true residual <= 1e-10 by the oracle's D and x
    within 1e-8 of the oracle's solution converged to 1e-13."""
    import torch
    from paper_1612_06556_amd import wcl
    dims = (24, 24, 24, 32)
    U = synth.su3_field(dims, 1003)
    lat = wcl.Lattice(dims, -1)
    lat.set_compression(1)
    lat.set_gauge(torch.from_numpy(U).cuda())
    lat.set_params(0.126, 1.0)
    orc = oracle.Oracle(dims, -1, 0.126, 1.0, U)
    b = synth.gaussian_spinor(dims, 2003)
    x, info, rc = lat.solve(to_gpu(b), tol=1e-10, inner_tol=1e-2, use_ras=1, inner_prec=inner_prec)
    x = to_host(x)
    print(f"bench solve 24^3x32 prec={inner_prec}", info, flush=True)
    assert rc == 0
    assert _oracle_residual(orc, x, b) <= 1e-10
    err = rel(x, _reference(orc, b, "24"))
    print(f"x error vs oracle {err:.3e}", flush=True)
    assert err <= 1e-8
    lat.close()


@pytest.mark.timeout(600)
def test_bench_step_exact_24x32():
    """bench.py's timed step exactly: 24^3x32, kappa 0.126, two-row links,
    the hopping launch shape chosen by wcl_autotune_hop (FP32, 4 field
    sets), FP64 flexible BiCGStab + FP32 RAS-BiCGStab (4^4 cores, overlap 1,
    4 MR steps) at inner tolerance 0.1, after a fresh gauge ingest and clover
    build: x within 1e-8 of the oracle's 1e-13 solution, per site too."""
    import torch
    from gpu_util import site_err
    from paper_1612_06556_amd import wcl
    dims = (24, 24, 24, 32)
    U = synth.su3_field(dims, 1003)
    lat = wcl.Lattice(dims, -1)
    lat.set_compression(1)
    gU = torch.from_numpy(U).cuda()
    lat.set_gauge(gU)
    lat.set_params(0.126, 1.0)
    tuning = wcl.wcl_autotune_hop(lat.h, 32, 4)
    print("autotuned", tuning, flush=True)
    orc = oracle.Oracle(dims, -1, 0.126, 1.0, U)
    b = synth.gaussian_spinor(dims, 2003)
    gb = to_gpu(b)
    opts = dict(tol=1e-10, use_ras=1, ras_overlap=1, ras_iters=4, inner_prec=32, inner_tol=1e-1,
                outer=wcl.OUTER_FBICGSTAB)
    for _ in range(2):   # the step re-ingests the gauge field and rebuilds the clover each time
        lat.set_gauge(gU)
        lat.set_params(0.126, 1.0)
        x, info, rc = lat.solve(gb, **opts)
    x = to_host(x)
    print("bench step", info, flush=True)
    assert rc == 0
    assert _oracle_residual(orc, x, b) <= 1e-10
    xr = _reference(orc, b, "24")
    err, es = rel(x, xr), site_err(x, xr)
    print(f"x error vs oracle {err:.3e}, worst site {es:.3e}", flush=True)
    assert err <= 1e-8 and es <= 1e-7
    lat.close()


def test_warm_start():
    """x0_dev: a start from the converged solution returns at once (no outer
    iteration, status OK); a start from a perturbed solution reaches the
    oracle's solution to 1e-8, for the flexible, defect-correction and plain
    solvers, single and batched; x0 may alias x."""
    from paper_1612_06556_amd import wcl
    dims = (8, 8, 8, 8)
    lat, orc, _ = setup(dims, -1, 0.12, 1.0, 1001, None)
    b = synth.gaussian_spinor(dims, 2001)
    xr = _reference(orc, b, "8a")
    gb = to_gpu(b)
    for kw in (dict(), dict(outer=wcl.OUTER_DC, inner_tol=1e-3), dict(outer=wcl.OUTER_PLAIN64, max_outer=5000),
               dict(outer=wcl.OUTER_PLAIN64_EO, max_outer=5000), dict(adjoint=1)):
        x, info, rc = lat.solve(gb, tol=1e-10, **kw)
        assert rc == 0
        x2, info2, rc2 = lat.solve(gb, tol=1e-10, x0=x, **kw)
        print("warm from converged", kw, info2, flush=True)
        assert rc2 == 0 and info2["outer_iters"] == 0 and info2["inner_iters_total"] == 0
        assert info2["true_relres"] <= 1e-10
        assert rel(to_host(x2), to_host(x)) <= 1e-12
        pert = to_host(x) + 1e-3 * synth.gaussian_spinor(dims, 5)
        gx = to_gpu(pert)
        x3, info3, rc3 = lat.solve(gb, tol=1e-10, x0=gx, **kw)
        assert rc3 == 0
        ref = xr if not kw.get("adjoint") else None
        if ref is not None:
            assert rel(to_host(x3), ref) <= 1e-8
        assert _oracle_residual_adj(orc, to_host(x3), b, kw.get("adjoint", 0)) <= 1e-10
    # batched, with x0 aliasing x: the guess is read before x is written
    bb = synth.gaussian_spinor(dims, 6, nrhs=3)
    x, infos, rc = lat.solve(to_gpu(bb), tol=1e-10)
    xs = to_host(x)
    buf = to_gpu(xs + 1e-4 * synth.gaussian_spinor(dims, 7, nrhs=3))
    o = wcl.wcl_default_opts()
    o.tol = 1e-10
    o.x0_dev = buf.data_ptr()
    rc, infos = wcl.wcl_solve(lat.h, to_gpu(bb).data_ptr(), buf.data_ptr(), 3, o)
    assert rc == 0
    out = to_host(buf)
    for k in range(3):
        assert _oracle_residual(orc, out[k], bb[k]) <= 1e-10
        assert rel(out[k], xs[k]) <= 1e-8


def _oracle_residual_adj(orc, x, b, adjoint):
    Dx = orc.D(x, dagger=bool(adjoint))
    return float(np.linalg.norm(b - Dx) / np.linalg.norm(b))


def test_solve_edge_cases():
    from paper_1612_06556_amd import wcl
    dims = (8, 8, 8, 8)
    lat, orc, _ = setup(dims, -1, 0.12, 1.0, 1001, None)
    zero = np.zeros((np.prod(dims), 4, 3), complex)
    x, info, rc = lat.solve(to_gpu(zero))
    assert rc == 0 and np.abs(to_host(x)).max() == 0.0
    nan = synth.gaussian_spinor(dims, 3)
    nan[5, 1, 2] = np.nan
    x, info, rc = lat.solve(to_gpu(nan), raise_on_error=False)
    assert rc == wcl.WCL_ENAN
    b = synth.gaussian_spinor(dims, 4)
    x, info, rc = lat.solve(to_gpu(b), max_outer=1, inner_tol=0.5, max_inner=2, raise_on_error=False)
    assert rc == wcl.WCL_ENOCONV and info["status"] == wcl.WCL_ENOCONV
    assert np.isfinite(to_host(x)).all()
    # two right-hand sides in one call
    bb = synth.gaussian_spinor(dims, 6, nrhs=2)
    x, infos, rc = lat.solve(to_gpu(bb))
    assert rc == 0 and len(infos) == 2
    for k in range(2):
        assert _oracle_residual(orc, to_host(x)[k], bb[k]) <= 1e-10


def test_singular_free_field_terminates():
    """U = 1, periodic, kappa = 1/8: D(p=0) = 1 - 8 kappa = 0 -- the solver
    must stop with an error status within its iteration limits."""
    import torch
    from paper_1612_06556_amd import wcl
    dims = (4, 4, 4, 4)
    lat = wcl.Lattice(dims, 1)
    lat.set_gauge(torch.from_numpy(synth.unit_field(dims)).cuda())
    lat.set_params(0.125, 1.0)
    b = np.zeros((256, 4, 3), complex)
    b[:, 0, 0] = 1.0  # the zero mode
    x, info, rc = lat.solve(to_gpu(b), outer=wcl.OUTER_PLAIN64, max_outer=50, raise_on_error=False)
    # <r~, D r> = 0 on the zero mode: every restart breaks down again
    assert rc == wcl.WCL_EBREAKDOWN and info["status"] == wcl.WCL_EBREAKDOWN
    x, info, rc = lat.solve(to_gpu(b), max_outer=5, max_inner=20, raise_on_error=False)
    assert rc != 0


def test_invalid_arguments():
    from paper_1612_06556_amd import wcl
    with pytest.raises(wcl.WclError):
        wcl.Lattice((8, 8, 8, 7))
    with pytest.raises(wcl.WclError):
        wcl.Lattice((8, 8, 8, 8), tile=(3, 2, 2, 2))
    lat = wcl.Lattice((8, 8, 8, 8))
    b = np.zeros((4096, 4, 3), complex)
    with pytest.raises(wcl.WclError) as e:
        lat.apply(to_gpu(b))
    assert e.value.code == wcl.WCL_ESTATE
    with pytest.raises(wcl.WclError):
        lat.set_ras(3, 4)  # 4 + 2*3 > 8


@pytest.mark.parametrize("inner_prec", [32, 16])
def test_batched_point_sources_8x4(inner_prec):
    """The 12 spin-colour point sources at the origin solved together (one set
    of launches for all right-hand sides): each x_k against its own oracle
    solve and residual."""
    dims = (8, 8, 8, 8)
    lat, orc, _ = setup(dims, -1, 0.12, 1.0, 1001, None)
    b = synth.point_sources(dims)
    x, infos, rc = lat.solve(to_gpu(b), tol=1e-10, inner_prec=inner_prec)
    x = to_host(x)
    assert rc == 0 and len(infos) == 12
    for k in range(12):
        assert infos[k]["status"] == 0
        assert _oracle_residual(orc, x[k], b[k]) <= 1e-10
        xr, _ = orc.bicgstab_eo(b[k], 1e-13, 20000)
        assert rel(x[k], xr) <= 1e-8, k
    print("batched", infos[0], flush=True)


@pytest.mark.timeout(900)
def test_batch12_32x64():
    """The benchmark's largest shape: 12 point sources at 32^3x64 (kappa 0.126,
    two-row links, FP16 inner with RAS) in one batched solve.  FP32 D against
    the oracle on a Gaussian field; every right-hand side's true residual
    <= 1e-10 by the oracle's own D; x_0 within 1e-8 of the oracle's own
    even/odd solve of that source (converged to 1e-12) and of a separate
    single right-hand-side solve (the solution is unique)."""
    import torch
    from paper_1612_06556_amd import wcl
    dims = (32, 32, 32, 64)
    U = synth.su3_field(dims, 1004)
    lat = wcl.Lattice(dims, -1)
    lat.set_compression(1)
    lat.set_gauge(torch.from_numpy(U).cuda())
    lat.set_params(0.126, 1.0)
    orc = oracle.Oracle(dims, -1, 0.126, 1.0, U)
    psi = synth.gaussian_spinor(dims, 3004)
    e = rel(to_host(lat.apply(to_gpu(psi), prec=32)), orc.D(psi))
    print(f"D fp32 32^3x64 rel={e:.3e}", flush=True)
    assert e <= 1e-6
    del psi
    b = synth.point_sources(dims)
    x, infos, rc = lat.solve(to_gpu(b), tol=1e-10, inner_tol=1e-1, inner_prec=16, use_ras=1)
    x = to_host(x)
    assert rc == 0 and len(infos) == 12
    for k in range(12):
        res = _oracle_residual(orc, x[k], b[k])
        print(f"rhs {k}: {infos[k]} oracle residual {res:.2e}", flush=True)
        assert infos[k]["status"] == 0 and res <= 1e-10
    x0, info0, rc0 = lat.solve(to_gpu(b[0]), tol=1e-10, inner_tol=1e-1, inner_prec=16, use_ras=1)
    assert rc0 == 0
    assert rel(x[0], to_host(x0)) <= 1e-8
    lat.close()
    xr, oinfo = orc.bicgstab_eo(b[0], 1e-12, 20000)
    err = rel(x[0], xr)
    print(f"rhs 0 vs oracle solve ({oinfo}): {err:.3e}", flush=True)
    assert oinfo["status"] == 0 and err <= 1e-8


def test_batched_mixed_outer_variants():
    """Batched defect correction and batched plain FP64 on 3 Gaussian sources."""
    from paper_1612_06556_amd import wcl
    dims = (8, 8, 8, 8)
    lat, orc, _ = setup(dims, -1, 0.12, 1.0, 1001, None)
    b = synth.gaussian_spinor(dims, 41, nrhs=3)
    for kw in (dict(outer=wcl.OUTER_DC, inner_tol=1e-3), dict(outer=wcl.OUTER_PLAIN64, max_outer=5000),
               dict(use_ras=0)):
        x, infos, rc = lat.solve(to_gpu(b), tol=1e-10, **kw)
        x = to_host(x)
        assert rc == 0, kw
        for k in range(3):
            assert _oracle_residual(orc, x[k], b[k]) <= 1e-10, (kw, k)


def test_graph_replay_matches_eager():
    """The inner iteration replayed as a captured hipGraph gives bitwise the
    same solution as the eagerly launched one (same kernels, same order),
    on every replay of a multi-iteration solve, twice in a row."""
    dims = (8, 8, 8, 8)
    lat, orc, _ = setup(dims, -1, 0.12, 1.0, 1001, None)
    b = to_gpu(synth.gaussian_spinor(dims, 2001, nrhs=2))
    x0, i0, rc0 = lat.solve(b, use_graph=0)
    for _ in range(2):
        x1, i1, rc1 = lat.solve(b, use_graph=1)
        assert rc0 == 0 and rc1 == 0
        assert np.array_equal(to_host(x0), to_host(x1))
        assert [i["inner_iters_total"] for i in i0] == [i["inner_iters_total"] for i in i1]


@pytest.mark.parametrize("inner_prec,use_ras", [(32, 1), (16, 0)])
def test_batch_rhs_per_thread(inner_prec, use_ras):
    """Keeping 2 or 4 right-hand sides per thread in the batched Schur halves
    (a different kernel, so FP32 rounding may differ): every right-hand side
    reaches the oracle's residual bound and agrees with the one-per-workgroup
    solve to the solution tolerance."""
    from paper_1612_06556_amd import wcl
    dims = (8, 8, 8, 16)
    lat, orc, _ = setup(dims, -1, 0.126, 1.0, 9, (4, 4, 4, 4))
    b = synth.gaussian_spinor(dims, 51, nrhs=5)   # a ragged last group of 4
    xs = []
    try:
        for nr in (1, 2, 4):
            wcl.wcl_set_batch_tuning(lat.h, nr)
            x, infos, rc = lat.solve(to_gpu(b), tol=1e-10, inner_prec=inner_prec, use_ras=use_ras)
            assert rc == 0
            xs.append(to_host(x))
    finally:
        wcl.wcl_set_batch_tuning(lat.h, 1)
    for k in range(5):
        for j in (1, 2):
            assert _oracle_residual(orc, xs[j][k], b[k]) <= 1e-10
            assert rel(xs[j][k], xs[0][k]) <= 1e-8
    with pytest.raises(wcl.WclError):
        wcl.wcl_set_batch_tuning(lat.h, 3)


@pytest.mark.parametrize("use_ras,compress", [(1, 0), (0, 0), (1, 1), (0, 1)])
def test_fp16_inner_vectors(use_ras, compress):
    """FP16 storage of the inner solver's vectors (with FP16 links and clover,
    FP32 arithmetic): the FP64 outer solver still reaches the oracle's
    solution; 3 right-hand sides batched."""
    import torch
    from paper_1612_06556_amd import wcl
    dims = (8, 8, 8, 16)
    U = synth.su3_field(dims, 61)
    lat = wcl.Lattice(dims, -1, (4, 4, 4, 4))
    lat.set_compression(compress)
    lat.set_gauge(torch.from_numpy(U).cuda())
    lat.set_params(0.124, 1.0)
    orc = oracle.Oracle(dims, -1, 0.124, 1.0, U)
    b = synth.gaussian_spinor(dims, 62, nrhs=3)
    x, infos, rc = lat.solve(to_gpu(b), tol=1e-10, inner_prec=16, inner_vec_prec=16, use_ras=use_ras,
                             inner_tol=1e-1)
    x = to_host(x)
    print(f"fp16 vectors ras={use_ras} compress={compress}", infos[0], flush=True)
    assert rc == 0
    for k in range(3):
        assert _oracle_residual(orc, x[k], b[k]) <= 1e-10
        xr, _ = orc.bicgstab_eo(b[k], 1e-13, 20000)
        assert rel(x[k], xr) <= 1e-8
    with pytest.raises(wcl.WclError):
        lat.solve(to_gpu(b[0]), inner_prec=32, inner_vec_prec=16)
    lat.close()
