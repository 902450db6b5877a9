"""The persistent inner solver (opts.persistent: every inner BiCGStab
iteration of a preconditioner call in one cooperative launch, reductions fused
into the hop epilogues) against the FP64 oracle and against the per-launch
path, through the C ABI.

The fused reductions add in another order than the per-launch dot kernels, so
the two paths agree to rounding, not bitwise: each solution is compared with
the oracle's (1e-8 at a true residual <= 1e-10 measured by the oracle's own
D) and with the other path's (1e-8); inner iteration counts are reported."""
import numpy as np
import pytest

import oracle
from gpu_util import rel, setup, site_err, to_gpu, to_host
from paper_1612_06556_amd import synth

pytestmark = pytest.mark.gpu

_refs = {}


def _ref(orc, b, key):
    if key not in _refs:
        x, info = orc.bicgstab_eo(b, 1e-13, 20000)
        assert info["status"] == 0
        _refs[key] = x
    return _refs[key]


def _res(orc, x, b):
    return float(np.linalg.norm(b - orc.D(x)) / np.linalg.norm(b))


@pytest.mark.parametrize("use_ras,inner_prec,vec16,outer", [
    (1, 32, 0, 0), (0, 32, 0, 0), (1, 16, 0, 0), (0, 16, 1, 0), (1, 16, 1, 0), (1, 32, 0, 1), (0, 32, 0, 1)])
def test_persistent_8x4(use_ras, inner_prec, vec16, outer):
    dims = (8, 8, 8, 8)
    lat, orc, _ = setup(dims, -1, 0.12, 1.0, 1001, None)
    b = synth.gaussian_spinor(dims, 2001)
    gb = to_gpu(b)
    kw = dict(tol=1e-10, use_ras=use_ras, inner_prec=inner_prec, inner_vec_prec=16 if vec16 else 32,
              inner_tol=1e-2, outer=outer, max_outer=200)
    xe, ie, rce = lat.solve(gb, **kw)
    xp, ip, rcp = lat.solve(gb, persistent=1, **kw)
    print(f"ras={use_ras} prec={inner_prec} vec16={vec16} outer={outer}: eager {ie} persistent {ip}", flush=True)
    assert rce == 0 and rcp == 0
    xp, xe = to_host(xp), to_host(xe)
    xr = _ref(orc, b, "8")
    assert _res(orc, xp, b) <= 1e-10
    assert rel(xp, xr) <= 1e-8 and site_err(xp, xr) <= 1e-7
    assert rel(xp, xe) <= 1e-8


@pytest.mark.timeout(600)
@pytest.mark.parametrize("use_ras,inner_prec", [(1, 32), (0, 32), (0, 16)])
def test_persistent_24x32(use_ras, inner_prec):
    """The benchmark's system (two-row links, inner tolerance 0.1)."""
    import torch
    from paper_1612_06556_amd import wcl
    dims = (24, 24, 24, 32)
    key = "24"
    if key not in _refs:
        U = synth.su3_field(dims, 1003)
        lat = wcl.Lattice(dims, -1)
        lat.set_compression(1)
        lat.set_gauge(torch.from_numpy(U).cuda())
        lat.set_params(0.126, 1.0)
        orc = oracle.Oracle(dims, -1, 0.126, 1.0, U)
        _refs["24lat"] = (lat, orc)
    lat, orc = _refs["24lat"]
    b = synth.gaussian_spinor(dims, 2003)
    xr = _ref(orc, b, key)
    x, info, rc = lat.solve(to_gpu(b), tol=1e-10, inner_tol=1e-1, use_ras=use_ras, inner_prec=inner_prec,
                            persistent=1)
    x = to_host(x)
    print(f"persistent 24^3x32 ras={use_ras} prec={inner_prec}: {info}", flush=True)
    assert rc == 0 and _res(orc, x, b) <= 1e-10
    assert rel(x, xr) <= 1e-8 and site_err(x, xr) <= 1e-7


@pytest.mark.parametrize("inner_prec", [32, 16])
def test_persistent_batched_point_sources(inner_prec):
    """The 12 spin-colour point sources in one persistent launch per inner
    solve (per right-hand-side scalars, converged ones masked)."""
    dims = (8, 8, 8, 8)
    lat, orc, _ = setup(dims, -1, 0.12, 1.0, 1001, None)
    b = synth.point_sources(dims)
    x, infos, rc = lat.solve(to_gpu(b), tol=1e-10, inner_prec=inner_prec, persistent=1)
    x = to_host(x)
    assert rc == 0 and len(infos) == 12
    for k in range(12):
        assert infos[k]["status"] == 0
        assert _res(orc, x[k], b[k]) <= 1e-10
        xr, _ = orc.bicgstab_eo(b[k], 1e-13, 20000)
        assert rel(x[k], xr) <= 1e-8, k
    print("persistent batched", infos[0], flush=True)


def test_persistent_profile_and_refusals():
    """The persistent launches are counted in their own profiling class; the
    option refuses settings it does not run."""
    from paper_1612_06556_amd import wcl
    dims = (8, 8, 8, 8)
    lat, orc, _ = setup(dims, -1, 0.12, 1.0, 1001, None)
    gb = to_gpu(synth.gaussian_spinor(dims, 2001))
    wcl.wcl_profile(lat.h, 1)
    x, info, rc = lat.solve(gb, tol=1e-10, persistent=1)
    st = wcl.wcl_profile_read(lat.h, wcl.K_INNER)
    wcl.wcl_profile(lat.h, 0)
    assert rc == 0 and st["launches"] == 2 * info["outer_iters"] and st["ms"] > 0 and st["flops"] > 0
    for kw in (dict(use_graph=1), dict(ras_solver=wcl.RAS_JACOBI), dict(ras_mult=1),
               dict(outer=wcl.OUTER_PLAIN64)):
        with pytest.raises(wcl.WclError):
            lat.solve(gb, persistent=1, **kw)
    with pytest.raises(wcl.WclError):
        lat.solve(to_gpu(synth.gaussian_spinor(dims, 3, nrhs=17)), persistent=1)
    lat.set_ras(1, 4, 0, 0)
    x, info, rc = lat.solve(gb, tol=1e-10)
    assert rc == 0 and _res(orc, to_host(x), synth.gaussian_spinor(dims, 2001)) <= 1e-10
