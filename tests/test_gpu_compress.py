"""Two-row (12-real) link storage of the FP32 and FP16 tiers.

An SU(3) matrix is fixed by its first two rows (unitarity with unit
determinant makes row 2 the complex conjugate of row0 x row1), so the
compressed tiers must reproduce the same operator as the full-link tiers:
D, one RAS application and the mixed-precision solve are compared with the
FP64 oracle at the tolerances of the uncompressed tiers (FP32 1e-6, FP16
3e-3; RAS 1e-5 in FP32).  Links that are not SU(3) are refused."""
import numpy as np
import pytest

import oracle
from gpu_util import even_mask, rel, require_gpu, site_err, to_gpu, to_host
from paper_1612_06556_amd import synth

pytestmark = pytest.mark.gpu

TOL = {32: 1e-6, 16: 3e-3}
CASES = [  # dims, tbc, kappa, csw, seed, tile
    ((8, 8, 8, 8), -1, 0.12, 1.0, 1001, None),
    ((4, 6, 8, 4), -1, 0.125, 1.3, 7, None),        # 2^4 tiles, ragged last workgroup
    ((6, 4, 4, 8), 1, 0.126, 1.0, 8, (2, 2, 2, 4)),  # periodic, non-cubic tile
]


def _ids(c):
    return "x".join(map(str, c[0])) + f"_tbc{c[1]}"


def _lattice(dims, tbc, kappa, csw, seed, tile, compress=True):
    torch = require_gpu()
    from paper_1612_06556_amd import wcl
    U = synth.su3_field(dims, seed)
    lat = wcl.Lattice(dims, tbc, tile)
    if compress:
        lat.set_compression(1)
    lat.set_gauge(torch.from_numpy(U).cuda())
    lat.set_params(kappa, csw)
    return lat, U


@pytest.mark.parametrize("case", CASES, ids=_ids)
@pytest.mark.parametrize("prec", [32, 16])
def test_D_compressed(case, prec):
    dims, tbc, kappa, csw, seed, tile = case
    lat, U = _lattice(dims, tbc, kappa, csw, seed, tile)
    orc = oracle.Oracle(dims, tbc, kappa, csw, U)
    psi = synth.gaussian_spinor(dims, seed + 1)
    g = to_gpu(psi)
    for dag in (False, True):
        e = rel(to_host(lat.apply(g, dagger=dag, prec=prec)), orc.D(psi, dagger=dag))
        print(f"D12 dims={dims} prec={prec} dag={dag} rel={e:.3e}", flush=True)
        assert e <= TOL[prec]


@pytest.mark.parametrize("prec", [32, 16])
def test_ras_compressed(prec):
    from paper_1612_06556_amd import wcl
    dims = (8, 8, 8, 8)
    lat, U = _lattice(dims, -1, 0.12, 1.0, 1001, None)
    orc = oracle.Oracle(dims, -1, 0.12, 1.0, U)
    psi = synth.gaussian_spinor(dims, 1004)
    psi[~even_mask(dims)] = 0
    lat.set_ras(1, 4)
    e = rel(to_host(lat.apply_op(wcl.OP_RAS, to_gpu(psi), prec=prec)), orc.ras(psi, (4, 4, 4, 4), 1, 4))
    print(f"RAS12 prec={prec} rel={e:.3e}", flush=True)
    assert e <= (1e-5 if prec == 32 else 3e-3)


def test_ras_compressed_new_gauge():
    """A second wcl_set_gauge with two-row storage on rebuilds every copy the
    Schwarz kernel reads (field-major and per-site two-row links): one RAS
    application and one D application match the oracle of the new field, at
    16^3x8 (several workgroups per XCD, cores on every tile face)."""
    torch = require_gpu()
    from paper_1612_06556_amd import wcl
    dims = (16, 16, 16, 8)
    lat, U1 = _lattice(dims, -1, 0.124, 1.0, 1201, None)
    psi = synth.gaussian_spinor(dims, 1203)
    psi[~even_mask(dims)] = 0
    lat.set_ras(1, 4)
    r1 = to_host(lat.apply_op(wcl.OP_RAS, to_gpu(psi), prec=32))
    U2 = synth.su3_field(dims, 1202)
    lat.set_gauge(torch.from_numpy(U2).cuda())
    lat.set_params(0.124, 1.0)
    orc = oracle.Oracle(dims, -1, 0.124, 1.0, U2)
    r2 = to_host(lat.apply_op(wcl.OP_RAS, to_gpu(psi), prec=32))
    e = rel(r2, orc.ras(psi, (4, 4, 4, 4), 1, 4))
    ed = rel(to_host(lat.apply(to_gpu(psi), prec=32)), orc.D(psi))
    print(f"RAS12 new gauge rel={e:.3e} D rel={ed:.3e}", flush=True)
    assert e <= 1e-5 and ed <= TOL[32]
    assert rel(r1, r2) > 1e-3   # the first field's result differs
    lat.close()


@pytest.mark.parametrize("use_ras,inner_prec", [(1, 32), (0, 16), (1, 16)])
def test_solve_compressed(use_ras, inner_prec):
    dims = (8, 8, 8, 8)
    lat, U = _lattice(dims, -1, 0.124, 1.0, 21, None)
    orc = oracle.Oracle(dims, -1, 0.124, 1.0, U)
    b = synth.gaussian_spinor(dims, 22)
    x, info, rc = lat.solve(to_gpu(b), use_ras=use_ras, inner_prec=inner_prec, tol=1e-10)
    print("solve12", use_ras, inner_prec, info, flush=True)
    assert rc == 0 and info["true_relres"] <= 1e-10
    xr = to_host(x)
    assert rel(orc.D(xr), b) <= 1e-10


def test_compression_off_matches_full_links():
    """Turning compression off again gives back the full-link kernels: the
    result is bitwise that of a context that never compressed."""
    dims = (8, 8, 8, 8)
    lat, _ = _lattice(dims, -1, 0.12, 1.0, 1001, None)
    ref, _ = _lattice(dims, -1, 0.12, 1.0, 1001, None, compress=False)
    g = to_gpu(synth.gaussian_spinor(dims, 3))
    c32 = to_host(lat.apply(g, prec=32))
    lat.set_compression(0)
    f32 = to_host(lat.apply(g, prec=32))
    assert np.array_equal(f32, to_host(ref.apply(g, prec=32)))
    # the two storages agree to FP32 rounding of the rebuilt row
    assert rel(c32, f32) <= 1e-6


def test_non_su3_links_refused():
    torch = require_gpu()
    from paper_1612_06556_amd import wcl
    dims = (4, 4, 4, 4)
    U = synth.su3_field(dims, 31)
    bad = U.copy()
    bad[5, 2] *= 1.001  # a link off the group by 1e-3
    lat = wcl.Lattice(dims, -1)
    lat.set_gauge(torch.from_numpy(bad).cuda())
    lat.set_params(0.12, 1.0)
    with pytest.raises(wcl.WclError) as ei:
        lat.set_compression(1)
    assert ei.value.code == wcl.WCL_EINVAL and "SU(3)" in str(ei.value)
    # the context keeps working with full links
    psi = synth.gaussian_spinor(dims, 32)
    orc = oracle.Oracle(dims, -1, 0.12, 1.0, bad)
    assert rel(to_host(lat.apply(to_gpu(psi), prec=32)), orc.D(psi)) <= 1e-6
    # SU(3) links accepted; a later non-SU(3) field is refused and leaves no gauge
    lat.set_gauge(torch.from_numpy(U).cuda())
    lat.set_compression(1)
    with pytest.raises(wcl.WclError):
        lat.set_gauge(torch.from_numpy(bad).cuda())
    with pytest.raises(wcl.WclError) as ei:
        lat.set_params(0.12, 1.0)
    assert ei.value.code == wcl.WCL_ESTATE


def test_bench_shape_24x32_compressed():
    dims = (24, 24, 24, 32)
    lat, U = _lattice(dims, -1, 0.126, 1.0, 1003, None)
    orc = oracle.Oracle(dims, -1, 0.126, 1.0, U)
    psi = synth.gaussian_spinor(dims, 2003)
    ref = orc.D(psi)
    g = to_gpu(psi)
    for prec in (32, 16):
        e = rel(to_host(lat.apply(g, prec=prec)), ref)
        print(f"D12 24^3x32 prec={prec} rel={e:.3e}", flush=True)
        assert e <= TOL[prec]
    for prec in (32, 16):
        ms = lat.bench_hop(prec, 50, 4)
        print(f"hop12 prec={prec} cold {ms * 1e3:.2f} us", flush=True)
        assert ms > 0


def test_ras_bench_shape_24x32():
    """The benchmark's Schwarz application at full size (24^3x32, two-row
    links, 1728 blocks, the per-site FP32 link copy): one application against
    the oracle's, norm-wise and site by site."""
    from paper_1612_06556_amd import wcl
    dims = (24, 24, 24, 32)
    lat, U = _lattice(dims, -1, 0.126, 1.0, 1003, None)
    orc = oracle.Oracle(dims, -1, 0.126, 1.0, U)
    psi = synth.gaussian_spinor(dims, 2004)
    psi[~even_mask(dims)] = 0
    lat.set_ras(1, 4)
    ref = orc.ras(psi, (4, 4, 4, 4), 1, 4)
    for prec, tol, stol in ((32, 1e-5, 1e-5), (16, 3e-3, 3e-3)):
        out = to_host(lat.apply_op(wcl.OP_RAS, to_gpu(psi), prec=prec))
        e, es = rel(out, ref), site_err(out, ref)
        print(f"RAS12 24^3x32 prec={prec} rel={e:.3e} site={es:.3e}", flush=True)
        assert e <= tol and es <= stol
    lat.close()


def test_long_lattice_24x96():
    """The paper's long single-card lattice 24^3x96 (links beyond the Infinity
    Cache): two-row FP32 / FP16 D against the oracle."""
    dims = (24, 24, 24, 96)
    lat, U = _lattice(dims, -1, 0.126, 1.0, 1006, None)
    orc = oracle.Oracle(dims, -1, 0.126, 1.0, U)
    psi = synth.gaussian_spinor(dims, 2006)
    ref = orc.D(psi)
    g = to_gpu(psi)
    for prec in (32, 16):
        e = rel(to_host(lat.apply(g, prec=prec)), ref)
        print(f"D12 24^3x96 prec={prec} rel={e:.3e}", flush=True)
        assert e <= TOL[prec]
