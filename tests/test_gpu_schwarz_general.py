"""Schwarz block solves with the block vectors in device memory: explicit
cores (8 x 4 x 4 x 8 and others), overlap 2, and the BiCGStab block solver,
against the FP64 oracle's RAS with the same recipe (the paper leaves the
Schwarz recipe open, Sec. 2).  The same path at the
fused kernel's settings must agree with the fused kernel.  FP32 block
arithmetic: 1e-5 relative (FP16 links and clover: 3e-3)."""
import numpy as np
import pytest

import oracle
from gpu_util import even_mask, rel, require_gpu, to_gpu, to_host
from paper_1612_06556_amd import synth

pytestmark = pytest.mark.gpu

TOL = {32: 1e-5, 16: 3e-3}


def _lattice(dims, seed, kappa=0.124, csw=1.0, tbc=-1, compress=False):
    torch = require_gpu()
    from paper_1612_06556_amd import wcl
    U = synth.su3_field(dims, seed)
    lat = wcl.Lattice(dims, tbc)
    if compress:
        lat.set_compression(1)
    lat.set_gauge(torch.from_numpy(U).cuda())
    lat.set_params(kappa, csw)
    return lat, oracle.Oracle(dims, tbc, kappa, csw, U)


def _even(dims, seed):
    v = synth.gaussian_spinor(dims, seed)
    v[~even_mask(dims)] = 0
    return v


def _ras(lat, v, prec):
    from paper_1612_06556_amd import wcl
    return to_host(lat.apply_op(wcl.OP_RAS, to_gpu(v), prec=prec))


# dims, cores (None: tiles), overlap, iters, solver
CASES = [
    ((8, 8, 8, 8), (4, 4, 4, 4), 1, 4, 0),     # explicit tile cores: MR on the device-memory path
    ((8, 8, 8, 8), (4, 4, 4, 4), 1, 3, 1),     # Jacobi
    ((8, 8, 8, 8), None, 1, 2, 2),             # BiCGStab block solver
    ((8, 8, 8, 8), None, 2, 4, 0),             # overlap 2: extended block 8^4, beyond LDS
    ((8, 8, 8, 8), (2, 2, 2, 2), 0, 3, 2),     # 2^4 cores, no overlap
    ((16, 8, 8, 16), (8, 4, 4, 8), 1, 4, 0),   # 8 x 4 x 4 x 8 cores (1800 sites per parity)
    ((16, 8, 8, 16), (8, 4, 4, 8), 1, 2, 2),
    ((4, 6, 8, 4), (2, 2, 4, 2), 1, 3, 2),     # non-cubic, 2^4 tiles
]


def _ids(c):
    return f"{'x'.join(map(str, c[0]))}_c{'x'.join(map(str, c[1])) if c[1] else 'tile'}_d{c[2]}_it{c[3]}_s{c[4]}"


@pytest.mark.parametrize("case", CASES, ids=_ids)
@pytest.mark.parametrize("prec,compress", [(32, False), (32, True), (16, False), (16, True)])
def test_general_schwarz_vs_oracle(case, prec, compress):
    dims, cores, overlap, iters, solver = case
    lat, orc = _lattice(dims, 1101, compress=compress)
    lat.set_ras_cores(cores)
    lat.set_ras(overlap, iters, solver)
    v = _even(dims, 1102)
    out = _ras(lat, v, prec)
    ref = orc.ras(v, cores if cores else (4, 4, 4, 4), overlap, iters, solver)   # tiles of an 8^4 lattice: 4^4
    e = rel(out, ref)
    print(f"general RAS {_ids(case)} prec={prec} r12={compress} rel={e:.3e}", flush=True)
    assert e <= TOL[prec]
    assert np.abs(out[~even_mask(dims)]).max() == 0.0
    lat.close()


@pytest.mark.parametrize("solver", [0, 1])
def test_device_memory_path_matches_fused(solver):
    """Explicit cores equal to the tiles run the device-memory path; it must
    agree with the fused LDS kernel to FP32 rounding."""
    dims = (8, 8, 8, 16)
    lat, _ = _lattice(dims, 1103, kappa=0.126)
    v = _even(dims, 1104)
    lat.set_ras(1, 4, solver)
    fused = _ras(lat, v, 32)
    lat.set_ras_cores((4, 4, 4, 4))
    general = _ras(lat, v, 32)
    lat.set_ras_cores(None)
    again = _ras(lat, v, 32)
    e = rel(general, fused)
    print(f"device-memory vs fused solver={solver} rel={e:.3e}", flush=True)
    assert e <= 1e-5
    assert np.array_equal(again, fused)
    lat.close()


@pytest.mark.parametrize("solver", [0, 2])
def test_general_zero_blocks(solver):
    """An input supported in one core: blocks whose extended region misses it
    return exactly zero (minimal residual stops at <q, q> = 0, BiCGStab at
    rho = 0), also after a dense call has filled the block fields."""
    dims = (8, 8, 8, 16)
    lat, orc = _lattice(dims, 1105, kappa=0.126)
    lat.set_ras_cores((4, 4, 4, 4))
    lat.set_ras(1, 3, solver)
    _ras(lat, _even(dims, 1106), 32)
    n = np.arange(int(np.prod(dims)))
    x = np.stack([n % 8, (n // 8) % 8, (n // 64) % 8, n // 512], axis=1)
    v = _even(dims, 1107)
    v[~np.all(x < 4, axis=1)] = 0
    out = _ras(lat, v, 32)
    assert rel(out, orc.ras(v, (4, 4, 4, 4), 1, 3, solver)) <= 1e-5
    assert np.abs(out[(x[:, 3] >= 8) & (x[:, 3] < 12)]).max() == 0.0
    lat.close()


@pytest.mark.parametrize("opts", [
    dict(ras_solver=2, ras_iters=2),
    dict(ras_overlap=2),
    dict(ras_solver=2, ras_iters=2, inner_prec=16, inner_vec_prec=16),
], ids=["bicgstab", "overlap2", "bicgstab_fp16_vectors"])
def test_solve_with_general_schwarz(opts):
    dims = (8, 8, 8, 8)
    lat, orc = _lattice(dims, 1001, kappa=0.12, compress=True)
    b = synth.gaussian_spinor(dims, 2001)
    x, info, rc = lat.solve(to_gpu(b), tol=1e-10, **opts)
    print("solve general", opts, info, flush=True)
    assert rc == 0 and info["true_relres"] <= 1e-10
    xr, _ = orc.bicgstab_eo(b, 1e-13, 10000)
    assert rel(to_host(x), xr) <= 1e-8
    lat.close()


def test_solve_large_cores_batched():
    """8 x 4 x 4 x 8 cores with two right-hand sides in one solve."""
    dims = (16, 8, 8, 16)
    lat, orc = _lattice(dims, 1108, kappa=0.124)
    lat.set_ras_cores((8, 4, 4, 8))
    b = synth.gaussian_spinor(dims, 1109, nrhs=2)
    x, infos, rc = lat.solve(to_gpu(b), tol=1e-10)
    assert rc == 0
    xh = to_host(x)
    for k in range(2):
        print("large cores rhs", k, infos[k], flush=True)
        assert infos[k]["true_relres"] <= 1e-10
        assert rel(orc.D(xh[k]), b[k]) <= 1e-10
    lat.close()


def test_solve_opts_ras_block():
    """opts.ras_block sets the Schwarz cores as wcl_set_ras_cores does: the
    solve is bitwise that of the explicit call, reaches the oracle's x, the
    cores stay for later solves, and bad cores are refused."""
    from paper_1612_06556_amd import wcl
    dims = (16, 8, 8, 16)
    lat, orc = _lattice(dims, 1112, kappa=0.124)
    b = synth.gaussian_spinor(dims, 1113)
    x1, i1, rc1 = lat.solve(to_gpu(b), tol=1e-10, ras_block=(8, 4, 4, 8))
    x2, i2, rc2 = lat.solve(to_gpu(b), tol=1e-10)            # the cores stay
    lat.set_ras_cores(None)
    x3, i3, rc3 = lat.solve(to_gpu(b), tol=1e-10)            # tile cores again
    lat.set_ras_cores((8, 4, 4, 8))
    x4, i4, rc4 = lat.solve(to_gpu(b), tol=1e-10)
    print("ras_block", i1, i3, flush=True)
    assert rc1 == rc2 == rc3 == rc4 == 0
    assert np.array_equal(to_host(x1), to_host(x4)) and np.array_equal(to_host(x2), to_host(x4))
    assert i1["inner_iters_total"] == i4["inner_iters_total"]
    assert not np.array_equal(to_host(x1), to_host(x3))
    xr, _ = orc.bicgstab_eo(b, 1e-13, 10000)
    assert rel(to_host(x1), xr) <= 1e-8
    for bad in ((3, 4, 4, 4), (16, 8, 8, 16)):   # odd; too large with overlap 1
        with pytest.raises(wcl.WclError) as ei:
            lat.solve(to_gpu(b), tol=1e-10, ras_block=bad)
        assert ei.value.code == wcl.WCL_EINVAL
    lat.close()


def test_general_schwarz_refusals():
    from paper_1612_06556_amd import wcl
    dims = (8, 8, 8, 8)
    lat, _ = _lattice(dims, 1110)
    for bad in ((3, 4, 4, 4), (4, 4, 4, 6), (8, 4, 4, 4)):   # odd, not dividing, too large with overlap 1
        with pytest.raises(wcl.WclError) as ei:
            lat.set_ras_cores(bad)
        assert ei.value.code == wcl.WCL_EINVAL
    lat.set_ras_cores((4, 4, 4, 4))
    with pytest.raises(wcl.WclError):
        lat.set_ras(1, 4, 0, 1)          # multiplicative on explicit cores
    with pytest.raises(wcl.WclError):
        lat.set_ras(1, 4, 3)             # unknown block solver
    lat.set_ras_cores(None)
    with pytest.raises(wcl.WclError):
        lat.set_ras(1, 2, 2, 1)          # multiplicative with BiCGStab
    lat.set_ras(1, 4, 0, 1)              # fused settings: accepted
    with pytest.raises(wcl.WclError):
        lat.set_ras_cores((4, 4, 4, 4))  # explicit cores while multiplicative
    lat.close()


@pytest.mark.parametrize("opts", [dict(ras_solver=2, ras_iters=2), dict(ras_overlap=2)],
                         ids=["bicgstab", "overlap2"])
def test_general_schwarz_graph_replay(opts):
    """The device-memory block solves inside a captured inner iteration
    (kernels only, block fields cleared by a kernel, no memset nodes): every
    replay of a multi-iteration solve, twice in a row, gives bitwise the
    eagerly launched solution, for two right-hand sides."""
    dims = (8, 8, 8, 8)
    lat, _ = _lattice(dims, 1001, kappa=0.12, compress=True)
    b = to_gpu(synth.gaussian_spinor(dims, 2001, nrhs=2))
    x0, i0, rc0 = lat.solve(b, tol=1e-10, use_graph=0, **opts)
    for _ in range(2):
        x1, i1, rc1 = lat.solve(b, tol=1e-10, use_graph=1, **opts)
        assert rc0 == 0 and rc1 == 0
        assert np.array_equal(to_host(x0), to_host(x1))
        assert [i["inner_iters_total"] for i in i0] == [i["inner_iters_total"] for i in i1]
    lat.close()


def test_schwarz_on_xrow_tiles():
    """On a layout whose tiles span whole x-rows (8x4x8x4 on 8^3x16) the tile
    cores cannot be extended by the overlap (WCL_EINVAL); explicit 4^4 cores
    run the device-memory block path: one RAS application against the
    oracle's RAS of the same recipe, and the solve reaches the oracle's x."""
    torch = require_gpu()
    from paper_1612_06556_amd import wcl
    dims = (8, 8, 8, 16)
    U = synth.su3_field(dims, 1120)
    lat = wcl.Lattice(dims, -1, (8, 4, 8, 4))
    lat.set_gauge(torch.from_numpy(U).cuda())
    lat.set_params(0.124, 1.0)
    orc = oracle.Oracle(dims, -1, 0.124, 1.0, U)
    b = synth.gaussian_spinor(dims, 1121)
    with pytest.raises(wcl.WclError) as ei:
        lat.solve(to_gpu(b), tol=1e-10)          # tile cores with overlap 1 exceed x
    assert ei.value.code == wcl.WCL_EINVAL
    lat.set_ras_cores((4, 4, 4, 4))
    v = _even(dims, 1122)
    for prec in (32, 16):
        e = rel(_ras(lat, v, prec), orc.ras(v, (4, 4, 4, 4), 1, 4, 0))
        print(f"xrow tiles RAS prec={prec} rel={e:.3e}", flush=True)
        assert e <= TOL[prec]
    x, info, rc = lat.solve(to_gpu(b), tol=1e-10)
    xr, _ = orc.bicgstab_eo(b, 1e-13, 10000)
    print("xrow tiles solve", info, flush=True)
    assert rc == 0 and rel(to_host(x), xr) <= 1e-8
    lat.close()
