"""GPU parity of every operator step against the FP64 oracle, through the
C ABI (wcl_apply / wcl_apply_op).

Tolerances (relative, norm-wise): FP64 path 1e-13; FP32 1e-6; FP16 storage
3e-3 -- the targets set for this hot path.  Lattices span several tiles and
a ragged last workgroup; the 24^3x32 case is the benchmark's shape."""
import numpy as np
import pytest

from gpu_util import even_mask, rel, setup, to_gpu, to_host
from paper_1612_06556_amd import synth

pytestmark = pytest.mark.gpu

TOL = {64: 1e-13, 32: 1e-6, 16: 3e-3}
CASES = [  # dims, tbc, kappa, csw, seed, tile
    ((8, 8, 8, 8), -1, 0.12, 1.0, 1001, None),
    ((4, 6, 8, 4), -1, 0.125, 1.3, 7, None),        # 2^4 tiles, Vh = 384: ragged workgroup
    ((6, 4, 4, 8), 1, 0.126, 1.0, 8, (2, 2, 2, 4)),  # periodic, non-cubic tile
    ((8, 8, 8, 16), -1, 0.126, 1.0, 9, (4, 4, 4, 4)),
    ((8, 8, 8, 16), -1, 0.126, 1.0, 11, (8, 4, 8, 4)),  # tiles spanning whole x-rows (and z)
]


def _ids(c):
    return "x".join(map(str, c[0])) + f"_tbc{c[1]}" + ("_tile" + "x".join(map(str, c[5])) if c[5] else "")


@pytest.mark.parametrize("case", CASES, ids=_ids)
@pytest.mark.parametrize("prec", [64, 32, 16])
def test_D_and_Ddag(case, prec):
    dims, tbc, kappa, csw, seed, tile = case
    lat, orc, _ = setup(dims, tbc, kappa, csw, seed, tile)
    psi = synth.gaussian_spinor(dims, seed + 1)
    g = to_gpu(psi)
    for dag in (False, True):
        out = to_host(lat.apply(g, dagger=dag, prec=prec))
        ref = orc.D(psi, dagger=dag)
        e = rel(out, ref)
        print(f"D dims={dims} prec={prec} dag={dag} rel={e:.3e}", flush=True)
        assert e <= TOL[prec]


@pytest.mark.parametrize("case", CASES[:2], ids=_ids)
@pytest.mark.parametrize("prec", [64, 32, 16])
def test_hop_clover_schur(case, prec):
    from paper_1612_06556_amd import wcl
    dims, tbc, kappa, csw, seed, tile = case
    lat, orc, _ = setup(dims, tbc, kappa, csw, seed, tile)
    psi = synth.gaussian_spinor(dims, seed + 2)
    ev = even_mask(dims)
    g = to_gpu(psi)
    pe = psi.copy()
    pe[~ev] = 0
    checks = {
        "hop": (wcl.OP_HOP, orc.hop(psi)),
        "clover": (wcl.OP_CLOVER, orc.clover(psi)),
        "clover_inv": (wcl.OP_CLOVER_INV, orc.clover_inv(psi)),
        "schur": (wcl.OP_SCHUR, orc.schur(pe)),
    }
    if prec == 64:
        checks["schur_rhs"] = (wcl.OP_SCHUR_RHS, orc.schur_rhs(psi))
    for name, (op, ref) in checks.items():
        out = to_host(lat.apply_op(op, g, prec=prec))
        e = rel(out, ref)
        print(f"{name} dims={dims} prec={prec} rel={e:.3e}", flush=True)
        assert e <= TOL[prec], name


@pytest.mark.parametrize("case", [CASES[0], CASES[3]], ids=_ids)
@pytest.mark.parametrize("prec", [32, 16])
def test_ras_block_solve(case, prec):
    """One RAS application (4^4 cores, overlap 1, 4 MR steps) vs the oracle's
    FP64 RAS with the same recipe: 1e-5 in FP32 arithmetic, 3e-3 with FP16
    links and clover."""
    from paper_1612_06556_amd import wcl
    dims, tbc, kappa, csw, seed, tile = case
    lat, orc, _ = setup(dims, tbc, kappa, csw, seed, tile)
    psi = synth.gaussian_spinor(dims, seed + 3)
    psi[~even_mask(dims)] = 0
    lat.set_ras(1, 4)
    out = to_host(lat.apply_op(wcl.OP_RAS, to_gpu(psi), prec=prec))
    ref = orc.ras(psi, (4, 4, 4, 4), 1, 4)
    e = rel(out, ref)
    print(f"ras dims={dims} prec={prec} rel={e:.3e}", flush=True)
    assert e <= (1e-5 if prec == 32 else 3e-3)


@pytest.mark.parametrize("overlap,solver,iters", [(1, 1, 4), (0, 0, 4), (0, 1, 3)])
def test_ras_variants(overlap, solver, iters):
    """Block Jacobi steps and overlap 0 against the oracle's RAS (FP32, 1e-5)."""
    from paper_1612_06556_amd import wcl
    dims = (8, 8, 8, 16)
    lat, orc, _ = setup(dims, -1, 0.126, 1.0, 9, (4, 4, 4, 4))
    psi = synth.gaussian_spinor(dims, 15)
    psi[~even_mask(dims)] = 0
    lat.set_ras(overlap, iters, solver)
    try:
        out = to_host(lat.apply_op(wcl.OP_RAS, to_gpu(psi), prec=32))
    finally:
        lat.set_ras(1, 4, 0)
    ref = orc.ras(psi, (4, 4, 4, 4), overlap, iters, solver)
    e = rel(out, ref)
    print(f"ras overlap={overlap} solver={solver} rel={e:.3e}", flush=True)
    assert e <= 1e-5


@pytest.mark.parametrize("prec,overlap,solver", [(32, 1, 0), (16, 1, 0), (32, 0, 1)])
def test_sap_application(prec, overlap, solver):
    """Multiplicative Schwarz (16 colour sweeps with residual updates) against
    the oracle's: FP32 1e-5, FP16 links and clover 3e-3."""
    from paper_1612_06556_amd import wcl
    dims = (8, 8, 8, 16)
    lat, orc, _ = setup(dims, -1, 0.126, 1.0, 9, (4, 4, 4, 4))
    psi = synth.gaussian_spinor(dims, 17)
    psi[~even_mask(dims)] = 0
    lat.set_ras(overlap, 4, solver, 1)
    try:
        out = to_host(lat.apply_op(wcl.OP_RAS, to_gpu(psi), prec=prec))
    finally:
        lat.set_ras(1, 4, 0, 0)
    ref = orc.sap(psi, (4, 4, 4, 4), overlap, 4, solver)
    e = rel(out, ref)
    print(f"sap prec={prec} overlap={overlap} solver={solver} rel={e:.3e}", flush=True)
    assert e <= (1e-5 if prec == 32 else 3e-3)


def test_ras_small_cores():
    """2^4 cores with overlap 1 on a 4x4x4x8 lattice (extended block = 4^4)."""
    from paper_1612_06556_amd import wcl
    dims = (4, 4, 4, 8)
    lat, orc, _ = setup(dims, -1, 0.125, 1.0, 12, (2, 2, 2, 2))
    psi = synth.gaussian_spinor(dims, 13)
    psi[~even_mask(dims)] = 0
    lat.set_ras(1, 3)
    out = to_host(lat.apply_op(wcl.OP_RAS, to_gpu(psi), prec=32))
    ref = orc.ras(psi, (2, 2, 2, 2), 1, 3)
    assert rel(out, ref) <= 1e-5
    # two-row links (the per-site FP32 copy; FP16) on the small-block kernel
    lat.set_compression(1)
    for prec, tol in ((32, 1e-5), (16, 3e-3)):
        out = to_host(lat.apply_op(wcl.OP_RAS, to_gpu(psi), prec=prec))
        assert rel(out, ref) <= tol


def test_multi_rhs_apply():
    dims = (8, 8, 8, 8)
    lat, orc, _ = setup(dims, -1, 0.12, 1.0, 1001, None)
    psi = synth.gaussian_spinor(dims, 5, nrhs=3)
    out = to_host(lat.apply(to_gpu(psi), prec=32))
    for k in range(3):
        assert rel(out[k], orc.D(psi[k])) <= 1e-6


def test_bench_shape_24x32():
    """The benchmark's lattice: FP32 and FP16 D against the oracle at 24^3x32."""
    dims = (24, 24, 24, 32)
    lat, orc, _ = setup(dims, -1, 0.126, 1.0, 1003, None)
    psi = synth.gaussian_spinor(dims, 2003)
    g = to_gpu(psi)
    ref = orc.D(psi)
    for prec in (32, 16):
        e = rel(to_host(lat.apply(g, prec=prec)), ref)
        print(f"D 24^3x32 prec={prec} rel={e:.3e}", flush=True)
        assert e <= TOL[prec]


def test_ras_op_launch_accounting():
    """One RAS application through wcl_apply_op is one launch over the tiles
    of one right-hand side: its recorded work equals the single-rhs count."""
    from paper_1612_06556_amd import wcl
    dims = (8, 8, 8, 8)
    lat, orc, _ = setup(dims, -1, 0.12, 1.0, 1001, None)
    psi = synth.gaussian_spinor(dims, 3)
    lat.set_ras(1, 4)
    wcl.wcl_profile(lat.h, 1)
    lat.apply_op(wcl.OP_RAS, to_gpu(psi), prec=32)
    st = wcl.wcl_profile_read(lat.h, wcl.K_RAS)
    wcl.wcl_profile(lat.h, 0)
    # per block and MR step: in-block hops x 168 + 1296 x 504 + 648 x 240; 16 tiles, 4 steps
    hops = 2 * 4 * 5 * 6 ** 3
    expect = (hops * 168 + 1296 * 504 + 648 * 240) * 4 * 16
    assert st["launches"] == 1
    assert st["flops"] == expect


def test_profile_mask_times_selected_classes():
    """With the class mask set to RAS only, RAS launches carry timing events
    and hop launches are counted (launches, flops) with no time; the full
    mask times both again."""
    from paper_1612_06556_amd import wcl
    dims = (8, 8, 8, 8)
    lat, _, _ = setup(dims, -1, 0.12, 1.0, 1001, None)
    b = to_gpu(synth.gaussian_spinor(dims, 2001))
    lat.set_ras(1, 4)
    for mask, hop_timed in ((1 << wcl.K_RAS, False), (7, True)):
        wcl.wcl_profile(lat.h, 1)
        wcl.wcl_profile_mask(lat.h, mask)
        lat.solve(b, tol=1e-10)
        hop = wcl.wcl_profile_read(lat.h, wcl.K_HOP)
        ras = wcl.wcl_profile_read(lat.h, wcl.K_RAS)
        wcl.wcl_profile(lat.h, 0)
        assert hop["launches"] > 0 and hop["flops"] > 0 and ras["launches"] > 0
        assert ras["ms"] > 0
        assert (hop["ms"] > 0) == hop_timed
    wcl.wcl_profile_mask(lat.h, 15)
    with pytest.raises(wcl.WclError):
        wcl.wcl_profile_mask(lat.h, 16)


def test_bench_entry_points():
    """wcl_bench_hop / wcl_bench_clover run on rotating copies and leave the
    context's fields intact (D still matches the oracle afterwards)."""
    dims = (8, 8, 8, 16)
    lat, orc, _ = setup(dims, -1, 0.126, 1.0, 9, (4, 4, 4, 4))
    for prec in (32, 16):
        assert lat.bench_hop(prec, 5, 3) > 0
        assert lat.bench_clover(prec, 5, 3) > 0
    psi = synth.gaussian_spinor(dims, 41)
    assert rel(to_host(lat.apply(to_gpu(psi), prec=32)), orc.D(psi)) <= 1e-6


def test_stream_ceiling_entry_point():
    """wcl_bench_stream returns positive read and copy rates on a small buffer."""
    from paper_1612_06556_amd import wcl
    lat, _, _ = setup((8, 8, 8, 8), -1, 0.12, 1.0, 1001, None)
    r, c = wcl.wcl_bench_stream(lat.h, 16, 3)
    assert r > 0 and c > 0
    with pytest.raises(wcl.WclError):
        wcl.wcl_bench_stream(lat.h, 0.5, 3)


@pytest.mark.parametrize("prec", [32, 16])
def test_ras_zero_blocks(prec):
    """Blocks whose input is zero return zero (regression: their output was
    left as the previous call's).  First a dense input fills the output, then
    an input supported in one core only is compared with the oracle."""
    from paper_1612_06556_amd import wcl
    dims = (8, 8, 8, 16)
    lat, orc, _ = setup(dims, -1, 0.126, 1.0, 9, (4, 4, 4, 4))
    lat.set_ras(1, 4, 0)
    dense = synth.gaussian_spinor(dims, 71)
    dense[~even_mask(dims)] = 0
    lat.apply_op(wcl.OP_RAS, to_gpu(dense), prec=prec)
    n = np.arange(int(np.prod(dims)))
    x = np.stack([n % 8, (n // 8) % 8, (n // 64) % 8, n // 512], axis=1)
    v = synth.gaussian_spinor(dims, 72)
    v[~(np.all(x < 4, axis=1) & even_mask(dims))] = 0
    out = to_host(lat.apply_op(wcl.OP_RAS, to_gpu(v), prec=prec))
    ref = orc.ras(v, (4, 4, 4, 4), 1, 4)
    e = rel(out, ref)
    print(f"ras zero blocks prec={prec} rel={e:.3e}", flush=True)
    assert e <= (1e-5 if prec == 32 else 3e-3)
    # cores at t = 8..11: their extended blocks (t = 7..12) miss the support
    assert np.abs(out[(x[:, 3] >= 8) & (x[:, 3] < 12)]).max() == 0.0


def test_xrow_tiles_bench_layout():
    """The layout the benchmark times its cold hops on besides 4^4 tiles:
    24x4x8x4 tiles (whole x-rows) at 24^3x32.  H and D in FP32 and FP16,
    full and two-row links, with the autotuned launch shape under temporal
    and non-temporal loads, against the oracle (norm-wise and per site);
    staged and unstaged give bitwise one result."""
    from paper_1612_06556_amd import wcl
    from gpu_util import site_err
    dims = (24, 24, 24, 32)
    lat, orc, _ = setup(dims, -1, 0.126, 1.0, 1003, (24, 4, 8, 4))
    psi = synth.gaussian_spinor(dims, 2003)
    g = to_gpu(psi)
    ref_hop, ref_d = orc.hop(psi), orc.D(psi)
    site_tol = {32: 1e-5, 16: 3e-2}   # 10x the norm-wise bound, as the launch-shape tests
    for comp in (0, 1):
        lat.set_compression(comp)
        for prec in (32, 16):
            for nt in (1, 0):
                wcl.wcl_set_tuning(lat.h, 128, 2, 1, nt)
                t = lat.autotune(prec, 1, wcl.TUNE_HOP)
                hop = lat.apply_op(wcl.OP_HOP, g, prec=prec)
                d = to_host(lat.apply(g, prec=prec))
                wcl.wcl_set_hop_staging(lat.h, 0)
                hop_u = lat.apply_op(wcl.OP_HOP, g, prec=prec)
                wcl.wcl_set_hop_staging(lat.h, 1)
                assert bool((hop == hop_u).all())
                hop = to_host(hop)
                e_h, e_d = rel(hop, ref_hop), rel(d, ref_d)
                s_h = site_err(hop, ref_hop)
                print(f"xrow tiles comp={comp} prec={prec} nt={nt} shape={t['hop_block']}/{t['hop_depth']}/"
                      f"{t['hop_tiles']} hop rel={e_h:.3e} site={s_h:.3e} D rel={e_d:.3e}", flush=True)
                assert e_h <= TOL[prec] and e_d <= TOL[prec] and s_h <= site_tol[prec]
    wcl.wcl_set_tuning(lat.h, 256, 2, 1, 0)


def test_hop_variants_bitwise_many_rhs():
    """Every launch variant of the hop and of the Schur operator (workgroup
    64 / 128 / 256, LDS staging on or off, pipeline depth 2 or 3) gives
    bitwise the same result in FP32 and with FP16 storage, with full and
    two-row links, over 12 right-hand sides at 16^3x32: 19 million outputs
    per check, so that a rounding difference between variants (one fused
    multiply-add paired differently) shows.  The first variant matches the
    oracle."""
    from paper_1612_06556_amd import wcl
    dims = (16, 16, 16, 32)
    lat, orc, _ = setup(dims, -1, 0.126, 1.0, 1003)
    psi = np.stack([synth.gaussian_spinor(dims, 600 + k) for k in range(12)])
    pe = psi.copy()
    pe[:, ~even_mask(dims)] = 0
    g, ge = to_gpu(psi), to_gpu(pe)
    refs = {wcl.OP_HOP: orc.hop(psi[0]), wcl.OP_SCHUR: orc.schur(pe[0])}
    variants = [(blk, 2, stage) for blk in (64, 128, 256) for stage in (1, 0)] + [(blk, 3, 0) for blk in (64, 128, 256)]
    for comp in (0, 1):
        lat.set_compression(comp)
        for prec in (32, 16):
            for op, inp in ((wcl.OP_HOP, g), (wcl.OP_SCHUR, ge)):
                first = None
                for blk, depth, stage in variants:
                    wcl.wcl_set_tuning(lat.h, blk, depth, 1, 0)
                    wcl.wcl_set_hop_staging(lat.h, stage)
                    out = lat.apply_op(op, inp, prec=prec)
                    if first is None:
                        first = out
                        e = rel(to_host(out[0]), refs[op])
                        print(f"variants comp={comp} prec={prec} op={op} oracle rel={e:.3e}", flush=True)
                        assert e <= TOL[prec]
                    else:
                        assert bool((out == first).all()), (comp, prec, op, blk, depth, stage)
    wcl.wcl_set_tuning(lat.h, 256, 2, 1, 0)
    wcl.wcl_set_hop_staging(lat.h, 1)


@pytest.mark.parametrize("case", CASES, ids=_ids)
@pytest.mark.parametrize("block", [64, 128, 256])
def test_hop_staging(case, block):
    """Staged input spinors (LDS copy of the workgroup's own half-sites), with
    temporal or non-temporal operator loads, give bitwise the unstaged
    kernel's result for every workgroup size, on ragged last workgroups and
    for batched right-hand sides; all match the oracle."""
    from paper_1612_06556_amd import wcl
    dims, tbc, kappa, csw, seed, tile = case
    lat, orc, _ = setup(dims, tbc, kappa, csw, seed, tile)
    psi = synth.gaussian_spinor(dims, seed + 7, nrhs=2)
    g = to_gpu(psi)
    pe = psi[0].copy()
    pe[~even_mask(dims)] = 0
    ge = to_gpu(pe)
    for prec in (64, 32, 16):
        res = {}
        for stage, nt in ((1, 0), (0, 0), (1, 1), (0, 1)):   # staged / unstaged, temporal / non-temporal
            wcl.wcl_set_tuning(lat.h, block, 2, 1, nt)
            wcl.wcl_set_hop_staging(lat.h, stage)
            res[stage, nt] = (to_host(lat.apply(g, prec=prec)), to_host(lat.apply_op(wcl.OP_HOP, g[0], prec=prec)),
                              to_host(lat.apply_op(wcl.OP_SCHUR, ge, prec=prec)))
        wcl.wcl_set_tuning(lat.h, 256, 2, 1, 0)
        wcl.wcl_set_hop_staging(lat.h, 1)
        for key in ((0, 0), (1, 1), (0, 1)):
            for a, b in zip(res[1, 0], res[key]):
                assert np.array_equal(a, b)
        d, hop, schur = res[1, 0]
        for k in range(2):
            assert rel(d[k], orc.D(psi[k])) <= TOL[prec]
        assert rel(hop, orc.hop(psi[0])) <= TOL[prec]
        assert rel(schur, orc.schur(pe)) <= TOL[prec]
        print(f"staging dims={dims} block={block} prec={prec} ok", flush=True)
