"""Every launch shape of the hopping kernel that the solver or the autotuner
can select, against the FP64 oracle (through the C ABI).

wcl_autotune_hop chooses among 64/128/256 threads per workgroup, pipeline
depth 2 or 3, XCD-aware or plain workgroup order and 1/2/4/8 site blocks per
workgroup; wcl_set_tuning adds non-temporal operator loads and
wcl_set_hop_staging the LDS copy of the input spinors.  Each shape is a different kernel instantiation (for full or two-row
links, FP32 or FP16 storage), so each is compared with the oracle: D, the
hopping term H and the Schur operator Dhat, norm-wise (FP32 1e-6, FP16 3e-3)
and site by site (largest site error over the rms site norm <= 10x the
norm-wise bound, so that one wrong site cannot hide in the norm)."""
import itertools

import numpy as np
import pytest

from gpu_util import even_mask, rel, setup, site_err, to_gpu, to_host
from paper_1612_06556_amd import synth

pytestmark = pytest.mark.gpu

TOL = {32: 1e-6, 16: 3e-3}
CASES = [  # dims, tbc, kappa, csw, seed, tile
    ((8, 8, 8, 8), -1, 0.12, 1.0, 1001, None),
    ((4, 6, 8, 4), -1, 0.125, 1.3, 7, None),          # 2^4 tiles, ragged last workgroup
    ((24, 24, 24, 32), -1, 0.126, 1.0, 1003, None),   # the benchmark's lattice
    ((8, 8, 8, 16), -1, 0.126, 1.0, 1005, (8, 4, 8, 4)),  # tiles spanning whole x-rows
]
# block, depth, xcd, nt, stage, site blocks per workgroup
SHAPES = [s + (1,) for s in itertools.product((64, 128, 256), (2, 3), (0, 1), (0, 1), (1, 0))]
SHAPES += [s + (t,) for s in itertools.product((64, 128, 256), (2, 3), (0, 1), (0, 1), (1,)) for t in (2, 4, 8)]

_refs = {}


def _reference(case, orc, psi, pe):
    key = (case[0], case[4])
    if key not in _refs:
        _refs.clear()
        _refs[key] = (orc.D(psi), orc.hop(psi), orc.schur(pe))
    return _refs[key]


def _ids(c):
    return "x".join(map(str, c[0]))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("case", CASES, ids=_ids)
@pytest.mark.parametrize("compress", [0, 1])
def test_every_hop_shape(case, compress):
    from paper_1612_06556_amd import wcl
    dims, tbc, kappa, csw, seed, tile = case
    lat, orc, _ = setup(dims, tbc, kappa, csw, seed, tile)
    psi = synth.gaussian_spinor(dims, seed + 11)
    pe = psi.copy()
    pe[~even_mask(dims)] = 0
    g, ge = to_gpu(psi), to_gpu(pe)
    ref_d, ref_h, ref_s = _reference(case, orc, psi, pe)
    worst = {}
    lat.set_compression(compress)
    try:
        for prec in (32, 16):
            for block, depth, xcd, nt, stage, tpw in SHAPES:
                wcl.wcl_set_tuning(lat.h, block, depth, xcd, nt)
                wcl.wcl_set_hop_staging(lat.h, stage)
                wcl.wcl_set_hop_tiles(lat.h, tpw)
                outs = (to_host(lat.apply(g, prec=prec)), to_host(lat.apply_op(wcl.OP_HOP, g, prec=prec)),
                        to_host(lat.apply_op(wcl.OP_SCHUR, ge, prec=prec)))
                for name, out, ref in zip(("D", "H", "Dhat"), outs, (ref_d, ref_h, ref_s)):
                    e, es = rel(out, ref), site_err(out, ref)
                    tag = (prec, name)
                    worst[tag] = max(worst.get(tag, (0.0, 0.0)), (e, es))
                    assert e <= TOL[prec] and es <= 10 * TOL[prec], (prec, block, depth, xcd, nt, stage, tpw, name,
                                                                     e, es)
    finally:
        wcl.wcl_set_tuning(lat.h, 256, 2, 1, 0)
        wcl.wcl_set_hop_staging(lat.h, 1)
        wcl.wcl_set_hop_tiles(lat.h, 1)
        lat.set_compression(0)
    for tag, (e, es) in sorted(worst.items()):
        print(f"dims={dims} compress={compress} prec={tag[0]} {tag[1]}: worst rel {e:.2e}, worst site {es:.2e} "
              f"over {len(SHAPES)} shapes", flush=True)


def test_autotuner_picks_a_tested_shape():
    """The autotuner's choice is one of the shapes compared above, and the
    operator it leaves selected still matches the oracle."""
    from paper_1612_06556_amd import wcl
    case = CASES[0]
    dims, tbc, kappa, csw, seed, tile = case
    lat, orc, _ = setup(dims, tbc, kappa, csw, seed, tile)
    try:
        for compress, prec in ((0, 32), (1, 32), (1, 16)):
            lat.set_compression(compress)
            best = wcl.wcl_autotune_hop(lat.h, prec, 2)
            assert (best["hop_block"], best["hop_depth"], best["hop_xcd"]) in {s[:3] for s in SHAPES}
            psi = synth.gaussian_spinor(dims, 77)
            out = to_host(lat.apply(to_gpu(psi), prec=prec))
            ref = orc.D(psi)
            assert rel(out, ref) <= TOL[prec] and site_err(out, ref) <= 10 * TOL[prec]
    finally:
        wcl.wcl_set_tuning(lat.h, 256, 2, 1, 0)
        lat.set_compression(0)


@pytest.mark.parametrize("nrhs", [1, 12])
def test_bench_hop_batched(nrhs):
    """wcl_bench_hop times nrhs right-hand sides per launch (the 12-source
    propagator batch) and leaves the context's fields intact."""
    from paper_1612_06556_amd import wcl
    dims = (8, 8, 8, 16)
    lat, orc, _ = setup(dims, -1, 0.126, 1.0, 9, (4, 4, 4, 4))
    for rpt in (1, 4):
        wcl.wcl_set_batch_tuning(lat.h, rpt)
        assert lat.bench_hop(32, 5, 2, nrhs=nrhs) > 0
        assert lat.bench_hop(16, 5, 2, nrhs=nrhs) > 0
    wcl.wcl_set_batch_tuning(lat.h, 1)
    with pytest.raises(wcl.WclError):
        lat.bench_hop(32, 5, 2, nrhs=65)
    psi = synth.gaussian_spinor(dims, 41)
    assert rel(to_host(lat.apply(to_gpu(psi), prec=32)), orc.D(psi)) <= 1e-6


def test_project_autotuner():
    """wcl_autotune: the hop shape, the batched right-hand sides per thread and
    the Schwarz choice (by measured time to solution) come from the parity-tested
    candidate sets; the result is cached per (lattice, precision, nrhs, flags);
    the operator and a solve with the chosen recipe still match the oracle."""
    from paper_1612_06556_amd import wcl
    dims = (8, 8, 8, 16)
    lat, orc, _ = setup(dims, -1, 0.126, 1.0, 9, (4, 4, 4, 4))
    try:
        t = lat.autotune(32, 1, wcl.TUNE_HOP)
        assert t["cached"] == 0 and (t["hop_block"], t["hop_depth"], t["hop_xcd"], t["hop_tiles"]) in \
            {(s[0], s[1], s[2], s[5]) for s in SHAPES}
        assert lat.autotune(32, 1, wcl.TUNE_HOP)["cached"] == 1
        tb = lat.autotune(16, 4, wcl.TUNE_HOP | wcl.TUNE_BATCH)
        assert tb["rhs_per_thread"] in (1, 2, 4)
        psi = synth.gaussian_spinor(dims, 81)
        for prec in (32, 16):
            out = to_host(lat.apply(to_gpu(psi), prec=prec))
            assert rel(out, orc.D(psi)) <= TOL[prec]
        b = synth.gaussian_spinor(dims, 82)
        opts = dict(tol=1e-10, inner_tol=1e-1, use_ras=1, ras_overlap=1)
        ts = lat.autotune(32, 1, wcl.TUNE_SCHWARZ, b=to_gpu(b), **opts)
        print("autotuned", t, tb, ts, flush=True)
        assert (ts["use_ras"], ts["ras_overlap"]) in {(1, 1), (1, 0), (0, 1)} and ts["solve_ms"] > 0
        x, info, rc = lat.solve(to_gpu(b), **dict(opts, use_ras=ts["use_ras"], ras_overlap=ts["ras_overlap"]))
        xr, _ = orc.bicgstab_eo(b, 1e-13, 20000)
        assert rc == 0 and rel(to_host(x), xr) <= 1e-8
        with pytest.raises(wcl.WclError):
            lat.autotune(32, 1, wcl.TUNE_SCHWARZ)   # needs a source and options
    finally:
        wcl.wcl_set_tuning(lat.h, 256, 2, 1, 0)
        wcl.wcl_set_hop_tiles(lat.h, 1)
        wcl.wcl_set_batch_tuning(lat.h, 1)
        lat.set_ras(1, 4, 0, 0)
