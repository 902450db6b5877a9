"""wcl_apply_noalloc (the D application that allocates nothing, for callers
that cannot call hipMalloc) against wcl_apply, through the C ABI.

Both run the same kernels, so the results must agree bitwise; both are also
compared with the FP64 oracle at the D tolerances (FP64 1e-13, FP32 1e-6,
FP16 storage 3e-3).  Two calls in a row share the GPU's one fixed scratch
array: the first on 16^3x32 with two right-hand sides, the second on a
smaller lattice with one; a lattice beyond the scratch size is refused."""
import numpy as np
import pytest

import oracle
from gpu_util import rel, require_gpu, site_err, to_gpu, to_host
from paper_1612_06556_amd import synth

pytestmark = pytest.mark.gpu

TOL = {64: 1e-13, 32: 1e-6, 16: 3e-3}


def _lattice(dims, seed, kappa, compress=0):
    torch = require_gpu()
    from paper_1612_06556_amd import wcl
    U = synth.su3_field(dims, seed)
    lat = wcl.Lattice(dims, -1)
    lat.set_compression(compress)
    lat.set_gauge(torch.from_numpy(U).cuda())
    lat.set_params(kappa, 1.0)
    return lat, oracle.Oracle(dims, -1, kappa, 1.0, U)


def _noalloc(lat, psi, dagger, prec):
    from paper_1612_06556_amd import wcl
    torch = require_gpu()
    g, nrhs = lat._spinors(psi)
    out = torch.empty_like(g)
    lat._sync_stream()
    wcl.wcl_apply_noalloc(lat.h, g.data_ptr(), out.data_ptr(), nrhs, int(dagger), prec)
    return to_host(out)


def test_noalloc_matches_apply_two_calls():
    big, orc_big = _lattice((16, 16, 16, 32), 1002, 0.125)
    small, orc_small = _lattice((8, 8, 8, 8), 1001, 0.12, compress=1)
    psi_big = synth.gaussian_spinor((16, 16, 16, 32), 91, nrhs=2)
    psi_small = synth.gaussian_spinor((8, 8, 8, 8), 92)
    for prec in (64, 32, 16):
        for dagger in (0, 1):
            for lat, orc, psi in ((big, orc_big, psi_big), (small, orc_small, psi_small)):
                out = _noalloc(lat, to_gpu(psi), dagger, prec)
                ref_lib = to_host(lat.apply(to_gpu(psi), dagger=bool(dagger), prec=prec))
                assert np.array_equal(out, ref_lib), (lat.dims, prec, dagger)
                for k, p in enumerate(psi.reshape(-1, *psi.shape[-3:])):
                    o = out.reshape(-1, *psi.shape[-3:])[k]
                    ref = orc.D(p, dagger=bool(dagger))
                    e, es = rel(o, ref), site_err(o, ref)
                    assert e <= TOL[prec] and es <= 10 * TOL[prec], (lat.dims, prec, dagger, e, es)
                print(f"noalloc dims={lat.dims} prec={prec} dagger={dagger}: bitwise = wcl_apply", flush=True)
    big.close()
    small.close()


def test_noalloc_refuses_a_lattice_beyond_the_scratch():
    torch = require_gpu()
    from paper_1612_06556_amd import wcl
    dims = (16, 16, 16, 48)   # 196608 sites > 174762
    lat = wcl.Lattice(dims, -1)
    lat.set_gauge(torch.from_numpy(synth.unit_field(dims)).cuda())
    lat.set_params(0.12, 1.0)
    psi = to_gpu(synth.gaussian_spinor(dims, 3))
    out = torch.empty_like(psi)
    with pytest.raises(wcl.WclError) as e:
        wcl.wcl_apply_noalloc(lat.h, psi.data_ptr(), out.data_ptr(), 1, 0, 32)
    assert e.value.code == wcl.WCL_EINVAL and "scratch" in str(e.value)
    lat.close()
