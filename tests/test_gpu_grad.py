"""Backward pass on the GPU: adjoint solve, link and kappa gradients.

* wcl_grad against the oracle's gradient formula on the same (x, y), FP64
  both sides: 1e-10 (8^4 and the differentiation config's 16^3x32);
* the autograd gradient against FP64 central finite differences of
  L = Re<eta, D^-1 b> (GPU solves to 1e-12) on 4^4 and 6^4 lattices: 1e-5;
* grad_b = D^-dag eta against the oracle's dense-free check D^dag y = eta."""
import numpy as np
import pytest

from gpu_util import rel, setup, to_gpu, to_host
from paper_1612_06556_amd import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dims,kappa", [((8, 8, 8, 8), 0.12), ((16, 16, 16, 32), 0.125)])
def test_grad_kernel_vs_oracle(dims, kappa):
    lat, orc, _ = setup(dims, -1, kappa, 1.0, 1005, None)
    x = synth.gaussian_spinor(dims, 2005)
    y = synth.gaussian_spinor(dims, 3005)
    gU, gk = lat.grad(to_gpu(x), to_gpu(y))
    gU_o, gk_o = orc.grad(x, y)
    e = rel(to_host(gU), gU_o)
    print(f"grad dims={dims} link rel={e:.3e} kappa {gk:.12e} vs {gk_o:.12e}", flush=True)
    assert e <= 1e-10
    assert abs(gk - gk_o) <= 1e-10 * abs(gk_o)


def test_adjoint_solve():
    from paper_1612_06556_amd import wcl
    dims = (8, 8, 8, 8)
    lat, orc, _ = setup(dims, -1, 0.12, 1.0, 1001, None)
    eta = synth.gaussian_spinor(dims, 77)
    y, info, rc = lat.solve(to_gpu(eta), adjoint=1)
    y = to_host(y)
    assert rc == 0
    assert np.linalg.norm(eta - orc.D(y, dagger=True)) / np.linalg.norm(eta) <= 1e-10


def _loss_gpu(lat, U, kappa, b, eta, tile_opts):
    import torch
    lat.set_gauge(torch.from_numpy(U).cuda())
    lat.set_params(kappa, 1.0)
    x, info, rc = lat.solve(to_gpu(b), **tile_opts)
    return float(np.vdot(eta, to_host(x)).real)


@pytest.mark.parametrize("dims,tile", [((4, 4, 4, 4), (2, 2, 2, 2)), ((6, 6, 6, 6), (2, 2, 2, 2))])
def test_autograd_vs_finite_differences(dims, tile):
    import torch
    from paper_1612_06556_amd import autograd, wcl
    kappa = 0.125
    U = synth.su3_field(dims, 1005)
    b = synth.gaussian_spinor(dims, 2005)
    eta = synth.gaussian_spinor(dims, 3005)
    lat = wcl.Lattice(dims, -1, tile)
    opts = dict(tol=1e-12, use_ras=1)
    tU = torch.from_numpy(U).cuda().requires_grad_(True)
    tk = torch.tensor(kappa, dtype=torch.float64, requires_grad=True)
    tb = torch.from_numpy(b).cuda().requires_grad_(True)
    x = autograd.solve(tU, tk, tb, lat, 1.0, **opts)
    L = torch.real(torch.vdot(torch.from_numpy(eta).cuda().reshape(-1), x.reshape(-1)))
    L.backward()
    gU = to_host(tU.grad)
    gk = float(tk.grad)
    gb = to_host(tb.grad)
    h = 1e-5
    rng = np.random.default_rng(3)
    for _ in range(2):
        E = rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape)
        fd = (_loss_gpu(lat, U + h * E, kappa, b, eta, opts) - _loss_gpu(lat, U - h * E, kappa, b, eta, opts)) / (2 * h)
        an = float(np.vdot(gU, E).real)
        print(f"dU fd={fd:.10e} an={an:.10e}", flush=True)
        assert abs(fd - an) <= 1e-5 * abs(an)
    fd = (_loss_gpu(lat, U, kappa + h, b, eta, opts) - _loss_gpu(lat, U, kappa - h, b, eta, opts)) / (2 * h)
    print(f"dkappa fd={fd:.10e} an={gk:.10e}", flush=True)
    assert abs(fd - gk) <= 1e-5 * abs(gk)
    # grad_b = y = D^-dag eta (L is linear in b)
    import oracle
    orc = oracle.Oracle(dims, -1, kappa, 1.0, U)
    assert np.linalg.norm(eta - orc.D(gb, dagger=True)) / np.linalg.norm(eta) <= 1e-10


def test_backward_16x32_timed():
    """The differentiation workload (16^3x32, kappa 0.125): one forward and one
    backward through the library; the link gradient is compared to the
    oracle's formula evaluated on the GPU's own x and y."""
    import time
    import torch
    from paper_1612_06556_amd import autograd, wcl
    dims = (16, 16, 16, 32)
    lat, orc, U = setup(dims, -1, 0.125, 1.0, 1005, None)
    b = synth.gaussian_spinor(dims, 2005)
    eta = synth.gaussian_spinor(dims, 3005)
    tU = torch.from_numpy(U).cuda().requires_grad_(True)
    tk = torch.tensor(0.125, dtype=torch.float64, requires_grad=True)
    tb = torch.from_numpy(b).cuda().requires_grad_(True)
    t0 = time.perf_counter()
    x = autograd.solve(tU, tk, tb, lat, 1.0, tol=1e-10)
    L = torch.real(torch.vdot(torch.from_numpy(eta).cuda().reshape(-1), x.reshape(-1)))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    print(f"16^3x32 forward {1e3*(t1-t0):.1f} ms backward {1e3*(t2-t1):.1f} ms", flush=True)
    y = to_host(tb.grad)
    assert np.linalg.norm(eta - orc.D(y, dagger=True)) / np.linalg.norm(eta) <= 1e-10
    gU_o, gk_o = orc.grad(to_host(x.detach()), y)
    assert rel(to_host(tU.grad), gU_o) <= 1e-10
    assert abs(float(tk.grad) - gk_o) <= 1e-10 * abs(gk_o)
