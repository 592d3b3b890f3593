"""GPU parity of the wave, adjoint, VTI and TTI steps on degenerate grids: fewer cells
than the radius-4 stencil along one or more axes (one cell, one row, one or two planes),
so that nearly every stencil tap reads the halo and every tile is mostly lanes that only
help with loads.  Gate as for the other steps: one step from identical FP32 inputs,
normwise max error <= 1e-5 against the FP64 oracle; the output halo stays unwritten.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.helpers import interior, rel_errors

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
LAP = [float(v) for v in synth.LAPLACIAN_R4]
D1 = [float(v) for v in synth.FIRST_DERIV_R4]
FACES = synth.SPONGE_LATERAL_AND_BOTTOM
W = 2
DIMS = [(1, 1, 1), (3, 2, 1), (5, 1, 9), (2, 7, 3), (6, 3, 2)]


@pytest.fixture(scope="module")
def mms():
    import paper_2507_11067_amd as m
    return m


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def problem(mms, dims, seed, nt):
    nx, ny, nz = dims
    grid = mms.Grid(nx, ny, nz)
    v = synth.layered_velocity(nx, seed, nz=nz, ny=ny, sigma=2.0)
    eps, delta = synth.thomsen_fields(nx, ny, nz, seed + 1, sy=grid.sy)
    theta, phi = synth.tilt_fields(nx, ny, nz, seed + 2, sy=grid.sy)
    dt = 0.4 * 10.0 / v.max() / np.sqrt(1 + 2 * float(eps.max()))
    c2 = synth.padded_zeros(nx, ny, nz, sy=grid.sy)
    synth.interior(c2, nx, ny, nz)[...] = ((v * dt / 10.0) ** 2).astype(np.float32)
    f = (dt * dt * synth.ricker(nt, dt, 15.0) * 1e4).astype(np.float32)
    src = (min(2, nz - 1), ny // 2, nx // 2)
    fields = [synth.smooth_random_grid(seed + 3 + k, nx, ny, nz) for k in range(4)]
    ow = oracle.Wave(nx, ny, nz, c2, LAP, src, f, nt, W, 0.1, FACES)
    return grid, c2, f, src, (eps, delta, theta, phi), fields, ow


def check(got, ref, grid, what):
    g = got.cpu().numpy()
    rmax, rrms = rel_errors(interior(g, grid), interior(ref, grid))
    print(f"{what}: rel_max {rmax:.2e} rel_rms {rrms:.2e}")
    assert rmax <= 1e-5, (what, rmax, rrms)
    assert np.count_nonzero(g) == np.count_nonzero(interior(g, grid)), what


@pytest.mark.parametrize("dims", DIMS, ids=lambda d: "x".join(map(str, d)))
def test_wave_and_adjoint_steps_degenerate(mms, dims):
    nt, n = 6, 2
    grid, c2, f, src, _, (up, uc, l2, l1), ow = problem(mms, dims, 200, nt)
    traces = torch.zeros((nt, grid.ny, grid.nx), device=DEV)
    w = mms.Wave(grid, T(c2), LAP, nt, 1.0, W, 0.1, FACES, src, T(f), traces)
    un = grid.zeros(DEV)
    w.step(n, T(up), T(uc), un)
    resid = np.random.default_rng(201).standard_normal((nt, grid.ny, grid.nx)).astype(np.float32)
    grad = torch.full(dims[::-1], 0.25, dtype=torch.float64, device=DEV)
    l0 = grid.zeros(DEV)
    w.adjoint_step(n, T(l2), T(l1), l0, resid=T(resid), u_n=T(uc), grad=grad)
    torch.cuda.synchronize()
    ref, tr = ow.step(n, up, uc)
    check(un, ref, grid, f"step {dims}")
    np.testing.assert_array_equal(traces[n].cpu().numpy(), tr.astype(np.float32))
    g = ow.zeros()
    synth.interior(g, *dims)[...] = 0.25
    lref = ow.adjoint_step(n, l2, l1, resid[n], uc, g)
    check(l0, lref, grid, f"adjoint step {dims}")
    rg, _ = rel_errors(grad.cpu().numpy() - 0.25, interior(g, grid) - 0.25)
    assert rg <= 1e-5, rg


@pytest.mark.parametrize("dims", DIMS, ids=lambda d: "x".join(map(str, d)))
def test_vti_and_tti_steps_degenerate(mms, dims):
    nt, n = 6, 2
    grid, c2, f, src, (eps, delta, theta, phi), (hp, hc, vp, vc), ow = problem(mms, dims, 210, nt)
    w = mms.Wave(grid, T(c2), LAP, nt, 1.0, W, 0.1, FACES, src, T(f))
    a = (1 + 2 * eps).astype(np.float32)
    b = np.sqrt(1 + 2 * delta).astype(np.float32)
    hn, vn = grid.zeros(DEV), grid.zeros(DEV)
    w.vti_step(n, T(a), T(b), T(hp), T(hc), hn, T(vp), T(vc), vn)
    t = mms.Tti(grid, T(eps), T(delta), T(theta), T(phi), 0.1, 1.0, D1)
    pn, qn = grid.zeros(DEV), grid.zeros(DEV)
    w.tti_step(n, t, T(hp), T(hc), pn, T(vp), T(vc), qn)
    torch.cuda.synchronize()
    rh, rv, _ = ow.vti_step(n, a, b, hp, hc, vp, vc)
    check(hn, rh, grid, f"VTI H {dims}")
    check(vn, rv, grid, f"VTI V {dims}")
    rp, rq, _ = ow.tti_step(ow.tti(eps, delta, theta, phi, 0.1, 1.0, D1), n, hp, hc, vp, vc)
    check(pn, rp, grid, f"TTI p {dims}")
    check(qn, rq, grid, f"TTI q {dims}")
