"""GPU parity of the fused pseudo-acoustic VTI step against the FP64 oracle.

Gates as for the acoustic step: one step from identical FP32 inputs, normwise
max error <= 1e-5; a multi-step run is gated at 1e-3 (numbers are printed).
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
FACES = synth.SPONGE_LATERAL_AND_BOTTOM


@pytest.fixture(scope="module")
def mms():
    import paper_2507_11067_amd as m
    return m


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def smooth(seed, grid):
    return synth.smooth_random_grid(seed, grid.nx, grid.ny, grid.nz)


def medium(mms, nx, ny, nz, seed, nt):
    """Layered C2 (Courant 0.4), Thomsen fields, a scaled Ricker source near the top."""
    grid = mms.Grid(nx, ny, nz)
    v = synth.layered_velocity(nx, seed, nz=nz, ny=ny, sigma=2.0)
    dt = 0.4 * 10.0 / v.max() / np.sqrt(1.5)
    c2 = synth.padded_zeros(nx, ny, nz, sy=grid.sy)
    synth.interior(c2, nx, ny, nz)[...] = ((v * dt / 10.0) ** 2).astype(np.float32)
    eps, delta = synth.thomsen_fields(nx, ny, nz, seed + 1, sy=grid.sy)
    a = (1 + 2 * eps).astype(np.float32)
    b = np.sqrt(1 + 2 * delta).astype(np.float32)
    f = (dt * dt * synth.ricker(nt, dt, 15.0) * 1e4).astype(np.float32)
    src = (min(2, nz - 1), ny // 2, nx // 2)
    return grid, c2, a, b, f, src


@pytest.mark.parametrize("dims", [(20, 20, 20), (37, 19, 11), (300, 10, 21)],
                         ids=lambda d: "x".join(map(str, d)))
def test_vti_step_parity(mms, dims):
    nx, ny, nz = dims
    nt, n = 8, 3
    grid, c2, a, b, f, src = medium(mms, nx, ny, nz, 30, nt)
    hp, hc, vp, vc = (smooth(31 + k, grid) for k in range(4))
    traces = torch.zeros((nt, ny, nx), device=DEV)
    w = mms.Wave(grid, T(c2), LAP, nt, 1.0, 4, 0.1, FACES, src, T(f), traces)
    hn, vn = grid.zeros(DEV), grid.zeros(DEV)
    w.vti_step(n, T(a), T(b), T(hp), T(hc), hn, T(vp), T(vc), vn)
    # in place: next = prev for both fields gives the same bits
    hpt, vpt = T(hp), T(vp)
    w2 = mms.Wave(grid, T(c2), LAP, nt, 1.0, 4, 0.1, FACES, src, T(f))
    w2.vti_step(n, T(a), T(b), hpt, T(hc), hpt, vpt, T(vc), vpt)
    torch.cuda.synchronize()
    ow = oracle.Wave(nx, ny, nz, c2, LAP, src, f, nt, 4, 0.1, FACES)
    rh, rv, tr = ow.vti_step(n, a, b, hp, hc, vp, vc)
    for got, ref in ((hn, rh), (vn, rv)):
        g = got.cpu().numpy()
        rmax, rrms = rel_errors(interior(g, grid), interior(ref, grid))
        assert rmax <= 1e-5, (rmax, rrms)
        # the halo stays zero
        assert np.count_nonzero(g) == np.count_nonzero(interior(g, grid))
    assert torch.equal(hpt, hn) and torch.equal(vpt, vn)
    np.testing.assert_array_equal(traces[n].cpu().numpy(), tr.astype(np.float32))
    assert torch.count_nonzero(traces[:n]) == 0 and torch.count_nonzero(traces[n + 1:]) == 0


def test_vti_step_reads_halo_as_stored(mms):
    """Halo cells of H^n (x and y neighbours) and V^n (z neighbours) enter the step as stored:
    random values in the whole padded arrays of both fields at both levels; the outputs'
    halos are never written."""
    nx, ny, nz = 37, 19, 11
    nt, n = 8, 3
    grid, c2, a, b, f, src = medium(mms, nx, ny, nz, 30, nt)
    rng = np.random.default_rng(33)
    hp, hc, vp, vc = (rng.uniform(-1, 1, grid.shape).astype(np.float32) for _ in range(4))
    w = mms.Wave(grid, T(c2), LAP, nt, 1.0, 4, 0.1, FACES, src, T(f))
    hn, vn = grid.zeros(DEV).fill_(7.0), grid.zeros(DEV).fill_(7.0)
    w.vti_step(n, T(a), T(b), T(hp), T(hc), hn, T(vp), T(vc), vn)
    torch.cuda.synchronize()
    rh, rv, _ = oracle.Wave(nx, ny, nz, c2, LAP, src, f, nt, 4, 0.1, FACES).vti_step(
        n, a, b, hp, hc, vp, vc)
    for got, ref in ((hn, rh), (vn, rv)):
        g = got.cpu().numpy()
        rmax, rrms = rel_errors(interior(g, grid), interior(ref, grid))
        assert rmax <= 1e-5, (rmax, rrms)
        interior(g, grid)[...] = 7.0
        assert np.all(g == 7.0)


@pytest.mark.parametrize("radius", [1, 2, 3])
def test_vti_step_parity_short_radius(mms, radius):
    nx, ny, nz = 45, 13, 17
    nt, n = 4, 2
    grid, c2, a, b, f, src = medium(mms, nx, ny, nz, 40 + radius, nt)
    rng = np.random.default_rng(radius)
    lap = [float(v) for v in rng.uniform(-1, 1, radius + 1).astype(np.float32)]
    hp, hc, vp, vc = (smooth(44 + k, grid) for k in range(4))
    w = mms.Wave(grid, T(c2), lap, nt, 1.0, 0, 0.0, 0, src, T(f))
    hn, vn = grid.zeros(DEV), grid.zeros(DEV)
    w.vti_step(n, T(a), T(b), T(hp), T(hc), hn, T(vp), T(vc), vn)
    torch.cuda.synchronize()
    ow = oracle.Wave(nx, ny, nz, c2, lap, src, f, nt)
    rh, rv, _ = ow.vti_step(n, a, b, hp, hc, vp, vc)
    for got, ref in ((hn, rh), (vn, rv)):
        rmax, rrms = rel_errors(interior(got.cpu().numpy(), grid), interior(ref, grid))
        assert rmax <= 1e-5, (radius, rmax, rrms)


def test_vti_isotropic_equals_acoustic_kernel(mms):
    """a = b = 1 and H = V: both VTI outputs are the acoustic step of the wave kernel."""
    nx, ny, nz = 70, 33, 29
    nt, n = 6, 4
    grid, c2, _, _, f, src = medium(mms, nx, ny, nz, 50, nt)
    one = T(np.ones(grid.shape, np.float32))
    up, uc = T(smooth(51, grid)), T(smooth(52, grid))
    w = mms.Wave(grid, T(c2), LAP, nt, 1.0, 4, 0.1, FACES, src, T(f))
    hn, vn, un = grid.zeros(DEV), grid.zeros(DEV), grid.zeros(DEV)
    w.vti_step(n, one, one, up, uc, hn, up, uc, vn)
    w.step(n, up, uc, un)
    torch.cuda.synchronize()
    for got in (hn, vn):
        rmax, _ = rel_errors(interior(got.cpu().numpy(), grid), interior(un.cpu().numpy(), grid))
        assert rmax <= 1e-6, rmax


def test_vti_forward_run_vs_oracle(mms):
    """40^3, 200 steps from rest with the Ricker source: H traces and final fields vs FP64."""
    n, nt = 40, 200
    grid, c2, a, b, f, src = medium(mms, n, n, n, 60, nt)
    traces = torch.zeros((nt, n, n), device=DEV)
    w = mms.Wave(grid, T(c2), LAP, nt, 1.0, 8, 0.015, FACES, src, T(f), traces)
    H = [grid.zeros(DEV) for _ in range(2)]
    V = [grid.zeros(DEV) for _ in range(2)]
    at, bt = T(a), T(b)
    w.record(0, H[0])
    for k in range(1, nt):
        # H^{k+1} overwrites H^{k-1}
        w.vti_step(k, at, bt, H[(k - 1) % 2], H[k % 2], H[(k + 1) % 2],
                   V[(k - 1) % 2], V[k % 2], V[(k + 1) % 2])
    torch.cuda.synchronize()
    ow = oracle.Wave(n, n, n, c2, LAP, src, f, nt, 8, 0.015, FACES)
    z = ow.zeros()
    res = ow.vti_forward(a, b, z, z, z, z)
    rmax, rrms = rel_errors(traces.cpu().numpy(), res["traces"])
    rH, _ = rel_errors(interior(H[nt % 2].cpu().numpy(), grid), interior(res["last"][1], grid))
    rV, _ = rel_errors(interior(V[nt % 2].cpu().numpy(), grid), interior(res["last"][3], grid))
    print(f"VTI 40^3 x {nt}: traces rel_max {rmax:.2e} rel_rms {rrms:.2e}; "
          f"H {rH:.2e} V {rV:.2e}")
    assert rmax <= 1e-3 and rH <= 1e-3 and rV <= 1e-3
    # anisotropy matters: the isotropic run differs
    ow_iso = oracle.Wave(n, n, n, c2, LAP, src, f, nt, 8, 0.015, FACES)
    ones = np.ones_like(z)
    iso = ow_iso.vti_forward(ones, ones, z, z, z, z)
    assert rel_errors(res["traces"], iso["traces"])[0] > 1e-2


def test_vti_rejects_bad_arguments(mms):
    grid, c2, a, b, f, src = medium(mms, 12, 10, 9, 70, 4)
    w = mms.Wave(grid, T(c2), LAP, 4, 1.0, 0, 0.0, 0, src, T(f))
    fs = [T(smooth(71 + k, grid)) for k in range(4)]
    out = [grid.zeros(DEV) for _ in range(2)]
    at, bt = T(a), T(b)
    with pytest.raises(mms.MmsError):
        w.vti_step(0, at, bt, fs[0], fs[1], out[0], fs[2], fs[3], out[1])
    with pytest.raises(mms.MmsError):
        w.vti_step(4, at, bt, fs[0], fs[1], out[0], fs[2], fs[3], out[1])
    with pytest.raises(mms.MmsError):     # output aliases the current level
        w.vti_step(1, at, bt, fs[0], fs[1], fs[1], fs[2], fs[3], out[1])
    with pytest.raises(mms.MmsError):     # both outputs in one buffer
        w.vti_step(1, at, bt, fs[0], fs[1], out[0], fs[2], fs[3], out[0])
    with pytest.raises(mms.MmsError):     # V output aliases H^{n-1}
        w.vti_step(1, at, bt, fs[0], fs[1], out[0], fs[2], fs[3], fs[0])
