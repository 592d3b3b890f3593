"""Parity at the workloads' full sizes, in the launch configuration bench.py times:
one acoustic step at 400^3 (with receivers and the FP64 image), the first 40
RTM steps at 400^3 from rest, one adjoint step with gradient at 256^3, one VTI
step at 400^3 -- every output point against the FP64 oracle -- and one TTI step
at 400^3 on its top planes.

Gates: one step from identical FP32 inputs, normwise max error <= 1e-5; the
40-step run accumulates rounding and is gated at 1e-4 (numbers are printed).
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


@pytest.fixture(scope="module")
def mms():
    import paper_2507_11067_amd as m
    return m


@pytest.fixture(scope="module")
def rtm400():
    return synth.wave_setup(400, 64, seed=7, sponge_width=32)


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def uniform(seed, n):
    return synth.uniform_grid(seed, n, n, n)


def test_wave_step_400(mms, rtm400):
    s = rtm400
    n, nt, k = 400, s.nt, 7
    grid = mms.Grid(n, n, n)
    up, uc = uniform(91, n), uniform(92, n)
    traces = torch.zeros((nt, n, n), device=DEV)
    image = torch.full((n, n, n), 0.5, dtype=torch.float64, device=DEV)
    w = mms.Wave(grid, T(s.c2), LAP, nt, 1.0, s.sponge_width, s.sponge_alpha, s.sponge_faces,
                 s.src, T(s.src_dt2f), traces, image)
    un = grid.zeros(DEV)
    w.step(k, T(up), T(uc), un)
    torch.cuda.synchronize()
    ow = oracle.Wave.from_setup(s, LAP)
    img = ow.zeros()
    synth.interior(img, n, n, n)[...] = 0.5
    ref, tr = ow.step(k, up, uc, image=img)
    rmax, rrms = rel_errors(interior(un.cpu().numpy(), grid), interior(ref, grid))
    print(f"wave step 400^3: rel_max {rmax:.2e} rel_rms {rrms:.2e}")
    assert rmax <= 1e-5, (rmax, rrms)
    np.testing.assert_array_equal(traces[k].cpu().numpy(), tr.astype(np.float32))
    ri, _ = rel_errors(image.cpu().numpy() - 0.5, interior(img, grid) - 0.5)
    assert ri <= 1e-5, ri


def test_rtm_first_40_steps_400(mms, rtm400):
    s = rtm400
    n, nt = 400, 41
    grid = mms.Grid(n, n, n)
    traces = torch.zeros((nt, n, n), device=DEV)
    image = torch.zeros((n, n, n), dtype=torch.float64, device=DEV)
    f = s.src_dt2f[:nt]
    w = mms.Wave(grid, T(s.c2), LAP, nt, 1.0, s.sponge_width, s.sponge_alpha, s.sponge_faces,
                 s.src, T(f), traces, image)
    bufs = [grid.zeros(DEV) for _ in range(3)]
    w.record(0, bufs[0])
    w.forward(1, nt, [bufs[i % 3] for i in range(nt + 1)])
    torch.cuda.synchronize()
    ow = oracle.Wave(n, n, n, s.c2, LAP, s.src, f, nt, s.sponge_width, s.sponge_alpha,
                     s.sponge_faces)
    z = ow.zeros()
    res = ow.forward(z, z, image=True)
    ru, rrms = rel_errors(interior(bufs[nt % 3].cpu().numpy(), grid), interior(res["last"][1], grid))
    ri, _ = rel_errors(image.cpu().numpy(), interior(res["image"], grid))
    rt, _ = rel_errors(traces.cpu().numpy(), res["traces"])
    print(f"RTM 400^3 x {nt - 1} steps: u rel_max {ru:.2e} rel_rms {rrms:.2e}; image {ri:.2e}; "
          f"traces {rt:.2e}")
    assert ru <= 1e-4 and ri <= 1e-4 and rt <= 1e-4
    assert np.abs(res["traces"]).max() > 0      # the wave has reached the receivers


def test_adjoint_step_256(mms):
    s = synth.wave_setup(256, 16, seed=8, sponge_width=32)
    n, nt, k = 256, s.nt, 9
    grid = mms.Grid(n, n, n)
    l2, l1, un = uniform(93, n), uniform(94, n), uniform(95, n)
    resid = np.random.default_rng(96).uniform(-1, 1, (nt, n, n)).astype(np.float32)
    w = mms.Wave(grid, T(s.c2), LAP, nt, 1.0, s.sponge_width, s.sponge_alpha, s.sponge_faces,
                 s.src, T(s.src_dt2f))
    grad = torch.full((n, n, n), 0.25, dtype=torch.float64, device=DEV)
    l0 = grid.zeros(DEV)
    w.adjoint_step(k, T(l2), T(l1), l0, resid=T(resid), u_n=T(un), grad=grad)
    torch.cuda.synchronize()
    ow = oracle.Wave.from_setup(s, LAP)
    g = ow.zeros()
    synth.interior(g, n, n, n)[...] = 0.25
    ref = ow.adjoint_step(k, l2, l1, resid[k], un, g)
    rmax, rrms = rel_errors(interior(l0.cpu().numpy(), grid), interior(ref, grid))
    rg, _ = rel_errors(grad.cpu().numpy() - 0.25, interior(g, grid) - 0.25)
    print(f"adjoint step 256^3: lam rel_max {rmax:.2e} rel_rms {rrms:.2e}; grad {rg:.2e}")
    assert rmax <= 1e-5 and rg <= 1e-5, (rmax, rg)


def test_adjoint_step_mu_256(mms):
    """The same adjoint step carried in mu = C2 G lam (the form the gradient workload runs):
    lam^{n+1}, lam^{n+2} converted in, one mu-form step with the gradient in blocks of 8 (as
    the autograd driver runs it), lam^n converted back; every point against the oracle."""
    s = synth.wave_setup(256, 16, seed=8, sponge_width=32)
    n, nt, k = 256, s.nt, 9
    grid = mms.Grid(n, n, n)
    l2, l1, un = uniform(93, n), uniform(94, n), uniform(95, n)
    resid = np.random.default_rng(96).uniform(-1, 1, (nt, n, n)).astype(np.float32)
    w = mms.Wave(grid, T(s.c2), LAP, nt, 1.0, s.sponge_width, s.sponge_alpha, s.sponge_faces,
                 s.src, T(s.src_dt2f))
    # the block in progress started at a step whose partial held zero (phase 0 writes it)
    w.set_accumulation(torch.zeros((n, n, n), device=DEV), 8)
    grad = torch.full((n, n, n), 0.25, dtype=torch.float64, device=DEV)
    mu = [grid.zeros(DEV) for _ in range(3)]
    w.scale_mu(T(l1), mu[1], +1)
    w.scale_mu(T(l2), mu[2], +1)
    # nt - 1 - k = 6: the step in phase 6 of its block; a second call closes the block
    w.adjoint_mu(k, k, mu, us=[T(un)], resid=T(resid), grad=grad)
    torch.cuda.synchronize()
    part_only = grad.clone()
    z = [grid.zeros(DEV) for _ in range(3)]
    w.adjoint_mu(k - 1, k - 1, [z[0], mu[0], z[1]], us=[grid.zeros(DEV)], grad=grad)
    l0 = grid.zeros(DEV)
    w.scale_mu(mu[0], l0, -1)
    torch.cuda.synchronize()
    ow = oracle.Wave.from_setup(s, LAP)
    g = ow.zeros()
    synth.interior(g, n, n, n)[...] = 0.25
    ref = ow.adjoint_step(k, l2, l1, resid[k], un, g)
    rmax, rrms = rel_errors(interior(l0.cpu().numpy(), grid), interior(ref, grid))
    rg, _ = rel_errors(grad.cpu().numpy() - 0.25, interior(g, grid) - 0.25)
    print(f"adjoint step 256^3 (mu form): lam rel_max {rmax:.2e} rel_rms {rrms:.2e}; grad {rg:.2e}")
    # inside a block the FP64 gradient is untouched (the term waits in the FP32 partial)
    assert np.abs(part_only.cpu().numpy() - 0.25).max() <= 1e-15
    assert rmax <= 1e-5 and rg <= 1e-5, (rmax, rg)


def test_vti_step_400(mms, rtm400):
    s = rtm400
    n, nt, k = 400, s.nt, 6
    grid = mms.Grid(n, n, n)
    eps, delta = synth.thomsen_fields(n, n, n, 10, sy=grid.sy)
    a = (1 + 2 * eps).astype(np.float32)
    b = np.sqrt(1 + 2 * delta).astype(np.float32)
    shrink = 1.0 / (1.0 + 2.0 * float(eps.max()))
    hp, hc, vp, vc = (uniform(97 + i, n) for i in range(4))
    traces = torch.zeros((nt, n, n), device=DEV)
    w = mms.Wave(grid, T(s.c2), LAP, nt, shrink, s.sponge_width, s.sponge_alpha, s.sponge_faces,
                 s.src, T(s.src_dt2f), traces)
    hn, vn = grid.zeros(DEV), grid.zeros(DEV)
    w.vti_step(k, T(a), T(b), T(hp), T(hc), hn, T(vp), T(vc), vn)
    torch.cuda.synchronize()
    # the oracle takes C2 itself: the same FP32 product the kernel forms
    c2s = (np.float32(shrink) * s.c2).astype(np.float32)
    ow = oracle.Wave(n, n, n, c2s, LAP, s.src, s.src_dt2f, nt, s.sponge_width, s.sponge_alpha,
                     s.sponge_faces)
    rh, rv, tr = ow.vti_step(k, a, b, hp, hc, vp, vc)
    for name, got, ref in (("H", hn, rh), ("V", vn, rv)):
        rmax, rrms = rel_errors(interior(got.cpu().numpy(), grid), interior(ref, grid))
        print(f"VTI step 400^3 {name}: rel_max {rmax:.2e} rel_rms {rrms:.2e}")
        assert rmax <= 1e-5, (name, rmax, rrms)
    np.testing.assert_array_equal(traces[k].cpu().numpy(), tr.astype(np.float32))


def test_tti_step_400_top_slab(mms, rtm400):
    """One TTI step at 400^3 in the benchmark's configuration, checked on the top 24
    planes (receivers and source included) against the oracle run on the top 28
    planes: those outputs read only planes < 28, and the bottom sponge does not reach
    them (W = 32 from z = 399), so the slab sees the same operands."""
    s = rtm400
    n, nt, k, zs = 400, s.nt, 6, 28
    grid = mms.Grid(n, n, n)
    eps, delta = synth.thomsen_fields(n, n, n, 12, sy=grid.sy)
    theta, phi = synth.tilt_fields(n, n, n, 13, sy=grid.sy)
    shrink = 1.0 / (1.0 + 2.0 * float(eps.max()))
    d1 = [float(v) for v in synth.FIRST_DERIV_R4]
    fields = [uniform(101 + i, n) for i in range(4)]
    traces = torch.zeros((nt, n, n), device=DEV)
    w = mms.Wave(grid, T(s.c2), LAP, nt, shrink, s.sponge_width, s.sponge_alpha, s.sponge_faces,
                 s.src, T(s.src_dt2f), traces)
    t = mms.Tti(grid, T(eps), T(delta), T(theta), T(phi), 0.1, 1.0, d1)
    pn, qn = grid.zeros(DEV), grid.zeros(DEV)
    w.tti_step(k, t, *[T(a) for a in fields[:2]], pn, *[T(a) for a in fields[2:]], qn)
    torch.cuda.synchronize()
    top = lambda a: np.ascontiguousarray(a[:zs + 8])     # planes -4 .. zs+3 of the padded array
    c2s = (np.float32(shrink) * s.c2).astype(np.float32)
    ow = oracle.Wave(n, n, zs, top(c2s), LAP, s.src, s.src_dt2f, nt, s.sponge_width,
                     s.sponge_alpha, s.sponge_faces & ~32)      # no bottom face in the slab
    tt = ow.tti(top(eps), top(delta), top(theta), top(phi), 0.1, 1.0, d1)
    rp, rq, tr = ow.tti_step(tt, k, *[top(a) for a in fields])
    H = 4
    for name, got, ref in (("p", pn, rp), ("q", qn, rq)):
        g = got.cpu().numpy()[H:H + 24, H:H + n, H:H + n]
        r = ref[H:H + 24, H:H + n, H:H + n]
        rmax, rrms = rel_errors(g, r)
        print(f"TTI step 400^3 top planes {name}: rel_max {rmax:.2e} rel_rms {rrms:.2e}")
        assert rmax <= 1e-5, (name, rmax, rrms)
    np.testing.assert_array_equal(traces[k].cpu().numpy(), tr.astype(np.float32))
