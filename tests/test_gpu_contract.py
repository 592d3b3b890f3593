"""GPU checks of the boundary's own promises (include/mmstencil.h), called through the C ABI:
reductions on different streams with their own workspaces do not disturb each other, the
result pair counts NaN and Inf terms, and the chain-rule scaling reads its FP64 factor on
the device."""
import ctypes

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def mms():
    import paper_2507_11067_amd as m
    return m


def vp(t):
    return ctypes.c_void_p(t.data_ptr())


def test_reductions_on_two_streams_concurrently(mms):
    """A flat dot product and a grid dot product enqueued on two streams with no
    synchronisation between them, three times over: each matches its FP64 sum (the
    partial sums live in the caller's workspaces, not in shared library state)."""
    from paper_2507_11067_amd import _lib
    L = _lib.lib()
    n = 1 << 26
    rng = np.random.default_rng(90)
    x = rng.uniform(-1, 1, n).astype(np.float32)
    y = rng.uniform(-1, 1, n).astype(np.float32)
    ref_flat = float(np.dot(x.astype(np.float64), y.astype(np.float64)))
    grid = mms.Grid(256, 250, 240)
    a = synth.uniform_grid(91, grid.nx, grid.ny, grid.nz, sy=grid.sy)
    b = synth.uniform_grid(92, grid.nx, grid.ny, grid.nz, sy=grid.sy)
    I = lambda t: synth.interior(t, grid.nx, grid.ny, grid.nz).astype(np.float64)
    ref_grid = float(np.sum(I(a) * I(b)))
    dx, dy = torch.from_numpy(x).to(DEV), torch.from_numpy(y).to(DEV)
    da, db = torch.from_numpy(a).to(DEV), torch.from_numpy(b).to(DEV)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    outs = [torch.full((3, 2), -1.0, dtype=torch.float64, device=DEV) for _ in range(2)]
    works = [torch.empty(_lib.MMS_REDUCE_WORK, dtype=torch.float64, device=DEV) for _ in range(2)]
    g = grid.c()
    torch.cuda.synchronize()
    for rep in range(3):
        assert L.mms_flat_dot_f64(vp(dx), vp(dy), n, vp(outs[0][rep]), vp(works[0]),
                                  ctypes.c_void_p(s1.cuda_stream)) == 0
        assert L.mms_dot_f64(vp(da), vp(db), ctypes.byref(g), vp(outs[1][rep]), vp(works[1]),
                             ctypes.c_void_p(s2.cuda_stream)) == 0
    torch.cuda.synchronize()
    f, gr = outs[0].cpu().numpy(), outs[1].cpu().numpy()
    print(f"flat {f[:, 0]} vs {ref_flat}; grid {gr[:, 0]} vs {ref_grid}")
    assert np.all(f[:, 1] == 0) and np.all(gr[:, 1] == 0)
    assert np.all(f[:, 0] == f[0, 0]) and np.all(gr[:, 0] == gr[0, 0])   # bit-reproducible
    assert abs(f[0, 0] - ref_flat) <= 1e-12 * np.sum(np.abs(x.astype(np.float64) * y))
    assert abs(gr[0, 0] - ref_grid) <= 1e-12 * np.sum(np.abs(I(a) * I(b)))


def test_reductions_count_nonfinite_terms(mms):
    """NaN and Inf inputs are counted in the result pair and make the binding raise
    MMS_EUNSTABLE; halo cells are not read, so a NaN there changes nothing."""
    x = np.random.default_rng(93).standard_normal(100003).astype(np.float32)
    x[[5, 777, 100002]] = np.nan
    x[[12, 13]] = np.inf
    t = torch.from_numpy(x).to(DEV)
    out = torch.zeros(2, dtype=torch.float64, device=DEV)
    with pytest.raises(mms.MmsError) as e:
        mms.flat_dot(t, None, out=out)
    assert e.value.code == -5
    assert out[1].item() >= 5
    ok = torch.from_numpy(np.nan_to_num(x, nan=0.0, posinf=0.0)).to(DEV)
    assert mms.flat_dot(ok) == pytest.approx(float(np.sum(np.nan_to_num(x, nan=0.0, posinf=0.0)
                                                           .astype(np.float64) ** 2)), rel=1e-12)
    # misfit: a pair with a count, no exception until it is checked
    r = torch.empty_like(t)
    pair = mms.flat_misfit(t, torch.zeros_like(t), resid=r)
    assert pair[1].item() >= 5
    with pytest.raises(mms.MmsError):
        mms.check_result(pair)
    # grid dot: NaN in the halo is never read; NaN in the interior is counted
    grid = mms.Grid(21, 13, 9)
    a = synth.uniform_grid(94, grid.nx, grid.ny, grid.nz, sy=grid.sy)
    a[0, 0, 0] = np.nan
    a[-1, -1, -1] = np.inf
    ta = torch.from_numpy(a).to(DEV)
    I = lambda u: synth.interior(u, grid.nx, grid.ny, grid.nz).astype(np.float64)
    assert mms.dot(ta, None, grid) == pytest.approx(float(np.sum(I(a) ** 2)), rel=1e-12)
    a[4 + 3, 4 + 2, 4 + 1] = np.nan
    with pytest.raises(mms.MmsError):
        mms.dot(torch.from_numpy(a).to(DEV), None, grid)
    # energy of a field holding a NaN
    n = 16
    g3 = mms.Grid(n, n, n)
    c2 = synth.padded_zeros(n, n, n)
    synth.interior(c2, n, n, n)[...] = 0.1
    w = mms.Wave(g3, torch.from_numpy(c2).to(DEV), [float(v) for v in synth.LAPLACIAN_R4], 4)
    u = synth.smooth_random_grid(95, n, n, n)
    e_ok = w.energy(torch.from_numpy(u).to(DEV), torch.from_numpy(u).to(DEV))
    assert np.isfinite(e_ok)
    u[4 + 5, 4 + 5, 4 + 5] = np.nan
    with pytest.raises(mms.MmsError) as e:
        w.energy(torch.from_numpy(u).to(DEV), torch.from_numpy(u).to(DEV))
    assert e.value.code == -5


def test_flat_scale_reads_factor_on_device(mms):
    """out = (float)(scale * in) with scale an FP64 device value, in place or not."""
    x = np.random.default_rng(96).standard_normal(70001).astype(np.float32)
    s = torch.tensor([0.3700000000000001], dtype=torch.float64, device=DEV)
    t = torch.from_numpy(x).to(DEV)
    out = torch.empty_like(t)
    mms.flat_scale(t, s, out)
    want = (0.3700000000000001 * x.astype(np.float64)).astype(np.float32)
    np.testing.assert_array_equal(out.cpu().numpy(), want)
    mms.flat_scale(t, s, t)
    np.testing.assert_array_equal(t.cpu().numpy(), want)
    empty = torch.empty(0, device=DEV)
    mms.flat_scale(empty, s, empty)
