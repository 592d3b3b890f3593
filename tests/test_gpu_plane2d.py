"""GPU parity of the 2-D star and box sweeps (Table I 2DStar / 2DBox, applied to
every plane of a stack) against the FP64 oracle.

Gate (normwise, one sweep from identical FP32 inputs): max|y - y*| / max|y*| <= 1e-5.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.helpers import halo_is_zero, interior, rel_errors, rel_errors_chunked

pytestmark = pytest.mark.gpu
TOL = 1e-5
DEV = "cuda:0"


@pytest.fixture(scope="module")
def mms():
    import paper_2507_11067_amd as m
    return m


def run(mms, x_np, grid, shape, r, c, out_fill=0.0):
    # grid.zeros() places the arrays (interior rows on 128-byte boundaries for Grid.aligned)
    x = grid.zeros(DEV)
    x.copy_(torch.from_numpy(x_np))
    out = grid.zeros(DEV).fill_(out_fill)
    mms.stencil_apply(x, out, grid, shape, r, c)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def coeffs(shape, seed, r):
    rng = np.random.default_rng(seed)
    w = 2 * r + 1
    return rng.uniform(-1, 1, (2, w) if shape == "star2d" else (w, w)).astype(np.float32)


ORACLE = {"star2d": oracle.star2d, "box2d": oracle.box2d}
SIZES = [(17, 19, 5), (133, 37, 3), (300, 20, 2), (1, 1, 1), (5, 3, 2), (64, 64, 9),
         (260, 9, 140)]


@pytest.mark.parametrize("shape", ["star2d", "box2d"])
@pytest.mark.parametrize("r", [1, 2, 3, 4])
@pytest.mark.parametrize("size", SIZES, ids=lambda s: "x".join(map(str, s)))
def test_plane2d_parity(mms, shape, r, size):
    nx, ny, nz = size
    grid = mms.Grid(nx, ny, nz)
    x = synth.uniform_grid(500 + r, nx, ny, nz, sy=grid.sy)
    c = coeffs(shape, 600 + r, r)
    got = run(mms, x, grid, shape, r, c, out_fill=7.0)
    ref = ORACLE[shape](x, nx, ny, nz, r, c)
    rmax, _ = rel_errors(interior(got, grid), interior(ref, grid))
    assert rmax <= TOL, rmax
    o = got.copy()
    H = grid.halo
    o[H:H + nz, H:H + ny, H:H + nx] = 0
    assert np.all((o == 7.0) | (o == 0)) and np.count_nonzero(o == 0) == nz * ny * nx


@pytest.mark.parametrize("shape", ["star2d", "box2d"])
def test_plane2d_nonzero_halo_and_wide_pitch(mms, shape):
    """Halo cells are read as stored (z-halo planes never); H = 8, wide pitch."""
    nx, ny, nz, H = 30, 21, 6, 8
    grid = mms.Grid(nx, ny, nz, halo=H, sy=64)
    x = np.random.default_rng(7).uniform(-1, 1, grid.shape).astype(np.float32)
    c = coeffs(shape, 8, 4)
    got = run(mms, x, grid, shape, 4, c)
    ref = ORACLE[shape](x, nx, ny, nz, 4, c, halo=H)
    rmax, _ = rel_errors(interior(got, grid), interior(ref, grid))
    assert rmax <= TOL


def test_plane2d_empty_and_deterministic(mms):
    grid = mms.Grid(40, 30, 0)
    x = grid.zeros(DEV)
    out = grid.zeros(DEV)
    mms.stencil_apply(x, out, grid, "box2d", 3, coeffs("box2d", 1, 3))
    g2 = mms.Grid(70, 50, 12)
    xt = torch.from_numpy(synth.uniform_grid(9, 70, 50, 12, sy=g2.sy)).to(DEV)
    a, b = g2.zeros(DEV), g2.zeros(DEV)
    c = coeffs("box2d", 2, 3)
    mms.stencil_apply(xt, a, g2, "box2d", 3, c)
    mms.stencil_apply(xt, b, g2, "box2d", 3, c)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.fixture(scope="module")
def big512():
    n = 512
    # the benchmark's layout: rows padded to 544, interior rows on 128-byte boundaries
    x = synth.uniform_grid(2, n, n, n, sy=((n + 8 + 31) // 32) * 32)
    return n, x, x.astype(np.float64)


TABLE1_2D = [("star2d", 2), ("star2d", 4), ("box2d", 2), ("box2d", 3)]


@pytest.mark.parametrize("shape,r", TABLE1_2D, ids=lambda v: str(v))
def test_table1_2d_512_full_grid(mms, big512, shape, r):
    """Table I 2-D kernels on the 512^3 stack in the benchmark's launch shape: every output
    against the full-grid FP64 oracle sweep."""
    n, x, x64 = big512
    grid = mms.Grid.aligned(n, n, n)
    c = synth.star2d_coeffs_laplacian(r) if shape == "star2d" else synth.box2d_coeffs(10 + r, r)
    got = run(mms, x, grid, shape, r, c)
    f = oracle.star2d if shape == "star2d" else oracle.box2d
    ref = f(x64, n, n, n, r, c)
    rmax, rrms = rel_errors_chunked(interior(got, grid), interior(ref, grid))
    del ref
    print(f"{shape} r{r} 512^3 full grid: rel_max {rmax:.2e} rel_rms {rrms:.2e}")
    assert rmax <= TOL, rmax
    assert halo_is_zero(got, grid)
