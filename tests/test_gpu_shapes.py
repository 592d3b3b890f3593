"""Extreme grid shapes against the FP64 oracle: long thin grids along each axis (many
tiles along one axis, one partial tile along the others) and a wide 8192^2 plane stack
(the largest block counts along x and y)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.helpers import interior, rel_errors, rel_errors_chunked

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = 1e-5


@pytest.fixture(scope="module")
def mms():
    import paper_2507_11067_amd as m
    return m


CASES = [("star", 4, "fp32"), ("box", 2, "fp32"), ("box", 2, "bf16x3"), ("box", 4, "fp16x3s"),
         ("star2d", 4, "fp32"), ("box2d", 3, "fp32")]


def coeffs(shape, r, seed):
    rng = np.random.default_rng(seed)
    w = 2 * r + 1
    dims = {"star": (3, w), "box": (w, w, w), "star2d": (2, w), "box2d": (w, w)}[shape]
    return rng.uniform(-1, 1, dims).astype(np.float32)


ORACLE = {"star": oracle.star, "box": oracle.box, "star2d": oracle.star2d, "box2d": oracle.box2d}


@pytest.mark.parametrize("dims", [(4100, 3, 5), (3, 2100, 5), (5, 3, 3000)],
                         ids=lambda d: "x".join(map(str, d)))
@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}{c[1]}_{c[2]}")
def test_long_thin_grids(mms, dims, case):
    shape, r, prec = case
    nx, ny, nz = dims
    grid = mms.Grid(nx, ny, nz)
    x = synth.uniform_grid(700, nx, ny, nz, sy=grid.sy)
    c = coeffs(shape, r, 701)
    out = torch.full(grid.shape, 3.0, device=DEV)
    mms.stencil_apply(torch.from_numpy(x).to(DEV), out, grid, shape, r, c, precision=prec)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = ORACLE[shape](x, nx, ny, nz, r, c)
    rmax, _ = rel_errors(interior(got, grid), interior(ref, grid))
    assert rmax <= TOL, rmax
    o = got.copy()
    o[4:4 + nz, 4:4 + ny, 4:4 + nx] = 0
    assert np.all((o == 3.0) | (o == 0)) and np.count_nonzero(o == 0) == nz * ny * nx


def test_wide_plane_stack_full_grid(mms):
    """8192 x 8192 x 2: 32 x 512 tiles per plane for the star, 1024 blocks per plane for
    the 2-D kernels; every output against the full-grid oracle sweep."""
    nx = ny = 8192
    nz = 2
    grid = mms.Grid(nx, ny, nz)
    x = synth.uniform_grid(702, nx, ny, nz, sy=grid.sy)
    x64 = x.astype(np.float64)
    xt = torch.from_numpy(x).to(DEV)
    out = grid.zeros(DEV)
    for shape, r in (("star", 4), ("star2d", 4), ("box2d", 3)):
        c = coeffs(shape, r, 704)
        mms.stencil_apply(xt, out, grid, shape, r, c)
        torch.cuda.synchronize()
        o = out.cpu().numpy()
        ref = ORACLE[shape](x64, nx, ny, nz, r, c)
        rmax, _ = rel_errors_chunked(interior(o, grid), interior(ref, grid), chunk=1)
        del ref
        assert rmax <= TOL, (shape, rmax)
