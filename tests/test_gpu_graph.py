"""Sweeps captured in a HIP graph (as the config-0 benchmark times them) give on every replay
the bits of the same sweeps launched eagerly: the star on its small-grid kernel and on the
z-marching kernel, and the FP32 box.  Between replays the program does eager work of its
own (refilling the output with a sentinel) and synchronises; every replay is checked, and the
output halo keeps the sentinel (sweeps never write it)."""
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


@pytest.mark.parametrize("shape,r,dims", [("star", 4, (64, 64, 64)), ("star", 4, (133, 100, 80)),
                                          ("box", 2, (40, 33, 29))],
                         ids=["star-direct-64", "star-marching-133x100x80", "box2-40x33x29"])
def test_graph_replay_matches_eager(mms, shape, r, dims):
    nx, ny, nz = dims
    grid = mms.Grid(nx, ny, nz)
    x = torch.from_numpy(synth.uniform_grid(11, nx, ny, nz, sy=grid.sy)).to(DEV)
    c = synth.star_coeffs_laplacian(r) if shape == "star" else synth.box_coeffs(3, r)
    ref = grid.zeros(DEV)
    mms.stencil_apply(x, ref, grid, shape, r, c)
    torch.cuda.synchronize()
    out = grid.zeros(DEV)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            mms.stencil_apply(x, out, grid, shape, r, c)
            mms.stencil_apply(x, out, grid, shape, r, c)
    torch.cuda.synchronize()
    H = grid.halo
    want = ref.cpu().numpy()[H:H + nz, H:H + ny, H:H + nx]
    for rep in range(3):
        out.fill_(7.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got[H:H + nz, H:H + ny, H:H + nx], want), rep
        halo = got.copy()
        halo[H:H + nz, H:H + ny, H:H + nx] = 7.0
        assert np.all(halo == 7.0), rep
