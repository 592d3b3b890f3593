"""mms_wave_energy_noalloc (partials in the library's static device scratch, no
allocation, no workspace) against mms_wave_energy with a caller workspace, called through
the C ABI: two calls in a row on one stream, the second on a smaller grid, then an empty
grid."""
import ctypes

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
LAP = [float(v) for v in synth.LAPLACIAN_R4]


def p(t):
    return ctypes.c_void_p(t.data_ptr())


def test_energy_noalloc_matches_workspace_entry():
    from paper_2507_11067_amd import Grid, Wave, _lib
    L = _lib.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for (nx, ny, nz), seed in (((96, 93, 89), 1), ((40, 37, 33), 2)):
        g = Grid(nx, ny, nz)
        rng = np.random.default_rng(seed)
        c2 = synth.padded_zeros(nx, ny, nz, sy=g.sy)
        synth.interior(c2, nx, ny, nz)[...] = rng.uniform(0.05, 0.15, (nz, ny, nx))
        w = Wave(g, torch.from_numpy(c2).to(DEV), LAP, 4)
        u0 = torch.from_numpy(synth.uniform_grid(10 + seed, nx, ny, nz, sy=g.sy)).to(DEV)
        u1 = torch.from_numpy(synth.uniform_grid(20 + seed, nx, ny, nz, sy=g.sy)).to(DEV)
        need = w.energy_work()
        assert 0 < need <= 65536
        work = torch.empty(need, dtype=torch.float64, device=DEV)
        ref = torch.full((2,), float("nan"), dtype=torch.float64, device=DEV)
        got = torch.full((2,), float("nan"), dtype=torch.float64, device=DEV)
        assert L.mms_wave_energy(ctypes.byref(w._w), p(u0), p(u1), p(ref), p(work), need,
                                 stream) == 0
        assert L.mms_wave_energy_noalloc(ctypes.byref(w._w), p(u0), p(u1), p(got), stream) == 0
        torch.cuda.synchronize()
        r, q = ref.cpu().numpy(), got.cpu().numpy()
        print(f"{nx}x{ny}x{nz}: workspace {r}, static scratch {q}")
        assert np.isfinite(r[0]) and r[1] == 0
        np.testing.assert_array_equal(q, r)      # same kernels, same order: bit-identical
    g0 = Grid(0, 5, 5)
    w0 = Wave(g0, g0.zeros(DEV), LAP, 4)
    z = g0.zeros(DEV)
    out = torch.full((2,), float("nan"), dtype=torch.float64, device=DEV)
    assert L.mms_wave_energy_noalloc(ctypes.byref(w0._w), p(z), p(z), p(out), stream) == 0
    torch.cuda.synchronize()
    assert out.cpu().tolist() == [0.0, 0.0]
