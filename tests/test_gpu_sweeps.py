"""GPU parity of the star and box sweeps against the FP64 oracle.

Gate (normwise, one sweep from identical FP32 inputs): max|y - y*| / max|y*|
<= 1e-5 for FP32, BF16X3 and FP16X3S; the BF16X1 variant is reported and only
checked to stay near its expected 1e-3 level.
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


def run(mms, x_np, grid, shape, r, c, prec="fp32", out_fill=0.0):
    # grid.zeros() places the arrays (interior rows on 128-byte boundaries for Grid.aligned)
    x = grid.zeros(DEV)
    x.copy_(torch.from_numpy(x_np))
    out = grid.zeros(DEV).fill_(out_fill)
    mms.stencil_apply(x, out, grid, shape, r, c, precision=prec)
    torch.cuda.synchronize()
    return out.cpu().numpy()


SIZES = [(8, 8, 8), (17, 19, 23), (5, 3, 2), (1, 1, 1), (64, 64, 64), (133, 37, 20)]
# grids of at most 2^20 points (all of SIZES) take the star's direct small-grid kernel;
# these larger ragged ones take the z-marching kernel
STAR_SIZES = SIZES + [(133, 100, 80), (70, 130, 150)]


@pytest.mark.parametrize("r", [1, 2, 3, 4])
@pytest.mark.parametrize("size", STAR_SIZES, ids=lambda s: "x".join(map(str, s)))
def test_star_parity(mms, r, size):
    nx, ny, nz = size
    grid = mms.Grid(nx, ny, nz)
    x = synth.uniform_grid(100 + r, nx, ny, nz, sy=grid.sy)
    c = synth.star_coeffs_random(200 + r, r)
    got = run(mms, x, grid, "star", r, c, out_fill=7.0)
    ref = oracle.star(x, nx, ny, nz, r, c)
    rmax, _ = rel_errors(interior(got, grid), interior(ref, grid))
    assert rmax <= TOL, rmax
    # the halo of the output is never written
    H = grid.halo
    o = got.copy()
    o[H:H + nz, H:H + ny, H:H + nx] = 0
    assert np.all((o == 7.0) | (o == 0))
    assert np.count_nonzero(o == 0) == nz * ny * nx


def test_star_laplacian_64_config0(mms):
    """Workload: radius-4 Laplacian star, 64^3, zero halo, uniform [-1, 1] (seed 1), 10 sweeps."""
    n = 64
    grid = mms.Grid(n, n, n)
    x = synth.uniform_grid(1, n, n, n, sy=grid.sy)
    c = synth.star_coeffs_laplacian(4)
    xt = torch.from_numpy(x).to(DEV)
    out = grid.zeros(DEV)
    outs = []
    for _ in range(10):
        mms.stencil_apply(xt, out, grid, "star", 4, c)
        outs.append(out.clone())
    torch.cuda.synchronize()
    ref = oracle.star(x, n, n, n, 4, c)
    for o in outs:  # repeated sweeps are bitwise identical
        assert torch.equal(o, outs[0])
    rmax, rrms = rel_errors(interior(outs[0].cpu().numpy(), grid), interior(ref, grid))
    print(f"star r4 64^3: rel_max {rmax:.2e} rel_rms {rrms:.2e}")
    assert rmax <= TOL


@pytest.mark.parametrize("dims", [(30, 21, 13, 64), (120, 100, 90, 160)],
                         ids=["direct-30x21x13", "marching-120x100x90"])
def test_star_nonzero_halo_and_wide_pitch(mms, dims):
    """Halo cells are read as stored; a wider row pitch and an 8-cell halo are honoured (by the
    small-grid kernel and by the z-marching one)."""
    nx, ny, nz, sy = dims
    H = 8
    grid = mms.Grid(nx, ny, nz, halo=H, sy=sy)
    rng = np.random.default_rng(5)
    x = rng.uniform(-1, 1, grid.shape).astype(np.float32)
    c = synth.star_coeffs_random(6, 4)
    got = run(mms, x, grid, "star", 4, c)
    ref = oracle.star(x, nx, ny, nz, 4, c, halo=H)
    rmax, _ = rel_errors(interior(got, grid), interior(ref, grid))
    assert rmax <= TOL


@pytest.mark.parametrize("r", [1, 2, 3, 4])
@pytest.mark.parametrize("shape,prec", [("box", "fp32"), ("box", "bf16x3"), ("box", "fp16x3s"),
                                        ("star2d", "fp32"), ("box2d", "fp32")])
def test_nonzero_halo_and_wide_pitch(mms, shape, prec, r):
    """Halo cells are read as stored by every sweep kernel (the star has its own case above):
    random values in an 8-cell halo, a row pitch wider than the rows need, and a ragged
    interior (30 x 21 x 13) so that tiles end inside the halo."""
    nx, ny, nz, H = 30, 21, 13, 8
    grid = mms.Grid(nx, ny, nz, halo=H, sy=64)
    rng = np.random.default_rng(50 + r)
    x = rng.uniform(-1, 1, grid.shape).astype(np.float32)
    w = 2 * r + 1
    if shape == "box":
        c, ref_fn = synth.box_coeffs(60 + r, r), oracle.box
    elif shape == "box2d":
        c, ref_fn = synth.box2d_coeffs(70 + r, r), oracle.box2d
    else:
        c, ref_fn = rng.uniform(-1, 1, (2, w)).astype(np.float32), oracle.star2d
    got = run(mms, x, grid, shape, r, c, prec)
    ref = ref_fn(x, nx, ny, nz, r, c, halo=H)
    rmax, rrms = rel_errors(interior(got, grid), interior(ref, grid))
    assert rmax <= TOL, (rmax, rrms)


@pytest.mark.parametrize("r", [1, 2, 3, 4])
@pytest.mark.parametrize("size", [(8, 8, 8), (17, 19, 23), (70, 33, 40), (3, 2, 5)],
                         ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "fp16x3s"])
def test_box_parity(mms, r, size, prec):
    nx, ny, nz = size
    grid = mms.Grid(nx, ny, nz)
    x = synth.uniform_grid(300 + r, nx, ny, nz, sy=grid.sy)
    c = synth.box_coeffs(400 + r, r)
    got = run(mms, x, grid, "box", r, c, prec)
    ref = oracle.box(x, nx, ny, nz, r, c)
    rmax, rrms = rel_errors(interior(got, grid), interior(ref, grid))
    assert rmax <= TOL, (rmax, rrms)
    assert halo_is_zero(got, grid)


@pytest.mark.parametrize("r", [2, 4])
def test_box_bf16x1_reported(mms, r):
    n = 40
    grid = mms.Grid(n, n, n)
    x = synth.uniform_grid(7, n, n, n, sy=grid.sy)
    c = synth.box_coeffs(8, r)
    got = run(mms, x, grid, "box", r, c, "bf16x1")
    ref = oracle.box(x, n, n, n, r, c)
    rmax, rrms = rel_errors(interior(got, grid), interior(ref, grid))
    print(f"box r{r} bf16x1: rel_max {rmax:.2e} rel_rms {rrms:.2e}")
    assert 1e-5 < rmax < 2e-2


def test_box_split_exact_on_representable_inputs(mms):
    """Data and weights exactly representable in BF16 and FP16: lo parts vanish and the
    MFMA result matches the FP32 sweep up to accumulation order."""
    n, r = 24, 3
    grid = mms.Grid(n, n, n)
    rng = np.random.default_rng(9)
    x = synth.padded_zeros(n, n, n, sy=grid.sy)
    synth.interior(x, n, n, n)[...] = rng.integers(-64, 65, (n, n, n)) / 64.0
    c = (rng.integers(-16, 17, (7, 7, 7)) / 16.0).astype(np.float32)
    ref = run(mms, x, grid, "box", r, c, "fp32")
    for prec in ("bf16x3", "fp16x3s", "bf16x1"):
        got = run(mms, x, grid, "box", r, c, prec)
        rmax, _ = rel_errors(interior(got, grid), interior(ref, grid))
        assert rmax <= 1e-6, (prec, rmax)


def test_box_large_values_fp16_scaling(mms):
    """Per-block power-of-two scaling keeps FP16 in range for data far outside [-1, 1]."""
    n, r = 32, 2
    grid = mms.Grid(n, n, n)
    x = synth.uniform_grid(10, n, n, n, lo=-3e6, hi=3e6, sy=grid.sy)
    c = synth.box_coeffs(11, r) * 1e3
    got = run(mms, x, grid, "box", r, c, "fp16x3s")
    ref = oracle.box(x, n, n, n, r, c)
    rmax, _ = rel_errors(interior(got, grid), interior(ref, grid))
    assert rmax <= TOL


@pytest.mark.parametrize("shape,prec", [("star", "fp32"), ("box", "fp32"), ("box", "bf16x3"),
                                        ("box", "fp16x3s")])
def test_empty_grid_is_noop(mms, shape, prec):
    grid = mms.Grid(0, 5, 6)
    x = grid.zeros(DEV)
    out = torch.full(grid.shape, 3.0, device=DEV)
    c = np.ones(27 if shape == "star" else 729, dtype=np.float32)
    mms.stencil_apply(x, out, grid, shape, 4, c, precision=prec)
    torch.cuda.synchronize()
    assert torch.all(out == 3.0)


@pytest.mark.parametrize("shape,prec,r", [("star", "fp32", 4), ("box", "fp32", 2),
                                          ("box", "bf16x3", 4), ("box", "fp16x3s", 3)])
def test_deterministic(mms, shape, prec, r):
    n = 48
    grid = mms.Grid(n, n, n)
    x = torch.from_numpy(synth.uniform_grid(12, n, n, n, sy=grid.sy)).to(DEV)
    c = synth.star_coeffs_random(13, r) if shape == "star" else synth.box_coeffs(13, r)
    a, b = grid.zeros(DEV), grid.zeros(DEV)
    mms.stencil_apply(x, a, grid, shape, r, c, precision=prec)
    mms.stencil_apply(x, b, grid, shape, r, c, precision=prec)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.fixture(scope="module")
def big512():
    """The benchmark's 512^3 input (uniform [-1, 1], seed 2) on its layout: rows padded to
    544, interior rows on 128-byte boundaries; plus a cache of full-grid oracle sweeps."""
    n = 512
    x = synth.uniform_grid(2, n, n, n, sy=((n + 8 + 31) // 32) * 32)
    return {"n": n, "x": x, "x64": x.astype(np.float64), "ref": {}}


def oracle_512(big, shape, r, c):
    """Interior of the full-grid FP64 oracle sweep, computed once per (shape, r)."""
    key = (shape, r)
    if key not in big["ref"]:
        n = big["n"]
        f = oracle.star if shape == "star" else oracle.box
        full = f(big["x64"], n, n, n, r, c)
        big["ref"][key] = np.ascontiguousarray(full[4:4 + n, 4:4 + n, 4:4 + n])
        del full
    return big["ref"][key]


def test_star_512_full_grid(mms, big512):
    """Full-size workload (512^3, radius-4 Laplacian) in the benchmark's launch shape, every
    one of the 134,217,728 outputs against the full-grid FP64 oracle sweep."""
    n = big512["n"]
    grid = mms.Grid.aligned(n, n, n)
    c = synth.star_coeffs_laplacian(4)
    got = run(mms, big512["x"], grid, "star", 4, c)
    rmax, rrms = rel_errors_chunked(interior(got, grid), oracle_512(big512, "star", 4, c))
    print(f"star r4 512^3 full grid: rel_max {rmax:.2e} rel_rms {rrms:.2e}")
    assert rmax <= TOL, rmax
    assert halo_is_zero(got, grid)


@pytest.mark.parametrize("r,prec", [(2, "fp32"), (4, "fp32"), (3, "fp32"), (3, "bf16x3"),
                                    (4, "bf16x3"), (3, "fp16x3s"), (4, "fp16x3s"),
                                    (4, "bf16x1"), (3, "bf16x1")])
def test_box_512_full_grid(mms, big512, r, prec):
    """Every output of the 512^3 box sweeps (the headline's radius-2 and radius-4 FP32
    boxes, and radius 3 and 4 in each split precision) against the full-grid FP64 oracle."""
    n = big512["n"]
    grid = mms.Grid.aligned(n, n, n)
    c = synth.box_coeffs({2: 3, 3: 6, 4: 4}[r], r)
    got = run(mms, big512["x"], grid, "box", r, c, prec)
    rmax, rrms = rel_errors_chunked(interior(got, grid), oracle_512(big512, "box", r, c))
    print(f"box r{r} {prec} 512^3 full grid: rel_max {rmax:.2e} rel_rms {rrms:.2e}")
    assert halo_is_zero(got, grid)
    if prec == "bf16x1":
        assert rmax < 2e-2      # the reduced-accuracy variant: reported, near its 2e-3 level
    else:
        assert rmax <= TOL, rmax


@pytest.mark.parametrize("dims", [(64, 64, 64, 4), (300, 9, 13, 4), (133, 37, 20, 4),
                                  (37, 19, 11, 8)],
                         ids=lambda d: "x".join(map(str, d[:3])) + f"-H{d[3]}")
def test_aligned_layout_bit_identical(mms, dims):
    """Sweeps on the 128-byte-row layout (Grid.aligned with zeros()'s placement) against the
    default layout: the same kernels at other addresses, so the interiors are bit-identical
    and the halo stays unwritten; the star is also checked against the oracle."""
    nx, ny, nz, H = dims
    ga, gd = mms.Grid.aligned(nx, ny, nz, H), mms.Grid(nx, ny, nz, H)
    xa_np = synth.uniform_grid(7, nx, ny, nz, halo=H, sy=ga.sy)
    xa = ga.zeros(DEV)
    xa.copy_(torch.from_numpy(xa_np))
    assert (xa.data_ptr() + 4 * ga.halo * (ga.sz + ga.sy + 1)) % 128 == 0
    xd = torch.from_numpy(synth.uniform_grid(7, nx, ny, nz, halo=H, sy=gd.sy)).to(DEV)
    rng = np.random.default_rng(8)
    cases = [("star", 4, synth.star_coeffs_random(9, 4), "fp32"),
             ("box", 1, synth.box_coeffs(10, 1), "fp32"),
             ("box", 2, synth.box_coeffs(11, 2), "fp32"),
             ("box", 4, synth.box_coeffs(12, 4), "bf16x3"),
             ("star2d", 4, rng.uniform(-1, 1, (2, 9)).astype(np.float32), "fp32"),
             ("box2d", 3, rng.uniform(-1, 1, (7, 7)).astype(np.float32), "fp32")]
    for shape, r, c, prec in cases:
        oa = ga.zeros(DEV).fill_(7.0)
        od = torch.full(gd.shape, 7.0, device=DEV)
        mms.stencil_apply(xa, oa, ga, shape, r, c, precision=prec)
        mms.stencil_apply(xd, od, gd, shape, r, c, precision=prec)
        torch.cuda.synchronize()
        a, d = oa.cpu().numpy(), od.cpu().numpy()
        assert np.array_equal(interior(a, ga), interior(d, gd)), (shape, r, prec)
        h = a.copy()
        interior(h, ga)[...] = 7.0
        assert np.all(h == 7.0), (shape, r, prec)
        if shape == "star":
            ref = oracle.star(xa_np, nx, ny, nz, r, c, halo=H)
            rmax, _ = rel_errors(interior(a, ga), interior(ref, ga))
            assert rmax <= TOL, rmax
