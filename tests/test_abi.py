"""The C ABI loads, exports every declared entry point and rejects bad arguments
on the host, before any HIP call (these tests need no GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mmstencil.h")


@pytest.fixture(scope="module")
def L():
    from paper_2507_11067_amd import _lib
    return _lib.lib()


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(mms_[a-z0-9_]+)\s*\(", text)))


def test_header_symbols_exported(L):
    names = declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    from paper_2507_11067_amd import _lib
    assert sorted(_lib.EXPORTS) == names


def test_version_and_strerror(L):
    assert L.mms_abi_version() == 4
    for code in (0, -1, -2, -3, -4, -5):
        assert L.mms_strerror(code)
    assert L.mms_strerror(-5) != L.mms_strerror(-99)


def grid(nx=16, ny=16, nz=16, H=4, sy=None, sz=None):
    from paper_2507_11067_amd._lib import MmsGrid
    sy = ((nx + 3) // 4) * 4 + 2 * H if sy is None else sy
    sz = sy * (ny + 2 * H) if sz is None else sz
    return MmsGrid(nx, ny, nz, H, 0, sy, sz)


FAKE_IN = ctypes.c_void_p(0x10000)    # never dereferenced: every case fails validation
FAKE_OUT = ctypes.c_void_p(0x4000000)


def apply(L, g, shape=0, r=4, ncoeffs=None, prec=0, inp=FAKE_IN, out=FAKE_OUT, coeffs=True):
    w = 2 * r + 1
    n = ncoeffs if ncoeffs is not None else {0: 3 * w, 1: w ** 3, 2: 2 * w, 3: w * w}.get(shape, 1)
    buf = (ctypes.c_float * max(n, 1))()
    c = ctypes.cast(buf, ctypes.POINTER(ctypes.c_float)) if coeffs else None
    return L.mms_stencil_apply(inp, out, ctypes.byref(g) if g is not None else None, shape, r,
                               c, n, prec, None)


def test_stencil_apply_validation(L):
    EINVAL, EUNS = -1, -2
    assert apply(L, grid(), r=0) == EUNS
    assert apply(L, grid(), r=5) == EUNS
    assert apply(L, grid(), shape=4) == EUNS
    assert apply(L, grid(), shape=-1) == EUNS
    assert apply(L, grid(), shape=0, prec=1) == EUNS        # split precision on a star
    assert apply(L, grid(), shape=2, prec=1) == EUNS        # ... or on a 2-D shape
    assert apply(L, grid(), shape=3, prec=3) == EUNS
    assert apply(L, grid(), shape=2, ncoeffs=27) == EINVAL  # star2d takes 2(2r+1)
    assert apply(L, grid(), shape=3, ncoeffs=80) == EINVAL  # box2d takes (2r+1)^2
    assert apply(L, grid(H=2), shape=3, r=4) == EINVAL      # x/y halo < radius
    assert apply(L, grid(), prec=7) == EUNS
    assert apply(L, None) == EINVAL
    assert apply(L, grid(), inp=None) == EINVAL
    assert apply(L, grid(), coeffs=False) == EINVAL
    assert apply(L, grid(), ncoeffs=26) == EINVAL
    assert apply(L, grid(), shape=1, ncoeffs=728) == EINVAL
    assert apply(L, grid(H=2), r=4) == EINVAL               # halo < radius
    assert apply(L, grid(H=6), r=4) == EINVAL               # halo not a multiple of 4
    assert apply(L, grid(sy=22)) == EINVAL                  # pitch not a multiple of 4
    assert apply(L, grid(sy=20)) == EINVAL                  # pitch too small
    assert apply(L, grid(sz=24 * 23)) == EINVAL             # plane stride too small
    assert apply(L, grid(nx=-1)) == EINVAL
    assert apply(L, grid(nx=2 ** 30 + 1)) == EINVAL         # beyond 2^30 cells per axis
    assert apply(L, grid(nz=2 ** 30 + 1)) == EINVAL
    assert apply(L, grid(), out=ctypes.c_void_p(0x10008)) == EINVAL  # misaligned / overlapping
    assert apply(L, grid(), out=ctypes.c_void_p(0x10010)) == EINVAL  # overlapping


def test_wave_validation(L):
    from paper_2507_11067_amd._lib import MmsWave
    lap = (ctypes.c_float * 5)(-2.8, 1.6, -0.2, 0.025, -0.0018)
    w = MmsWave(grid(), 4, lap, ctypes.c_void_p(0x20000), 1.0, 8, 0.015, 47, 10, 2, 3, 4,
                None, None, None)
    vp = ctypes.c_void_p
    a, b, c = vp(0x100000), vp(0x800000), vp(0x1000000)
    assert L.mms_wave_step(ctypes.byref(w), 0, a, b, c, None) == -1      # n out of range
    w.image, w.acc_block = vp(0x3000000), 8                            # block without workspace
    assert L.mms_wave_step(ctypes.byref(w), 1, a, b, c, None) == -1
    w.acc_block = -1
    assert L.mms_wave_step(ctypes.byref(w), 1, a, b, c, None) == -1
    w.image, w.acc_block = None, 0
    assert L.mms_wave_step(ctypes.byref(w), 10, a, b, c, None) == -1
    assert L.mms_wave_step(ctypes.byref(w), 1, a, b, b, None) == -1      # u_next aliases u_cur
    assert L.mms_wave_step(ctypes.byref(w), 1, None, b, c, None) == -1
    assert L.mms_wave_record(ctypes.byref(w), 0, a, None) == -1          # no trace buffer
    w.radius = 5
    assert L.mms_wave_step(ctypes.byref(w), 1, a, b, c, None) == -2
    w.radius = 4
    w.src_dt2f = vp(0x30000)
    w.src_z = 99                                                          # source off the grid
    assert L.mms_wave_step(ctypes.byref(w), 1, a, b, c, None) == -1
    w.src_z = 2
    assert L.mms_wave_adjoint_step(ctypes.byref(w), 3, a, b, b, None, None, None, None) == -1
    assert L.mms_wave_adjoint_step(ctypes.byref(w), 3, a, b, c, None, None, vp(0x40), None) == -1
    arr = (vp * 3)(a, b, c)
    assert L.mms_wave_forward(ctypes.byref(w), 0, 3, arr, None) == -1
    assert L.mms_wave_forward(ctypes.byref(w), 1, 11, arr, None) == -1
    # mu-form adjoint: range, missing entries, aliasing, workspace and direction checks
    mus = (vp * 5)(a, b, c, a, b)
    us = (vp * 5)(c, c, c, c, c)
    assert L.mms_wave_adjoint_mu(ctypes.byref(w), 10, 0, mus, None, None, None, None) == -1
    assert L.mms_wave_adjoint_mu(ctypes.byref(w), 2, 3, mus, None, None, None, None) == -1
    assert L.mms_wave_adjoint_mu(ctypes.byref(w), 2, 0, None, None, None, None, None) == -1
    assert L.mms_wave_adjoint_mu(ctypes.byref(w), 2, 0, mus, None, None, vp(0x40), None) == -1
    bad = (vp * 5)(b, c, a, a, c)                           # at n = 2, mu^n aliases mu^{n+1}
    assert L.mms_wave_adjoint_mu(ctypes.byref(w), 2, 0, bad, None, None, None, None) == -1
    hole = (vp * 5)(a, b, None, a, b)
    assert L.mms_wave_adjoint_mu(ctypes.byref(w), 2, 0, hole, None, None, None, None) == -1
    w.acc_block = 8                                                       # blocks need acc_part
    assert L.mms_wave_adjoint_mu(ctypes.byref(w), 2, 0, mus, us, None, vp(0x40), None) == -1
    w.acc_block = 0
    assert L.mms_wave_scale_mu(ctypes.byref(w), a, b, 0, None) == -1
    assert L.mms_wave_scale_mu(ctypes.byref(w), a, vp(0x100040), 1, None) == -1  # partial overlap
    assert L.mms_wave_scale_mu(ctypes.byref(w), None, b, 1, None) == -1


def test_reduction_validation(L):
    """Reductions need a result pair and a workspace of their own: missing, misaligned
    or overlapping buffers are refused before anything is enqueued."""
    vp = ctypes.c_void_p
    a, b = vp(0x100000), vp(0x800000)
    out, work = vp(0x2000000), vp(0x3000000)
    g = grid()
    for fn, args in ((L.mms_flat_dot_f64, (a, b, 100)), (L.mms_flat_misfit_f64, (a, b, None, 100))):
        assert fn(*args, None, work, None) == -1                   # no result pair
        assert fn(*args, out, None, None) == -1                    # no workspace
        assert fn(*args, vp(0x2000004), work, None) == -1          # misaligned result
        assert fn(*args, out, vp(0x3000004), None) == -1           # misaligned workspace
        assert fn(*args, vp(0x3000000 + 8 * 2047), work, None) == -1  # result inside the workspace
        assert fn(*args, vp(0x3000000 - 8), work, None) == -1      # result overlaps its first word
    assert L.mms_flat_dot_f64(a, b, -1, out, work, None) == -1
    assert L.mms_flat_misfit_f64(a, None, None, 100, out, work, None) == -1
    assert L.mms_dot_f64(a, b, ctypes.byref(g), out, None, None) == -1
    assert L.mms_dot_f64(None, b, ctypes.byref(g), out, work, None) == -1
    assert L.mms_dot_f64(a, b, ctypes.byref(grid(sy=22)), out, work, None) == -1
    # the chain-rule scaling
    assert L.mms_flat_scale_f32(a, None, b, 10, None) == -1
    assert L.mms_flat_scale_f32(a, out, b, -1, None) == -1
    assert L.mms_flat_scale_f32(a, vp(0x2000004), b, 10, None) == -1
    assert L.mms_flat_scale_f32(a, out, vp(0x100004), 10, None) == -1   # partial overlap
    # energy: workspace size from the grid, and the same buffer rules
    from paper_2507_11067_amd._lib import MmsWave
    lap = (ctypes.c_float * 5)(-2.8, 1.6, -0.2, 0.025, -0.0018)
    w = MmsWave(grid(), 4, lap, vp(0x20000), 1.0, 0, 0.0, 0, 10, 0, 0, 0, None, None, None)
    need = ctypes.c_int64(-1)
    assert L.mms_wave_energy_work(ctypes.byref(w), ctypes.byref(need)) == 0
    assert need.value >= 2 and need.value % 2 == 0
    assert L.mms_wave_energy_work(ctypes.byref(w), None) == -1
    assert L.mms_wave_energy(ctypes.byref(w), a, b, out, work, need.value - 1, None) == -1
    assert L.mms_wave_energy(ctypes.byref(w), a, b, out, None, need.value, None) == -1
    assert L.mms_wave_energy(ctypes.byref(w), a, None, out, work, need.value, None) == -1
    assert L.mms_wave_energy(ctypes.byref(w), a, b, work, work, need.value, None) == -1
    w.g.nx = 0
    assert L.mms_wave_energy_work(ctypes.byref(w), ctypes.byref(need)) == 0 and need.value == 0


def test_check_reduction_flags_nonfinite(L):
    """The MMS_EUNSTABLE path: a result pair reporting NaN or Inf terms, or a non-finite
    sum, is an error; a clean pair is not."""
    pair = lambda v, c: (ctypes.c_double * 2)(v, c)
    assert L.mms_check_reduction(pair(1.5, 0.0)) == 0
    assert L.mms_check_reduction(pair(0.0, 0.0)) == 0
    assert L.mms_check_reduction(pair(-1e300, 0.0)) == 0
    assert L.mms_check_reduction(pair(1.5, 1.0)) == -5
    assert L.mms_check_reduction(pair(float("nan"), 0.0)) == -5
    assert L.mms_check_reduction(pair(float("inf"), 0.0)) == -5
    assert L.mms_check_reduction(pair(float("-inf"), 2.0)) == -5
    assert L.mms_check_reduction(None) == -1
    import torch
    from paper_2507_11067_amd import MmsError, check_result
    assert check_result(torch.tensor([2.5, 0.0], dtype=torch.float64)) == 2.5
    with pytest.raises(MmsError) as e:
        check_result(torch.tensor([2.5, 3.0], dtype=torch.float64))
    assert e.value.code == -5


def test_python_binding_requires_library(monkeypatch, tmp_path):
    """The binding raises instead of computing anything on the CPU when the library is absent."""
    from paper_2507_11067_amd import _lib
    monkeypatch.setattr(_lib, "LIB", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.lib()


def test_grid_aligned_layout(L):
    """mms_grid_aligned against Grid.aligned, and zeros()'s placement: interior rows on
    128-byte (32-element) boundaries relative to the allocation."""
    import ctypes
    import torch
    from paper_2507_11067_amd import Grid, _lib
    for nx, ny, nz, H in [(512, 512, 512, 4), (400, 3, 2, 4), (1, 1, 1, 8), (0, 5, 5, 4),
                          (256, 7, 9, 32), (29, 2, 3, 12)]:
        g = _lib.MmsGrid()
        lead = ctypes.c_int64(-1)
        assert L.mms_grid_aligned(nx, ny, nz, H, ctypes.byref(g), ctypes.byref(lead)) == 0
        p = Grid.aligned(nx, ny, nz, H)
        assert (g.nx, g.ny, g.nz, g.halo, g.sy, g.sz) == (nx, ny, nz, H, p.sy, p.sz)
        assert lead.value == p.lead
        assert g.sy % 32 == 0 and g.sy >= ((nx + 3) // 4) * 4 + 2 * H and g.sy - 32 < ((nx + 3) // 4) * 4 + 2 * H
        t = p.zeros("cpu")
        assert tuple(t.shape) == p.shape and t.is_contiguous() and t.storage_offset() == p.lead
        assert (p.lead + H * (p.sz + p.sy + 1)) % 32 == 0
        assert not t.any()
    # the default layout keeps its pitch and no lead
    d = Grid(512, 512, 512)
    assert d.sy == 520 and d.lead == 0 and d.zeros("cpu").storage_offset() == 0
    g = _lib.MmsGrid()
    lead = ctypes.c_int64()
    for args in [(-1, 1, 1, 4), (1, 1, 1, 2), (1, 1, 1, 0), (1, -1, 1, 4)]:
        assert L.mms_grid_aligned(*args, ctypes.byref(g), ctypes.byref(lead)) == -1
    assert L.mms_grid_aligned(1, 1, 1, 4, None, ctypes.byref(lead)) == -1


def test_energy_noalloc_refuses_grids_beyond_its_scratch(L):
    """The no-allocation energy refuses, before any HIP call, a grid whose per-block
    partials do not fit its static scratch (4096^3: 131072 blocks), and names the sizes."""
    from paper_2507_11067_amd._lib import MmsWave
    vp = ctypes.c_void_p
    lap = (ctypes.c_float * 5)(-2.8, 1.6, -0.2, 0.025, -0.0018)
    big = grid(4096, 4096, 4096)
    w = MmsWave(big, 4, lap, vp(0x20000), 1.0, 0, 0.0, 0, 10, 0, 0, 0, None, None, None)
    need = ctypes.c_int64(0)
    assert L.mms_wave_energy_work(ctypes.byref(w), ctypes.byref(need)) == 0
    assert need.value > 65536
    assert L.mms_wave_energy_noalloc(ctypes.byref(w), vp(0x100000), vp(0x800000),
                                     vp(0x2000000), None) == -1
    msg = L.mms_last_error().decode()
    assert str(need.value) in msg and "65536" in msg
    small = MmsWave(grid(), 4, lap, vp(0x20000), 1.0, 0, 0.0, 0, 10, 0, 0, 0, None, None, None)
    assert L.mms_wave_energy_noalloc(ctypes.byref(small), vp(0x100000), None, vp(0x2000000),
                                     None) == -1
    assert L.mms_wave_energy_noalloc(ctypes.byref(small), vp(0x100000), vp(0x800000),
                                     vp(0x2000004), None) == -1      # misaligned result pair


def test_fp32_box_refuses_rows_too_long_for_tile_offsets(L):
    """From radius 2 on the FP32 box addresses its plane tile with 32-bit offsets; a
    pitch whose (33 + 2r) rows reach 2^32 elements is refused before any HIP call."""
    sy = 2 ** 28                                  # 37 rows: 9.9e9 elements
    g = grid(nx=4, ny=1, nz=1, sy=sy)
    nbytes = 9 * g.sz * 4                         # (nz + 2H) planes
    out = ctypes.c_void_p(0x10000 + nbytes)
    for r in (2, 3, 4):
        assert apply(L, g, shape=1, r=r, out=out) == -2, r
        assert "32-bit" in L.mms_last_error().decode()


def test_tti_refuses_rows_too_long_for_tile_offsets(L):
    """TTI pass 2 addresses its plane tiles with 32-bit offsets; a pitch whose 17 rows reach
    2^32 elements is refused before either pass is launched (no HIP call)."""
    from paper_2507_11067_amd._lib import MmsTti, MmsWave
    g = grid(nx=4, ny=1, nz=1, sy=2 ** 28)
    nbytes = 9 * g.sz * 4
    step = 4 * nbytes + (1 << 20)
    ptr = [ctypes.c_void_p(0x10000 + k * step) for k in range(12)]
    lap = (ctypes.c_float * 5)(-2.8, 1.6, -0.2, 0.025, -0.0018)
    w = MmsWave(g, 4, lap, ptr[0], 1.0, 0, 0.0, 0, 10, 0, 0, 0, None, None, None)
    d1 = (ctypes.c_float * 4)(0.8, -0.2, 0.038, -0.0036)
    t = MmsTti(ptr[1], ptr[2], ptr[3], ptr[4], 0.1, 1.0, d1, ptr[5])
    rc = L.mms_tti_step(ctypes.byref(w), ctypes.byref(t), 1, ptr[6], ptr[7], ptr[8], ptr[9],
                        ptr[10], ptr[11], None)
    assert rc == -2, rc
    assert "32-bit" in L.mms_last_error().decode()


def test_vti_refuses_rows_too_long_for_tile_offsets(L):
    """The VTI step addresses its H tile with 32-bit offsets; a pitch whose 17 rows reach
    2^32 elements is refused before the kernel is launched (no HIP call)."""
    from paper_2507_11067_amd._lib import MmsWave
    g = grid(nx=4, ny=1, nz=1, sy=2 ** 28)
    nbytes = 9 * g.sz * 4
    step = 4 * nbytes + (1 << 20)
    ptr = [ctypes.c_void_p(0x10000 + k * step) for k in range(9)]
    lap = (ctypes.c_float * 5)(-2.8, 1.6, -0.2, 0.025, -0.0018)
    w = MmsWave(g, 4, lap, ptr[0], 1.0, 0, 0.0, 0, 10, 0, 0, 0, None, None, None)
    rc = L.mms_vti_step(ctypes.byref(w), 1, ptr[1], ptr[2], ptr[3], ptr[4], ptr[5], ptr[6],
                        ptr[7], ptr[8], None)
    assert rc == -2, rc
    assert "32-bit" in L.mms_last_error().decode()


@pytest.mark.parametrize("empty", [dict(nx=0), dict(ny=0), dict(nz=0)], ids=["nx0", "ny0", "nz0"])
def test_steps_on_empty_grids_return_before_any_launch(L, empty):
    """The acoustic, adjoint, VTI and TTI steps on a grid with no interior cells validate
    their arguments and return MMS_OK without a HIP call (the pointers are never read)."""
    from paper_2507_11067_amd._lib import MmsTti, MmsWave
    g = grid(**empty)
    step = 4 * g.sz * (g.nz + 2 * g.halo) * 4 + (1 << 20)
    ptr = [ctypes.c_void_p(0x10000 + k * step) for k in range(16)]
    lap = (ctypes.c_float * 5)(-2.8, 1.6, -0.2, 0.025, -0.0018)
    w = MmsWave(g, 4, lap, ptr[0], 1.0, 0, 0.0, 0, 10, 0, 0, 0, None, None, None)
    assert L.mms_wave_step(ctypes.byref(w), 1, ptr[1], ptr[2], ptr[3], None) == 0
    assert L.mms_wave_adjoint_step(ctypes.byref(w), 3, ptr[1], ptr[2], ptr[3], None, None, None,
                                   None) == 0
    assert L.mms_vti_step(ctypes.byref(w), 1, ptr[1], ptr[2], ptr[3], ptr[4], ptr[5], ptr[6],
                          ptr[7], ptr[8], None) == 0
    d1 = (ctypes.c_float * 4)(0.8, -0.2, 0.038, -0.0036)
    t = MmsTti(ptr[9], ptr[10], ptr[11], ptr[12], 0.1, 1.0, d1, ptr[13])
    assert L.mms_tti_step(ctypes.byref(w), ctypes.byref(t), 1, ptr[1], ptr[2], ptr[3], ptr[4],
                          ptr[5], ptr[6], None) == 0
