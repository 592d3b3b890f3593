"""Shared helpers of the GPU parity tests: error metrics and tensor plumbing."""
import numpy as np


def rel_errors(got: np.ndarray, ref: np.ndarray):
    """Normwise errors: (max |got-ref| / max |ref|, ||got-ref||_2 / ||ref||_2)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = got - ref
    mref = np.max(np.abs(ref)) if ref.size else 0.0
    nref = np.linalg.norm(ref) if ref.size else 0.0
    rmax = float(np.max(np.abs(d)) / mref) if mref > 0 else float(np.max(np.abs(d), initial=0.0))
    rrms = float(np.linalg.norm(d) / nref) if nref > 0 else float(np.linalg.norm(d))
    return rmax, rrms


def interior(a, grid):
    H = grid.halo
    return a[H:H + grid.nz, H:H + grid.ny, H:H + grid.nx]


def halo_is_zero(a, grid):
    H = grid.halo
    m = np.ones(a.shape, dtype=bool)
    m[H:H + grid.nz, H:H + grid.ny, H:H + grid.nx] = False
    return not np.any(a[m])


def rel_errors_chunked(got: np.ndarray, ref: np.ndarray, chunk: int = 32):
    """rel_errors of two equally shaped [z][y][x] arrays, accumulated over chunks of z planes
    in FP64 (for full 512^3 grids: no whole-grid FP64 temporaries)."""
    assert got.shape == ref.shape
    dmax = rmax = dss = rss = 0.0
    for z0 in range(0, got.shape[0], chunk):
        g = np.asarray(got[z0:z0 + chunk], dtype=np.float64)
        r = np.asarray(ref[z0:z0 + chunk], dtype=np.float64)
        d = g - r
        dmax = max(dmax, float(np.max(np.abs(d))))
        rmax = max(rmax, float(np.max(np.abs(r))))
        dss += float(np.sum(d * d))
        rss += float(np.sum(r * r))
    return dmax / rmax, float(np.sqrt(dss / rss))
