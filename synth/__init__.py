"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds input recipes only: grids of random numbers, coefficient
tables, the layered velocity model, the Ricker source time function and the
padded-grid layout.  It contains none of the stencil or wave-step arithmetic;
the HIP library and the FP64 oracle each implement that on their own.

Layout convention (shared interface, not arithmetic): a grid is a float array of
shape ``[nz + 2H][ny + 2H][sy]`` with x fastest.  Interior point (z, y, x) lives
at ``[z + H][y + H][x + H]``.  ``sy`` is the row pitch in elements; it is a
multiple of 4 and leaves at least ``roundup4(nx) + 2H`` elements per row so that
16-byte loads of the last interior column stay inside the row.
"""
from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction

import numpy as np

HALO = 4

# Per-axis second-derivative weights of the radius-4 (8th-order) central
# difference at unit spacing, as the workload fixes them: centre, then k=1..4.
LAPLACIAN_R4 = (Fraction(-205, 72), Fraction(8, 5), Fraction(-1, 5),
                Fraction(8, 315), Fraction(-1, 560))
# 4th-order (radius-2) weights, used by the radius-2 stars of Table I
LAPLACIAN_R2 = (Fraction(-5, 2), Fraction(4, 3), Fraction(-1, 12))
# 8th-order central first derivative: D f(i) = sum_k d_k (f(i+k) - f(i-k)), k = 1..4
FIRST_DERIV_R4 = (Fraction(4, 5), Fraction(-1, 5), Fraction(4, 105), Fraction(-1, 280))


def row_pitch(nx: int, halo: int = HALO, align: int = 4) -> int:
    """Smallest row pitch that satisfies the layout rule, rounded up to ``align``."""
    need = ((nx + 3) // 4) * 4 + 2 * halo
    return ((need + align - 1) // align) * align


def padded_zeros(nx: int, ny: int, nz: int, halo: int = HALO, dtype=np.float32,
                 sy: int | None = None) -> np.ndarray:
    sy = row_pitch(nx, halo) if sy is None else sy
    return np.zeros((nz + 2 * halo, ny + 2 * halo, sy), dtype=dtype)


def interior(a: np.ndarray, nx: int, ny: int, nz: int, halo: int = HALO) -> np.ndarray:
    """View of the interior of a padded grid."""
    return a[halo:halo + nz, halo:halo + ny, halo:halo + nx]


def uniform_grid(seed: int, nx: int, ny: int, nz: int, halo: int = HALO,
                 lo: float = -1.0, hi: float = 1.0, sy: int | None = None) -> np.ndarray:
    """Padded FP32 grid, zero halo, interior uniform in [lo, hi) from ``seed``."""
    rng = np.random.default_rng(seed)
    a = padded_zeros(nx, ny, nz, halo, np.float32, sy)
    interior(a, nx, ny, nz, halo)[...] = rng.uniform(lo, hi, (nz, ny, nx)).astype(np.float32)
    return a


def laplacian_weights(radius: int = 4) -> np.ndarray:
    """FP32 per-axis weights [k = -r..r] of the radius-4 (8th-order) or radius-2
    (4th-order) Laplacian."""
    if radius not in (2, 4):
        raise ValueError("Laplacian weights are fixed for radius 2 and 4 only")
    half = [float(f) for f in (LAPLACIAN_R4 if radius == 4 else LAPLACIAN_R2)]
    return np.array(half[:0:-1] + half, dtype=np.float32)


def star_coeffs_laplacian(radius: int = 4) -> np.ndarray:
    """Star coefficient table [axis z, y, x][k = -r..r] (FP32) for the Laplacian."""
    w = laplacian_weights(radius)
    return np.stack([w, w, w]).astype(np.float32)


def star2d_coeffs_laplacian(radius: int = 4) -> np.ndarray:
    """2-D star table [axis y, x][k = -r..r] (FP32) for the Laplacian."""
    w = laplacian_weights(radius)
    return np.stack([w, w]).astype(np.float32)


def box2d_coeffs(seed: int, radius: int) -> np.ndarray:
    """2-D box weights [dy][dx]: uniform [-1, 1) in FP64, mean removed, cast to FP32."""
    rng = np.random.default_rng(seed)
    n = 2 * radius + 1
    c = rng.uniform(-1.0, 1.0, (n, n))
    c -= c.mean()
    return c.astype(np.float32)


def star_coeffs_random(seed: int, radius: int) -> np.ndarray:
    """Seeded, non-symmetric star coefficients [3][2r+1] in [-1, 1) (FP32)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, (3, 2 * radius + 1)).astype(np.float32)


def box_coeffs(seed: int, radius: int) -> np.ndarray:
    """Box coefficients [dz][dy][dx]: uniform [-1, 1) in FP64, mean removed, cast to FP32."""
    rng = np.random.default_rng(seed)
    n = 2 * radius + 1
    c = rng.uniform(-1.0, 1.0, (n, n, n))
    c -= c.mean()
    return c.astype(np.float32)


def ricker(nt: int, dt: float, f0: float = 15.0) -> np.ndarray:
    """Ricker wavelet samples f(n*dt), n = 0..nt-1, delayed by 1/f0 (FP64)."""
    t = np.arange(nt, dtype=np.float64) * dt - 1.0 / f0
    a = (np.pi * f0 * t) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def layered_velocity(n: int, seed: int | None, nz: int | None = None, ny: int | None = None,
                     perturb: float = 0.05, sigma: float = 8.0) -> np.ndarray:
    """Layered model (5 equal layers, 1500..4500 m/s) times (1 + perturb * p).

    ``p`` is seeded white noise smoothed by a Gaussian filter of width ``sigma``
    cells and scaled to max |p| = 1.  ``seed=None`` gives the layers alone.
    Returns the interior as FP64 [nz][ny][nx].
    """
    nx = n
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    layer = (5 * np.arange(nz)) // nz
    v = (1500.0 + 750.0 * layer)[:, None, None] * np.ones((nz, ny, nx))
    if seed is not None and perturb != 0.0:
        from scipy.ndimage import gaussian_filter
        rng = np.random.default_rng(seed)
        noise = rng.standard_normal((nz, ny, nx)).astype(np.float32)
        p = gaussian_filter(noise, sigma=sigma, mode="reflect").astype(np.float64)
        p /= np.abs(p).max()
        v *= 1.0 + perturb * p
    return v


@dataclass
class WaveSetup:
    """Everything a forward or adjoint run takes as input, on the padded layout."""
    nx: int
    ny: int
    nz: int
    h: float
    dt: float
    c2: np.ndarray            # padded FP32: (v dt / h)^2, zero halo
    src: tuple                # (z, y, x) interior index of the point source
    src_dt2f: np.ndarray      # FP32 [nt]: dt^2 * f(n dt)
    nt: int
    sponge_width: int
    sponge_alpha: float
    sponge_faces: int         # bit mask: 1 x-lo, 2 x-hi, 4 y-lo, 8 y-hi, 16 z-lo, 32 z-hi
    v: np.ndarray             # FP64 interior velocity


SPONGE_LATERAL_AND_BOTTOM = 1 | 2 | 4 | 8 | 32


def wave_setup(n: int, nt: int, seed: int | None, h: float = 10.0, courant: float = 0.4,
               f0: float = 15.0, src_depth_m: float = 50.0, sponge_width: int | None = None,
               sponge_alpha: float = 0.015, dt: float | None = None,
               v: np.ndarray | None = None) -> WaveSetup:
    """The acoustic workload recipe on an n^3 grid.

    ``dt`` defaults to courant * h / max(v); pass it explicitly to share one time
    step between a perturbed and an unperturbed model.
    """
    if v is None:
        v = layered_velocity(n, seed)
    if dt is None:
        dt = courant * h / float(v.max())
    if sponge_width is None:
        sponge_width = 32 if n >= 128 else 8
    c2 = padded_zeros(n, n, n)
    interior(c2, n, n, n)[...] = ((v * dt / h) ** 2).astype(np.float32)
    src = (int(round(src_depth_m / h)), n // 2, n // 2)
    src_dt2f = (dt * dt * ricker(nt, dt, f0)).astype(np.float32)
    return WaveSetup(n, n, n, h, dt, c2, src, src_dt2f, nt, sponge_width, sponge_alpha,
                     SPONGE_LATERAL_AND_BOTTOM, v)


def smooth_random_grid(seed: int, nx: int, ny: int, nz: int, sigma: float = 2.0) -> np.ndarray:
    """Padded FP32 grid with a seeded, Gaussian-smoothed interior of unit max."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    p = gaussian_filter(rng.standard_normal((nz, ny, nx)), sigma=sigma, mode="reflect")
    p /= np.abs(p).max()
    a = padded_zeros(nx, ny, nz)
    interior(a, nx, ny, nz)[...] = p.astype(np.float32)
    return a


def thomsen_fields(nx: int, ny: int, nz: int, seed: int, sy: int | None = None):
    """Padded FP32 Thomsen parameters (epsilon, delta) of a layered VTI medium:
    five depth layers with epsilon in [0.05, 0.25] and delta in [0, 0.12],
    delta <= epsilon, each with a smooth +-10% perturbation; zero halo."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    bounds = np.sort(rng.uniform(0.1, 0.9, 4)) * nz
    layer = np.searchsorted(bounds, np.arange(nz) + 0.5)
    eps_l = rng.uniform(0.05, 0.25, 5)
    del_l = np.minimum(rng.uniform(0.0, 0.12, 5), eps_l)
    noise = gaussian_filter(rng.standard_normal((nz, ny, nx)), sigma=4.0, mode="reflect")
    noise *= 0.1 / max(np.abs(noise).max(), 1e-30)
    out = []
    for vals in (eps_l, del_l):
        a = padded_zeros(nx, ny, nz, sy=sy)
        interior(a, nx, ny, nz)[...] = (vals[layer][:, None, None] * (1 + noise)).astype(np.float32)
        out.append(a)
    return out[0], out[1]


def tilt_fields(nx: int, ny: int, nz: int, seed: int, theta_max: float = np.pi / 4,
                sy: int | None = None):
    """Padded FP32 tilt (theta, from the vertical) and azimuth (phi) fields of a TTI
    medium: theta smooth in [0, theta_max], phi smooth over [0, 2 pi); zero halo."""
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    out = []
    for lo, hi in ((0.0, theta_max), (0.0, 2 * np.pi)):
        f = gaussian_filter(rng.standard_normal((nz, ny, nx)), sigma=6.0, mode="reflect")
        f = (f - f.min()) / max(f.max() - f.min(), 1e-30)
        a = padded_zeros(nx, ny, nz, sy=sy)
        interior(a, nx, ny, nz)[...] = (lo + (hi - lo) * f).astype(np.float32)
        out.append(a)
    return out[0], out[1]
