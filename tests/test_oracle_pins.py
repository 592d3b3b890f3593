"""Pins of the FP64 oracle to facts fixed outside of it.

Each test ties an oracle routine to something other than the oracle itself: the
point counts that Table I prints, the closed-form central-difference weights and
their moment conditions, exact derivatives of polynomials, the measured order of
accuracy, library correlations (scipy.ndimage) that compute the same definition,
the discrete energy that leapfrog conserves, reciprocity of the Green's function,
the dot-product identity of forward and adjoint and finite differences of the
misfit.  All of them run on the CPU.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import ndimage

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- coefficients
def fornberg_second_derivative(r):
    """Closed form of the symmetric 2r-th order weights of d2/dx2 at unit spacing."""
    c0 = -2 * sum(Fraction(1, k * k) for k in range(1, r + 1))
    ck = [Fraction(2 * (-1) ** (k + 1) * math.factorial(r) ** 2,
                   k * k * math.factorial(r - k) * math.factorial(r + k)) for k in range(1, r + 1)]
    return [c0] + ck


def moment_solve(r):
    """Solve sum_k c_k k^(2j) = 2 [j == 1], j = 0..r, for symmetric weights (exact)."""
    n = r + 1
    A = [[Fraction(1 if k == 0 else 0) if j == 0 else Fraction(0) for k in range(n)] for j in range(n)]
    for j in range(n):
        for k in range(n):
            A[j][k] = Fraction(1) if (j == 0 and k == 0) else (
                Fraction(0) if k == 0 else Fraction(2 * k ** (2 * j)))
    b = [Fraction(2 if j == 1 else 0) for j in range(n)]
    for col in range(n):  # Gauss-Jordan in rationals
        piv = next(i for i in range(col, n) if A[i][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        b[col], b[piv] = b[piv], b[col]
        for i in range(n):
            if i != col and A[i][col] != 0:
                f = A[i][col] / A[col][col]
                A[i] = [a - f * c for a, c in zip(A[i], A[col])]
                b[i] -= f * b[col]
    return [b[i] / A[i][i] for i in range(n)]


def test_laplacian_weights_closed_form():
    assert fornberg_second_derivative(4) == list(synth.LAPLACIAN_R4)
    assert fornberg_second_derivative(2) == list(synth.LAPLACIAN_R2)
    assert moment_solve(4) == list(synth.LAPLACIAN_R4)
    for r in (1, 2, 3):
        assert fornberg_second_derivative(r) == moment_solve(r)
    assert fornberg_second_derivative(1) == [Fraction(-2), Fraction(1)]


def exact_weights(r):
    half = [float(f) for f in fornberg_second_derivative(r)]
    w = np.array(half[:0:-1] + half)
    return np.stack([w, w, w])


# ---------------------------------------------------------- shapes (Table I)
def read_table1():
    rows = []
    with open(os.path.join(GOLDEN, "table1_points.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, dims, shape, r, pts = line.split()
            rows.append((name, int(dims), shape, int(r), int(pts)))
    return rows


@pytest.mark.parametrize("row", [r for r in read_table1() if r[1] == 3], ids=lambda r: r[0])
def test_point_counts_match_table1(row):
    """The impulse response of the oracle touches exactly the Table I point count."""
    _, _, shape, r, pts = row
    n = 2 * r + 3
    rng = np.random.default_rng(5)
    acc = np.zeros((n, n, n))
    for trial in range(2):  # random non-zero coefficients: no accidental cancellation
        if shape == "star":
            c = rng.uniform(0.5, 1.5, (3, 2 * r + 1))
        else:
            c = rng.uniform(0.5, 1.5, (2 * r + 1,) * 3)
        delta = synth.padded_zeros(n, n, n, dtype=np.float64)
        synth.interior(delta, n, n, n)[n // 2, n // 2, n // 2] = 1.0
        f = oracle.star if shape == "star" else oracle.box
        out = f(delta, n, n, n, r, c)
        acc += np.abs(synth.interior(out, n, n, n))
    assert int(np.count_nonzero(acc)) == pts


@pytest.mark.parametrize("row", [r for r in read_table1() if r[1] == 2], ids=lambda r: r[0])
def test_point_counts_match_table1_2d(row):
    """2-D kernels act on each plane of a stack: the impulse response stays in the
    impulse's plane and touches exactly the Table I point count there."""
    _, _, shape, r, pts = row
    n = 2 * r + 3
    rng = np.random.default_rng(6)
    acc = np.zeros((n, n, n))
    for trial in range(2):
        if shape == "star":
            c = rng.uniform(0.5, 1.5, (2, 2 * r + 1))
        else:
            c = rng.uniform(0.5, 1.5, (2 * r + 1,) * 2)
        delta = synth.padded_zeros(n, n, n, dtype=np.float64)
        synth.interior(delta, n, n, n)[n // 2, n // 2, n // 2] = 1.0
        f = oracle.star2d if shape == "star" else oracle.box2d
        acc += np.abs(synth.interior(f(delta, n, n, n, r, c), n, n, n))
    assert int(np.count_nonzero(acc)) == pts
    assert int(np.count_nonzero(acc[n // 2])) == pts


# ------------------------------------------------------------- star oracle
def poly_field(deg_max, seed, n=12, halo=4, pure_x_degree=None):
    """Random polynomial of total degree <= deg_max on the padded grid incl. halo,
    with its exact Laplacian (grid units).  Coordinates scaled to ~[-1, 1]."""
    rng = np.random.default_rng(seed)
    N = n + 2 * halo
    s = n / 2.0
    idx = (np.arange(N) - halo - (n - 1) / 2.0) / s
    Z, Y, X = np.meshgrid(idx, idx, idx, indexing="ij")
    u = np.zeros((N, N, N))
    lap = np.zeros((N, N, N))
    terms = []
    if pure_x_degree is not None:
        terms = [(pure_x_degree, 0, 0, 1.0)]
    else:
        for i in range(deg_max + 1):
            for j in range(deg_max + 1 - i):
                for k in range(deg_max + 1 - i - j):
                    terms.append((i, j, k, rng.uniform(-1, 1)))
    for i, j, k, a in terms:
        u += a * X ** i * Y ** j * Z ** k
        if i >= 2:
            lap += a * i * (i - 1) * X ** (i - 2) * Y ** j * Z ** k / s ** 2
        if j >= 2:
            lap += a * j * (j - 1) * X ** i * Y ** (j - 2) * Z ** k / s ** 2
        if k >= 2:
            lap += a * k * (k - 1) * X ** i * Y ** j * Z ** (k - 2) / s ** 2
    return u, lap


def test_star_exact_on_degree_9_polynomials():
    n = 12
    u, lap = poly_field(9, seed=1, n=n)
    out = oracle.star(u, n, n, n, 4, exact_weights(4))
    got = synth.interior(out, n, n, n)
    want = synth.interior(lap, n, n, n)
    assert np.max(np.abs(got - want)) <= 1e-10 * max(1.0, np.max(np.abs(want)))


def test_star_not_exact_at_degree_10():
    n = 12
    u, lap = poly_field(10, seed=0, n=n, pure_x_degree=10)
    out = oracle.star(u, n, n, n, 4, exact_weights(4))
    err = np.max(np.abs(synth.interior(out, n, n, n) - synth.interior(lap, n, n, n)))
    # the first neglected moment: sum_k c_k k^10 / 10! * d^10/dx^10 (X^10) / s^10
    s = n / 2.0
    expect = 2 * 576 / math.factorial(10) * math.factorial(10) / s ** 10
    assert abs(err - expect) < 1e-6 * expect


def test_star_constant_field_is_zero():
    n = 10
    u = np.full((n + 8, n + 8, n + 8), 3.25)
    out = oracle.star(u, n, n, n, 4, exact_weights(4))
    assert np.max(np.abs(synth.interior(out, n, n, n))) < 1e-13
    # zero halo: interior points at least r away from every face still see a constant
    z = synth.padded_zeros(n, n, n, dtype=np.float64)
    synth.interior(z, n, n, n)[...] = 3.25
    out = oracle.star(z, n, n, n, 4, exact_weights(4))
    assert np.max(np.abs(synth.interior(out, n, n, n)[4:-4, 4:-4, 4:-4])) < 1e-13


def sine_error(ppw, n=16):
    """Max relative error of the star on sin(kx)sin(ky)sin(kz) vs -|k|^2 u."""
    k = 2 * np.pi / ppw
    N = n + 8
    idx = np.arange(N) - 4.0
    Z, Y, X = np.meshgrid(idx, idx, idx, indexing="ij")
    u = np.sin(k * X + 0.3) * np.sin(k * Y + 0.7) * np.sin(k * Z + 1.1)
    out = oracle.star(u, n, n, n, 4, exact_weights(4))
    got = synth.interior(out, n, n, n)
    want = -3 * k * k * synth.interior(u, n, n, n)
    return np.max(np.abs(got - want)) / np.max(np.abs(want))


def test_star_convergence_order_8():
    ppws = np.array([16.0, 24.0, 32.0, 48.0])
    errs = np.array([sine_error(p) for p in ppws])
    slope = np.polyfit(np.log(ppws), np.log(errs), 1)[0]
    assert abs(slope + 8.0) < 0.3


def test_star_truncation_constant():
    """1-D symbol: c0 + 2 sum c_k cos(k t) = -t^2 + t^10/3150 + O(t^12).

    R(t) = (symbol + t^2) / t^10 is measured on a sine along x and extrapolated
    to t -> 0 by a quadratic fit in t^2 (the O(t^12), O(t^14) terms)."""
    n = 8
    ts, rs = [], []
    for ppw in (10.0, 12.0, 16.0, 20.0):
        t = 2 * np.pi / ppw
        N = n + 8
        idx = np.arange(N) - 4.0
        u = np.broadcast_to(np.sin(t * idx + 0.4)[None, None, :], (N, N, N)).copy()
        out = oracle.star(u, n, n, n, 4, exact_weights(4))
        got = synth.interior(out, n, n, n)
        ui = synth.interior(u, n, n, n)
        mask = np.abs(ui) > 0.5
        ts.append(t * t)
        rs.append(np.mean((got + t * t * ui)[mask] / ui[mask]) / t ** 10)
    fit = np.polyfit(ts, rs, 2)
    assert abs(fit[-1] * 3150 - 1) < 1e-4


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_star_matches_scipy_correlate1d(r):
    nx, ny, nz = 11, 9, 7
    rng = np.random.default_rng(10 + r)
    a = synth.padded_zeros(nx, ny, nz, dtype=np.float64)
    a[...] = rng.uniform(-1, 1, a.shape)  # non-zero halo is read as stored
    c = rng.uniform(-1, 1, (3, 2 * r + 1))
    out = oracle.star(a, nx, ny, nz, r, c)
    full = a[:, :, :nx + 8]
    ref = (ndimage.correlate1d(full, c[0], axis=0, mode="constant")
           + ndimage.correlate1d(full, c[1], axis=1, mode="constant")
           + ndimage.correlate1d(full, c[2], axis=2, mode="constant"))
    np.testing.assert_allclose(synth.interior(out, nx, ny, nz),
                               ref[4:4 + nz, 4:4 + ny, 4:4 + nx], rtol=0, atol=1e-13)


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_star2d_matches_scipy_correlate1d(r):
    nx, ny, nz = 13, 10, 3
    rng = np.random.default_rng(30 + r)
    a = synth.padded_zeros(nx, ny, nz, dtype=np.float64)
    a[...] = rng.uniform(-1, 1, a.shape)  # non-zero halo, also in z: never read
    c = rng.uniform(-1, 1, (2, 2 * r + 1))
    out = oracle.star2d(a, nx, ny, nz, r, c)
    full = a[:, :, :nx + 8]
    ref = (ndimage.correlate1d(full, c[0], axis=1, mode="constant")
           + ndimage.correlate1d(full, c[1], axis=2, mode="constant"))
    np.testing.assert_allclose(synth.interior(out, nx, ny, nz),
                               ref[4:4 + nz, 4:4 + ny, 4:4 + nx], rtol=0, atol=1e-13)
    # the same as the (pinned) 3-D star whose z weights are zero
    c3 = np.stack([np.zeros(2 * r + 1), c[0], c[1]])
    np.testing.assert_allclose(out, oracle.star(a, nx, ny, nz, r, c3), rtol=0, atol=1e-14)


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_box2d_matches_scipy_correlate(r):
    nx, ny, nz = 12, 9, 3
    rng = np.random.default_rng(40 + r)
    a = synth.padded_zeros(nx, ny, nz, dtype=np.float64)
    a[...] = rng.uniform(-1, 1, a.shape)
    c = rng.uniform(-1, 1, (2 * r + 1,) * 2)  # no symmetry: a transposed axis fails
    out = oracle.box2d(a, nx, ny, nz, r, c)
    ref = ndimage.correlate(a[:, :, :nx + 8], c[None], mode="constant")
    np.testing.assert_allclose(synth.interior(out, nx, ny, nz),
                               ref[4:4 + nz, 4:4 + ny, 4:4 + nx], rtol=0, atol=1e-12)
    idx = np.array([[0, 0, 0], [nz - 1, ny - 1, nx - 1], [1, 4, 7]])
    np.testing.assert_allclose(oracle.box2d_at(a, nx, ny, nz, r, c, idx),
                               synth.interior(out, nx, ny, nz)[idx[:, 0], idx[:, 1], idx[:, 2]],
                               rtol=0, atol=0)
    np.testing.assert_allclose(oracle.star2d_at(a, nx, ny, nz, r, c[:2], idx),
                               synth.interior(oracle.star2d(a, nx, ny, nz, r, c[:2]), nx, ny,
                                              nz)[idx[:, 0], idx[:, 1], idx[:, 2]], rtol=0, atol=0)


# -------------------------------------------------------------- box oracle
@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_box_matches_scipy_correlate(r):
    nx, ny, nz = 10, 7, 6
    rng = np.random.default_rng(20 + r)
    a = synth.padded_zeros(nx, ny, nz, dtype=np.float64)
    a[...] = rng.uniform(-1, 1, a.shape)
    c = rng.uniform(-1, 1, (2 * r + 1,) * 3)  # no symmetry: a transposed axis fails
    out = oracle.box(a, nx, ny, nz, r, c)
    ref = ndimage.correlate(a[:, :, :nx + 8], c, mode="constant")
    np.testing.assert_allclose(synth.interior(out, nx, ny, nz),
                               ref[4:4 + nz, 4:4 + ny, 4:4 + nx], rtol=0, atol=1e-12)


def test_box_dense_operator_8cubed():
    """Brute force: the dense 512x512 zero-halo operator built from numpy shifts."""
    n, r = 8, 2
    rng = np.random.default_rng(3)
    c = rng.uniform(-1, 1, (5, 5, 5))
    M = np.zeros((n ** 3, n ** 3))
    for q in range(n ** 3):  # column q = response to a unit impulse at q
        e = np.zeros((n, n, n))
        e.flat[q] = 1.0
        pad = np.pad(e, r)
        col = np.zeros((n, n, n))
        for dz in range(-r, r + 1):
            for dy in range(-r, r + 1):
                for dx in range(-r, r + 1):
                    col += c[dz + r, dy + r, dx + r] * pad[r + dz:r + dz + n, r + dy:r + dy + n,
                                                          r + dx:r + dx + n]
        M[:, q] = col.ravel()
    x = rng.uniform(-1, 1, (n, n, n))
    a = synth.padded_zeros(n, n, n, dtype=np.float64)
    synth.interior(a, n, n, n)[...] = x
    out = oracle.box(a, n, n, n, r, c)
    np.testing.assert_allclose(synth.interior(out, n, n, n).ravel(), M @ x.ravel(),
                               rtol=0, atol=1e-13)


def test_box_separable_and_r1_star():
    n = 9
    rng = np.random.default_rng(4)
    a = synth.padded_zeros(n, n, n, dtype=np.float64)
    synth.interior(a, n, n, n)[...] = rng.uniform(-1, 1, (n, n, n))
    az, ay, ax = (rng.uniform(-1, 1, 9) for _ in range(3))
    c = az[:, None, None] * ay[None, :, None] * ax[None, None, :]
    out = oracle.box(a, n, n, n, 4, c)
    x = a[:, :, :n + 8]
    ref = ndimage.correlate1d(ndimage.correlate1d(ndimage.correlate1d(
        x, az, axis=0, mode="constant"), ay, axis=1, mode="constant"), ax, axis=2, mode="constant")
    np.testing.assert_allclose(synth.interior(out, n, n, n), ref[4:-4, 4:-4, 4:-4], atol=1e-13)
    # r = 1 box holding the 7-point Laplacian pattern equals the r = 1 star
    c7 = np.zeros((3, 3, 3))
    c7[1, 1, 1] = -6
    for d in ((0, 1, 1), (2, 1, 1), (1, 0, 1), (1, 2, 1), (1, 1, 0), (1, 1, 2)):
        c7[d] = 1
    s = np.array([[1, -2, 1]] * 3, dtype=np.float64)
    np.testing.assert_allclose(oracle.box(a, n, n, n, 1, c7), oracle.star(a, n, n, n, 1, s),
                               atol=1e-14)


@pytest.mark.parametrize("r", [1, 2, 3, 4])
def test_sampled_definitions_match_full_grid_sweeps(r):
    """The point-list evaluators (star_at, box_at and the 2-D ones) return what the
    full-grid sweeps (pinned above to scipy, the dense operator and exact
    derivatives) return at the same points: non-symmetric weights, a non-zero halo,
    points on every face and corner of the interior as well as random ones."""
    nx, ny, nz = 13, 9, 11
    rng = np.random.default_rng(40 + r)
    a = synth.padded_zeros(nx, ny, nz, dtype=np.float64)
    a[...] = rng.uniform(-1, 1, a.shape)
    w = 2 * r + 1
    pts = [(z, y, x) for z in (0, nz - 1) for y in (0, ny - 1) for x in (0, nx - 1)]
    pts += [tuple(int(v) for v in rng.integers(0, (nz, ny, nx))) for _ in range(200)]
    pts = np.array(pts)
    I = lambda f: synth.interior(f, nx, ny, nz)[pts[:, 0], pts[:, 1], pts[:, 2]]
    cases = [(oracle.star_at, oracle.star, (3, w)), (oracle.box_at, oracle.box, (w, w, w)),
             (oracle.star2d_at, oracle.star2d, (2, w)), (oracle.box2d_at, oracle.box2d, (w, w))]
    for at, full, cshape in cases:
        c = rng.uniform(-1, 1, cshape)
        want = I(full(a, nx, ny, nz, r, c))
        got = at(a, nx, ny, nz, r, c, pts)
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-14 * np.abs(want).max())


# ------------------------------------------------------------------ sponge
def test_sponge_profile_closed_form():
    g = oracle.sponge_1d(100, 32, 0.015, True, True)
    assert g[0] == pytest.approx(math.exp(-(0.015 * 32) ** 2), rel=1e-15)
    assert g[99] == pytest.approx(math.exp(-(0.015 * 32) ** 2), rel=1e-15)
    assert g[31] == pytest.approx(math.exp(-0.015 ** 2), rel=1e-15)
    assert np.all(g[32:68] == 1.0)
    assert np.all(np.diff(g[:33]) > 0)
    g1 = oracle.sponge_1d(100, 32, 0.015, False, True)
    assert np.all(g1[:68] == 1.0) and g1[99] == g[99]


# -------------------------------------------------------------- wave oracle
def wave_problem(n, c2_value, seed, nt, lap=None, src=None, f=None, faces=0, width=0,
                 alpha=0.0, rand_c2=True):
    rng = np.random.default_rng(seed)
    c2 = synth.padded_zeros(n, n, n, dtype=np.float64)
    if rand_c2:
        synth.interior(c2, n, n, n)[...] = c2_value * rng.uniform(0.5, 1.0, (n, n, n))
    else:
        synth.interior(c2, n, n, n)[...] = c2_value
    lap = [float(v) for v in synth.LAPLACIAN_R4] if lap is None else lap
    src = (n // 2, n // 2, n // 2) if src is None else src
    f = np.zeros(nt) if f is None else f
    return oracle.Wave(n, n, n, c2, lap, src, f, nt, width, alpha, faces)


def energy(w, up, u, n):
    """E^{n+1/2} = sum (u^{n+1}-u^n)^2 / C2 - <u^{n+1}, S u^n>, interior sums."""
    lapc = np.array([w.lap[abs(k)] for k in range(-4, 5)])
    Su = oracle.star(up, n, n, n, 4, np.stack([lapc] * 3))
    I = lambda a: synth.interior(a, n, n, n)
    return np.sum((I(u) - I(up)) ** 2 / I(w.c2)) - np.sum(I(u) * I(Su))


def test_leapfrog_conserves_discrete_energy():
    n, nt = 16, 300
    w = wave_problem(n, 0.16, seed=1, nt=nt)
    u0 = synth.smooth_random_grid(2, n, n, n).astype(np.float64)
    u1 = synth.smooth_random_grid(3, n, n, n).astype(np.float64)
    e0 = energy(w, u0, u1, n)
    res = w.forward(u0, u1)
    a, b = res["last"]
    e1 = energy(w, a, b, n)
    assert e0 > 0
    assert abs(e1 - e0) <= 1e-12 * e0


def test_cfl_limit():
    """Stable just below the 8th-order 3-D limit 2/sqrt(3*6.5016) = 0.4529, unstable above."""
    n, nt = 12, 1500
    checker = synth.padded_zeros(n, n, n, dtype=np.float64)
    idx = np.indices((n, n, n)).sum(axis=0)
    synth.interior(checker, n, n, n)[...] = (-1.0) ** idx
    out = {}
    for courant in (0.44, 0.47):
        w = wave_problem(n, courant ** 2, seed=0, nt=nt, rand_c2=False)
        res = w.forward(checker, checker * 0.999)
        out[courant] = np.max(np.abs(res["last"][1]))
    assert out[0.44] < 10.0
    assert out[0.47] > 1e3


def test_reciprocity():
    n, nt = 14, 120
    rng = np.random.default_rng(7)
    f = rng.standard_normal(nt)
    s1, s2 = (4, 5, 6), (9, 8, 7)
    w1 = wave_problem(n, 0.12, seed=9, nt=nt, src=s1, f=f)
    w2 = wave_problem(n, 0.12, seed=9, nt=nt, src=s2, f=f)
    z = np.zeros(w1.shape)
    st1 = w1.forward(z, z, keep_states=True)["states"]
    st2 = w2.forward(z, z, keep_states=True)["states"]
    at = lambda p: (p[0] + 4, p[1] + 4, p[2] + 4)
    # C2(s) u_s(r) = C2(r) u_r(s): D u'' = S u + f delta_s / C2(s) with symmetric D, S
    lhs = w1.c2[at(s2)] * st2[:, at(s1)[0], at(s1)[1], at(s1)[2]]
    rhs = w1.c2[at(s1)] * st1[:, at(s2)[0], at(s2)[1], at(s2)[2]]
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * np.max(np.abs(lhs))
    assert np.max(np.abs(lhs)) > 0


def sponge_problem(n, nt, seed, f=None):
    return wave_problem(n, 0.15, seed=seed, nt=nt, src=(2, n // 2, n // 2), f=f,
                        faces=synth.SPONGE_LATERAL_AND_BOTTOM, width=4, alpha=0.1)


def test_adjoint_dot_product_fp64():
    n, nt = 12, 60
    rng = np.random.default_rng(11)
    f = rng.standard_normal(nt)
    w = sponge_problem(n, nt, seed=12, f=f)
    u0 = synth.smooth_random_grid(13, n, n, n, sigma=1.5).astype(np.float64)
    u1 = synth.smooth_random_grid(14, n, n, n, sigma=1.5).astype(np.float64)
    res = w.forward(u0, u1, keep_states=True)
    y = rng.standard_normal((nt, n, n))
    _, l0, l1, gs = w.adjoint(res["states"], y)
    lhs = np.sum(res["traces"] * y)
    I = lambda a: synth.interior(a, n, n, n)
    rhs = np.sum(I(u0) * I(l0)) + np.sum(I(u1) * I(l1)) + np.sum(f * gs)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_adjoint_single_step_matches_full_run():
    """The step routine reproduces the full adjoint run's recursion."""
    n, nt = 10, 12
    rng = np.random.default_rng(15)
    w = sponge_problem(n, nt, seed=16)
    u0 = synth.smooth_random_grid(17, n, n, n).astype(np.float64)
    u1 = synth.smooth_random_grid(18, n, n, n).astype(np.float64)
    st = w.forward(u0, u1, keep_states=True)["states"]
    y = rng.standard_normal((nt, n, n))
    g_full, l0_full, l1_full, _ = w.adjoint(st, y)
    l2, l1 = w.zeros(), w.zeros()
    g = w.zeros()
    for k in range(nt - 1, -1, -1):
        l0 = w.adjoint_step(k, l2, l1, y[k], st[k] if k >= 1 else None, g)
        l2, l1 = l1, l0
        if k == 1:
            lam1 = l0.copy()
    np.testing.assert_allclose(l1, l0_full, rtol=0, atol=1e-12 * np.abs(l0_full).max())
    np.testing.assert_allclose(lam1, l1_full, rtol=0, atol=1e-12 * np.abs(l1_full).max())
    np.testing.assert_allclose(g, g_full, rtol=0, atol=1e-12 * np.abs(g_full).max())


def test_gradient_finite_differences_fp64():
    n, nt = 12, 80
    rng = np.random.default_rng(21)
    f = np.sin(np.arange(nt) * 0.3) * np.exp(-((np.arange(nt) - 15) / 6.0) ** 2)
    w = sponge_problem(n, nt, seed=22, f=f)
    z = np.zeros(w.shape)
    d_obs = rng.standard_normal((nt, n, n)) * 1e-3
    res = w.forward(z, z, keep_states=True)
    resid = res["traces"] - d_obs
    g, _, _, _ = w.adjoint(res["states"], resid)

    def J(c2):
        ww = oracle.Wave(n, n, n, c2, w.lap, (2, n // 2, n // 2), f, nt, 4, 0.1,
                         synth.SPONGE_LATERAL_AND_BOTTOM)
        d = ww.forward(z, z)["traces"]
        return 0.5 * np.sum((d - d_obs) ** 2)

    pts = [tuple(rng.integers(0, n, 3)) for _ in range(16)]
    for p in pts:
        i = (p[0] + 4, p[1] + 4, p[2] + 4)
        eps = 1e-4 * w.c2[i]
        cp, cm = w.c2.copy(), w.c2.copy()
        cp[i] += eps
        cm[i] -= eps
        fd = (J(cp) - J(cm)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-6 * np.abs(g).max())


def test_forward_step_matches_run_and_records_traces():
    n, nt = 10, 6
    rng = np.random.default_rng(30)
    f = rng.standard_normal(nt)
    w = sponge_problem(n, nt, seed=31, f=f)
    u0 = synth.smooth_random_grid(32, n, n, n).astype(np.float64)
    u1 = synth.smooth_random_grid(33, n, n, n).astype(np.float64)
    res = w.forward(u0, u1, keep_states=True, image=True)
    a, b = u0, u1
    img = w.zeros()
    for k in range(1, nt):
        c, tr = w.step(k, a, b, image=img)
        np.testing.assert_array_equal(tr, res["traces"][k])
        np.testing.assert_array_equal(c, res["states"][k + 1])
        a, b = b, c
    np.testing.assert_array_equal(res["traces"][0], synth.interior(u0, n, n, n)[0])
    np.testing.assert_allclose(img, res["image"], rtol=1e-15)
    # the source enters with weight 1 at its cell when G = 1 there
    w0 = sponge_problem(n, nt, seed=31, f=np.zeros(nt))
    c0, _ = w0.step(3, u0, u1)
    c1, _ = w.step(3, u0, u1)
    d = c1 - c0
    assert d[2 + 4, n // 2 + 4, n // 2 + 4] == pytest.approx(f[3], rel=1e-12)
    d[2 + 4, n // 2 + 4, n // 2 + 4] = 0
    assert np.max(np.abs(d)) == 0


def test_image_is_sum_of_squared_new_levels():
    """The forward run's image is sum over the steps n = 1..nt-1 of (u^{n+1})^2 (the
    level each step produces, not the level it reads), summed here in numpy from the
    stored states; the halo stays zero."""
    n, nt = 10, 9
    rng = np.random.default_rng(34)
    w = sponge_problem(n, nt, seed=35, f=rng.standard_normal(nt))
    u0 = synth.smooth_random_grid(36, n, n, n).astype(np.float64)
    u1 = synth.smooth_random_grid(37, n, n, n).astype(np.float64)
    res = w.forward(u0, u1, keep_states=True, image=True)
    st = res["states"]             # st[k] = u^k, k = 0..nt
    want = np.sum(st[2:nt + 1] ** 2, axis=0)
    H = 4
    np.testing.assert_allclose(synth.interior(res["image"], n, n, n), synth.interior(want, n, n, n),
                               rtol=1e-14, atol=0)
    mask = np.ones(w.shape, dtype=bool)
    mask[H:H + n, H:H + n, H:H + n] = False
    assert not np.any(res["image"][mask])
    # the levels read (u^1 .. u^{nt-1}) give a different sum
    wrong = np.sum(st[1:nt] ** 2, axis=0)
    assert np.max(np.abs(synth.interior(wrong - want, n, n, n))) > 1e-3 * np.max(want)


# ------------------------------------------------------------ VTI oracle
def test_vti_reduces_to_acoustic():
    """epsilon = delta = 0 and equal fields: both VTI fields follow the acoustic step."""
    n, nt = 14, 40
    rng = np.random.default_rng(50)
    f = rng.standard_normal(nt)
    w = sponge_problem(n, nt, seed=51, f=f)
    u0 = synth.smooth_random_grid(52, n, n, n).astype(np.float64)
    u1 = synth.smooth_random_grid(53, n, n, n).astype(np.float64)
    ones = np.ones_like(u0)
    ac = w.forward(u0, u1)
    vt = w.vti_forward(ones, ones, u0, u1, u0, u1)
    scale = np.abs(ac["last"]).max()
    assert np.max(np.abs(vt["last"][0] - ac["last"][0])) <= 1e-12 * scale
    assert np.max(np.abs(vt["last"][1] - ac["last"][1])) <= 1e-12 * scale
    assert np.max(np.abs(vt["last"][3] - ac["last"][1])) <= 1e-12 * scale
    np.testing.assert_allclose(vt["traces"], ac["traces"], rtol=0,
                               atol=1e-12 * np.abs(ac["traces"]).max())


def test_vti_sine_mode_recurrence():
    """Radius-1 weights with a zero halo have sine eigenvectors, so a mode H = alpha Phi,
    V = beta Phi evolves by the 2x2 recurrence
    [alpha, beta]^{n+1} = 2 [.]^n - [.]^{n-1} - C2 M [.]^n,  M = [[a sxy, b sz], [b sxy, sz]]
    with -sxy, -sz the eigenvalues of Sxx + Syy and Szz; checked against the 3-D oracle."""
    n, nt = 11, 60
    kz, ky, kx = 2, 3, 1
    lam = lambda k: -4.0 * np.sin(np.pi * k / (2 * (n + 1))) ** 2
    sxy, sz = -(lam(kx) + lam(ky)), -lam(kz)
    a_val, b_val, c2_val = 1.3, 1.1, 0.2          # epsilon = 0.15 >= delta = 0.105
    i = np.arange(n)
    phi = lambda k: np.sin(np.pi * k * (i + 1) / (n + 1))
    Phi = phi(kz)[:, None, None] * phi(ky)[None, :, None] * phi(kx)[None, None, :]
    pad = lambda x: np.pad(x, 4)
    c2 = pad(np.full((n, n, n), c2_val))
    w = oracle.Wave(n, n, n, c2, [-2.0, 1.0], (0, 0, 0), np.zeros(nt), nt)
    al = [1.0, 0.9]
    be = [-0.5, -0.45]
    res = w.vti_forward(pad(np.full((n, n, n), a_val)), pad(np.full((n, n, n), b_val)),
                        pad(al[0] * Phi), pad(al[1] * Phi), pad(be[0] * Phi), pad(be[1] * Phi))
    M = np.array([[a_val * sxy, b_val * sz], [b_val * sxy, sz]])
    s_prev, s_cur = np.array([al[0], be[0]]), np.array([al[1], be[1]])
    for _ in range(1, nt):
        s_prev, s_cur = s_cur, 2 * s_cur - s_prev - c2_val * M @ s_cur
    I = lambda x: synth.interior(x, n, n, n)
    np.testing.assert_allclose(I(res["last"][1]), s_cur[0] * Phi, rtol=0, atol=1e-12)
    np.testing.assert_allclose(I(res["last"][3]), s_cur[1] * Phi, rtol=0, atol=1e-12)
    np.testing.assert_allclose(I(res["last"][0]), s_prev[0] * Phi, rtol=0, atol=1e-12)
    assert abs(s_cur[0]) > 0.05 and abs(s_cur[1]) > 0.05


def test_vti_step_matches_forward():
    n, nt = 9, 5
    rng = np.random.default_rng(60)
    f = rng.standard_normal(nt)
    w = sponge_problem(n, nt, seed=61, f=f)
    fields = [synth.smooth_random_grid(62 + k, n, n, n).astype(np.float64) for k in range(4)]
    a = synth.padded_zeros(n, n, n, dtype=np.float64)
    b = synth.padded_zeros(n, n, n, dtype=np.float64)
    synth.interior(a, n, n, n)[...] = 1 + 2 * rng.uniform(0, 0.2, (n, n, n))
    synth.interior(b, n, n, n)[...] = np.sqrt(1 + 2 * rng.uniform(0, 0.1, (n, n, n)))
    res = w.vti_forward(a, b, *fields)
    hp, hc, vp, vc = fields[0], fields[1], fields[2], fields[3]
    for k in range(1, nt):
        hn, vn, tr = w.vti_step(k, a, b, hp, hc, vp, vc)
        np.testing.assert_array_equal(tr, res["traces"][k])
        hp, hc, vp, vc = hc, hn, vc, vn
    np.testing.assert_array_equal(hc, res["last"][1])
    np.testing.assert_array_equal(vc, res["last"][3])


# ------------------------------------------------------------------- TTI oracle
D1 = [float(v) for v in synth.FIRST_DERIV_R4]


def first_derivative_closed_form(r):
    """Central first-derivative weights d_k, k = 1..r, of order 2r:
    d_k = (-1)^(k+1) (r!)^2 / (k (r-k)! (r+k)!)."""
    f = math.factorial
    return [Fraction((-1) ** (k + 1) * f(r) ** 2, k * f(r - k) * f(r + k)) for k in range(1, r + 1)]


def test_first_derivative_weights():
    d = first_derivative_closed_form(4)
    assert d == list(synth.FIRST_DERIV_R4)
    # moment conditions: sum_k d_k 2 k^(2j+1) = [j == 0], j = 0..r-1
    for j in range(4):
        assert sum(dk * 2 * Fraction(k + 1) ** (2 * j + 1) for k, dk in enumerate(d)) == (j == 0)
    assert first_derivative_closed_form(1) == [Fraction(1, 2)]


def tti_poly(deg, seed, n):
    """Random polynomial of total degree <= deg on the padded n^3 cube and its exact
    Hessian (grid units)."""
    rng = np.random.default_rng(seed)
    N = n + 8
    s = n / 2.0
    idx = (np.arange(N) - 4 - (n - 1) / 2.0) / s
    Z, Y, X = np.meshgrid(idx, idx, idx, indexing="ij")
    u = np.zeros((N, N, N))
    H = {k: np.zeros((N, N, N)) for k in ("xx", "yy", "zz", "xy", "yz", "xz")}
    P = lambda b, e: b ** e if e >= 0 else 0.0 * b
    for i in range(deg + 1):
        for j in range(deg + 1 - i):
            for k in range(deg + 1 - i - j):
                a = rng.uniform(-1, 1)
                u += a * X ** i * Y ** j * Z ** k
                H["xx"] += a * i * (i - 1) * P(X, i - 2) * Y ** j * Z ** k / s ** 2
                H["yy"] += a * j * (j - 1) * X ** i * P(Y, j - 2) * Z ** k / s ** 2
                H["zz"] += a * k * (k - 1) * X ** i * Y ** j * P(Z, k - 2) / s ** 2
                H["xy"] += a * i * j * P(X, i - 1) * P(Y, j - 1) * Z ** k / s ** 2
                H["yz"] += a * j * k * X ** i * P(Y, j - 1) * P(Z, k - 1) / s ** 2
                H["xz"] += a * i * k * P(X, i - 1) * Y ** j * P(Z, k - 1) / s ** 2
    return u, H


def tti_wave(n, nt=4, c2=None, lap=None, src=(0, 0, 0), f=None, W=0, alpha=0.0, faces=0):
    c2 = synth.padded_zeros(n, n, n, dtype=np.float64) if c2 is None else c2
    lap = [float(v) for v in synth.LAPLACIAN_R4] if lap is None else lap
    f = np.zeros(nt) if f is None else f
    return oracle.Wave(n, n, n, c2, lap, src, f, nt, W, alpha, faces)


def test_tti_operators_exact_on_degree_8_polynomials():
    """H1 = (n . grad)^2 with n = (sin t cos p, sin t sin p, cos t) at every cell, and
    L = Laplacian, exactly (to rounding) for polynomials of degree <= 8: the mixed
    derivatives are products of 8th-order first-derivative stencils."""
    n = 12
    u, H = tti_poly(8, seed=70, n=n)
    rng = np.random.default_rng(71)
    th = rng.uniform(0, np.pi, u.shape)
    ph = rng.uniform(0, 2 * np.pi, u.shape)
    w = tti_wave(n)
    t = w.tti(np.zeros_like(u), np.zeros_like(u), th, ph, 0.0, 1.0, D1)
    lf, h1 = w.tti_operators(t, u)
    nx_, ny_, nz_ = np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)
    want = (nx_ ** 2 * H["xx"] + ny_ ** 2 * H["yy"] + nz_ ** 2 * H["zz"] + 2 * nx_ * ny_ * H["xy"]
            + 2 * ny_ * nz_ * H["yz"] + 2 * nx_ * nz_ * H["xz"])
    I = lambda a: synth.interior(a, n, n, n)
    scale = np.max(np.abs(I(want)))
    assert np.max(np.abs(I(h1) - I(want))) <= 1e-9 * scale
    lap = H["xx"] + H["yy"] + H["zz"]
    assert np.max(np.abs(I(lf) - I(lap))) <= 1e-9 * np.max(np.abs(I(lap)))


def test_tti_mixed_derivative_not_exact_at_degree_9():
    n = 12
    N = n + 8
    s = n / 2.0
    idx = (np.arange(N) - 4 - (n - 1) / 2.0) / s
    Z, Y, X = np.meshgrid(idx, idx, idx, indexing="ij")
    u = X ** 9 * Z          # d/dx of x^9 is where the 8th-order stencil first errs
    want = 9 * X ** 8 / s ** 2
    th = np.full(u.shape, np.pi / 4)
    ph = np.zeros(u.shape)  # n = (1, 0, 1)/sqrt 2: H1 = (Dxx + Dzz)/2 + Dxz
    w = tti_wave(n)
    t = w.tti(np.zeros_like(u), np.zeros_like(u), th, ph, 0.0, 1.0, D1)
    _, h1 = w.tti_operators(t, u)
    exact = 0.5 * 72 * X ** 7 * Z / s ** 2 + want
    err = np.max(np.abs(synth.interior(h1 - exact, n, n, n)))
    assert err > 1e-6 * np.max(np.abs(synth.interior(exact, n, n, n)))


def tti_medium(n, seed, const_delta=None):
    rng = np.random.default_rng(seed)
    eps = synth.padded_zeros(n, n, n, dtype=np.float64)
    delta = synth.padded_zeros(n, n, n, dtype=np.float64)
    synth.interior(eps, n, n, n)[...] = rng.uniform(0.1, 0.3, (n, n, n))
    synth.interior(delta, n, n, n)[...] = (const_delta if const_delta is not None
                                            else rng.uniform(0.0, 0.1, (n, n, n)))
    return eps, delta


def test_tti_zero_tilt_reduces_to_vti():
    """theta = 0, sigma = 0, alpha = sqrt(1 + 2 delta): the TTI pair is the VTI pair."""
    n, nt, d0 = 12, 60, 0.08
    rng = np.random.default_rng(72)
    eps, delta = tti_medium(n, 73, const_delta=d0)
    c2 = synth.padded_zeros(n, n, n, dtype=np.float64)
    synth.interior(c2, n, n, n)[...] = rng.uniform(0.05, 0.12, (n, n, n))
    f = rng.standard_normal(nt)
    w = tti_wave(n, nt, c2, src=(3, 6, 5), f=f, W=3, alpha=0.1, faces=synth.SPONGE_LATERAL_AND_BOTTOM)
    zero = np.zeros_like(c2)
    alpha = math.sqrt(1 + 2 * d0)
    t = w.tti(eps, delta, zero, rng.uniform(0, 6, c2.shape), 0.0, alpha, D1)
    fields = [synth.smooth_random_grid(74 + k, n, n, n).astype(np.float64) for k in range(4)]
    tt = w.tti_forward(t, *fields)
    vt = w.vti_forward(1 + 2 * eps, np.sqrt(1 + 2 * delta), *fields)
    scale = np.max(np.abs(vt["last"]))
    assert np.max(np.abs(tt["last"] - vt["last"])) <= 1e-12 * scale
    np.testing.assert_allclose(tt["traces"], vt["traces"], rtol=0,
                               atol=1e-12 * np.max(np.abs(vt["traces"])))


def test_tti_axis_along_x_is_transposed_vti():
    """theta = pi/2, phi = 0 puts the symmetry axis on x: the TTI pair equals the VTI
    pair on the grid with x and z exchanged (no sponge, symmetric source)."""
    n, nt, d0 = 12, 40, 0.05
    rng = np.random.default_rng(75)
    eps, delta = tti_medium(n, 76, const_delta=d0)
    c2 = synth.padded_zeros(n, n, n, dtype=np.float64)
    synth.interior(c2, n, n, n)[...] = rng.uniform(0.05, 0.12, (n, n, n))
    assert c2.shape == (n + 8,) * 3
    T = lambda a: np.ascontiguousarray(np.swapaxes(a, 0, 2))
    f = rng.standard_normal(nt)
    alpha = math.sqrt(1 + 2 * d0)
    fields = [synth.smooth_random_grid(77 + k, n, n, n).astype(np.float64) for k in range(4)]
    w = tti_wave(n, nt, c2, src=(6, 6, 6), f=f)
    t = w.tti(eps, delta, np.full(c2.shape, np.pi / 2), np.zeros(c2.shape), 0.0, alpha, D1)
    tt = w.tti_forward(t, *fields)
    wv = tti_wave(n, nt, T(c2), src=(6, 6, 6), f=f)
    vt = wv.vti_forward(T(1 + 2 * eps), T(np.sqrt(1 + 2 * delta)), *[T(a) for a in fields])
    got = np.stack([T(a) for a in tt["last"]])
    scale = np.max(np.abs(vt["last"]))
    assert np.max(np.abs(got - vt["last"])) <= 1e-11 * scale


@pytest.mark.parametrize("axis", ["z", "x", "y"])
def test_tti_shear_and_alpha_terms_sine_mode(axis):
    """A constant medium whose symmetry axis lies along a grid axis, radius-1 weights
    and a zero halo: H1 is then the second difference along that axis and H2 the sum
    of the other two, and p = a Phi, q = b Phi on a sine eigenvector Phi stays a mode.
    With -s1, -s2 the eigenvalues of H1, H2 on Phi, the printed pair gives
      [a, b]^{n+1} = 2 [a, b]^n - [a, b]^{n-1} - C2 M [a, b]^n,
      M = [[(1+2eps) s2 + sigma s1,          alpha (1 - sigma) s1],
           [(1+2delta - sigma) s2 / alpha,   s1 + sigma s2       ]].
    sigma > 0 and alpha != sqrt(1 + 2 delta) make every term of both equations count:
    a sign flip of a sigma term, H1 and H2 exchanged inside one, or alpha moved from
    the denominator of (1+2delta)/alpha changes M."""
    n, nt = 11, 60
    kz, ky, kx = 2, 3, 1
    lam = lambda k: -4.0 * np.sin(np.pi * k / (2 * (n + 1))) ** 2
    s_axis = {"z": -lam(kz), "y": -lam(ky), "x": -lam(kx)}
    s1 = s_axis[axis]
    s2 = sum(v for a, v in s_axis.items() if a != axis)
    theta, phi = {"z": (0.0, 0.7), "x": (np.pi / 2, 0.0), "y": (np.pi / 2, np.pi / 2)}[axis]
    eps, delta, sigma, alpha, c2_val = 0.2, 0.1, 0.25, 0.6, 0.2
    i = np.arange(n)
    mode = lambda k: np.sin(np.pi * k * (i + 1) / (n + 1))
    Phi = mode(kz)[:, None, None] * mode(ky)[None, :, None] * mode(kx)[None, None, :]
    pad = lambda x: np.pad(x, 4)
    full = lambda v: pad(np.full((n, n, n), v))
    w = oracle.Wave(n, n, n, full(c2_val), [-2.0, 1.0], (0, 0, 0), np.zeros(nt), nt)
    t = w.tti(full(eps), full(delta), full(theta), full(phi), sigma, alpha, [0.5])
    a0, b0 = [1.0, 0.95], [-0.4, -0.42]
    res = w.tti_forward(t, pad(a0[0] * Phi), pad(a0[1] * Phi), pad(b0[0] * Phi), pad(b0[1] * Phi))
    M = np.array([[(1 + 2 * eps) * s2 + sigma * s1, alpha * (1 - sigma) * s1],
                  [(1 + 2 * delta - sigma) * s2 / alpha, s1 + sigma * s2]])
    s_prev, s_cur = np.array([a0[0], b0[0]]), np.array([a0[1], b0[1]])
    for _ in range(1, nt):
        s_prev, s_cur = s_cur, 2 * s_cur - s_prev - c2_val * M @ s_cur
    I = lambda x: synth.interior(x, n, n, n)
    np.testing.assert_allclose(I(res["last"][1]), s_cur[0] * Phi, rtol=0, atol=1e-12)
    np.testing.assert_allclose(I(res["last"][3]), s_cur[1] * Phi, rtol=0, atol=1e-12)
    np.testing.assert_allclose(I(res["last"][0]), s_prev[0] * Phi, rtol=0, atol=1e-12)
    np.testing.assert_allclose(I(res["last"][2]), s_prev[1] * Phi, rtol=0, atol=1e-12)
    assert abs(s_cur[0]) > 0.02 and abs(s_cur[1]) > 0.02


def test_tti_step_matches_forward():
    n, nt = 9, 5
    rng = np.random.default_rng(78)
    eps, delta = tti_medium(n, 79)
    th, ph = synth.tilt_fields(n, n, n, 80)
    c2 = synth.padded_zeros(n, n, n, dtype=np.float64)
    synth.interior(c2, n, n, n)[...] = rng.uniform(0.05, 0.1, (n, n, n))
    w = tti_wave(n, nt, c2, src=(2, 4, 4), f=rng.standard_normal(nt), W=3, alpha=0.1,
                 faces=synth.SPONGE_LATERAL_AND_BOTTOM)
    t = w.tti(eps, delta, th, ph, 0.1, 1.0, D1)
    fields = [synth.smooth_random_grid(81 + k, n, n, n).astype(np.float64) for k in range(4)]
    res = w.tti_forward(t, *fields)
    pp, pc, qp, qc = fields
    for k in range(1, nt):
        pn, qn, tr = w.tti_step(t, k, pp, pc, qp, qc)
        np.testing.assert_array_equal(tr, res["traces"][k])
        pp, pc, qp, qc = pc, pn, qc, qn
    np.testing.assert_array_equal(pc, res["last"][1])
    np.testing.assert_array_equal(qc, res["last"][3])
