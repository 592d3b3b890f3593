"""FP64 CPU oracle (test infrastructure).

Plain double-precision loops over the definitions of the star and box stencil
sweeps (Sec. I problem statement, Sec. II-A high-order case) and of the acoustic
wave step, its exact adjoint and the gradient with respect to C^2 = (v dt/h)^2.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP library:
the C source next to this file is compiled with gcc on its own and loaded
through ctypes.  Inputs arrive as the same FP32 values the GPU gets, promoted to
FP64, so a comparison measures kernel arithmetic and not input rounding.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mms_oracle.c")
_LIB = os.path.join(_HERE, "libmms_oracle.so")
# a prebuilt oracle library to load instead (the sanitizer test builds one with
# -fsanitize=address,undefined and runs the pins against it in a child process)
_LIB_OVERRIDE = os.environ.get("MMS_ORACLE_LIB")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 (no fast-math) and OpenMP."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_long), ("ny", ctypes.c_long), ("nz", ctypes.c_long),
                ("H", ctypes.c_long), ("sy", ctypes.c_long), ("sz", ctypes.c_long)]


_dp = ctypes.POINTER(ctypes.c_double)


class _Wave(ctypes.Structure):
    _fields_ = [("g", _Grid), ("r", ctypes.c_int), ("lap", _dp), ("c2", _dp),
                ("sponge_width", ctypes.c_int), ("sponge_alpha", ctypes.c_double),
                ("sponge_faces", ctypes.c_int), ("src_z", ctypes.c_long),
                ("src_y", ctypes.c_long), ("src_x", ctypes.c_long), ("src", _dp),
                ("nt", ctypes.c_int)]


class _Tti(ctypes.Structure):
    _fields_ = [("eps", _dp), ("delta", _dp), ("theta", _dp), ("phi", _dp),
                ("sigma", ctypes.c_double), ("alpha", ctypes.c_double), ("d1", _dp)]


def _load():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            lib = ctypes.CDLL(_LIB_OVERRIDE)
        else:
            build(force=False)
            lib = ctypes.CDLL(_LIB)
        gp = ctypes.POINTER(_Grid)
        wp = ctypes.POINTER(_Wave)
        lib.orc_star.argtypes = [_dp, _dp, gp, ctypes.c_int, _dp]
        lib.orc_box.argtypes = [_dp, _dp, gp, ctypes.c_int, _dp]
        lp = ctypes.POINTER(ctypes.c_long)
        lib.orc_star_at.argtypes = [_dp, gp, ctypes.c_int, _dp, ctypes.c_long, lp, _dp]
        lib.orc_box_at.argtypes = [_dp, gp, ctypes.c_int, _dp, ctypes.c_long, lp, _dp]
        for nm in ("orc_star2d", "orc_box2d"):
            getattr(lib, nm).argtypes = [_dp, _dp, gp, ctypes.c_int, _dp]
        for nm in ("orc_star2d_at", "orc_box2d_at"):
            getattr(lib, nm).argtypes = [_dp, gp, ctypes.c_int, _dp, ctypes.c_long, lp, _dp]
        lib.orc_sponge_1d.argtypes = [ctypes.c_long, ctypes.c_int, ctypes.c_double,
                                      ctypes.c_int, ctypes.c_int, _dp]
        lib.orc_wave_step.argtypes = [wp, ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
        lib.orc_wave_forward.argtypes = [wp, _dp, _dp, _dp, _dp, _dp, _dp]
        lib.orc_adjoint_step.argtypes = [wp, ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp]
        lib.orc_wave_adjoint.argtypes = [wp, _dp, _dp, _dp, _dp, _dp, _dp]
        lib.orc_vti_step.argtypes = [wp, ctypes.c_int] + [_dp] * 9
        lib.orc_vti_forward.argtypes = [wp] + [_dp] * 8
        tp = ctypes.POINTER(_Tti)
        lib.orc_tti_operators.argtypes = [wp, tp, _dp, _dp, _dp]
        lib.orc_tti_step.argtypes = [wp, tp, ctypes.c_int] + [_dp] * 7
        lib.orc_tti_forward.argtypes = [wp, tp] + [_dp] * 6
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _grid(a: np.ndarray, nx: int, ny: int, nz: int, halo: int) -> _Grid:
    assert a.ndim == 3 and a.shape[0] == nz + 2 * halo and a.shape[1] == ny + 2 * halo
    assert a.shape[2] >= nx + 2 * halo
    return _Grid(nx, ny, nz, halo, a.shape[2], a.shape[1] * a.shape[2])


def star(inp: np.ndarray, nx: int, ny: int, nz: int, radius: int, coeffs,
         halo: int = 4) -> np.ndarray:
    """Star sweep of a padded grid; coeffs [3][2r+1] (axis z, y, x).  Returns padded FP64."""
    a = _f64(inp)
    out = np.zeros_like(a)
    c = _f64(np.asarray(coeffs).reshape(3, 2 * radius + 1))
    g = _grid(a, nx, ny, nz, halo)
    _load().orc_star(_ptr(a), _ptr(out), ctypes.byref(g), radius, _ptr(c))
    return out


def box(inp: np.ndarray, nx: int, ny: int, nz: int, radius: int, coeffs,
        halo: int = 4) -> np.ndarray:
    """Box sweep of a padded grid; coeffs [dz][dy][dx].  Returns padded FP64."""
    a = _f64(inp)
    out = np.zeros_like(a)
    n = 2 * radius + 1
    c = _f64(np.asarray(coeffs).reshape(n, n, n))
    g = _grid(a, nx, ny, nz, halo)
    _load().orc_box(_ptr(a), _ptr(out), ctypes.byref(g), radius, _ptr(c))
    return out


def star2d(inp: np.ndarray, nx: int, ny: int, nz: int, radius: int, coeffs,
           halo: int = 4) -> np.ndarray:
    """2-D star on every z-plane (Table I 2DStar); coeffs [2][2r+1] (axis y, x)."""
    a = _f64(inp)
    out = np.zeros_like(a)
    c = _f64(np.asarray(coeffs).reshape(2, 2 * radius + 1))
    _load().orc_star2d(_ptr(a), _ptr(out), ctypes.byref(_grid(a, nx, ny, nz, halo)), radius,
                       _ptr(c))
    return out


def box2d(inp: np.ndarray, nx: int, ny: int, nz: int, radius: int, coeffs,
          halo: int = 4) -> np.ndarray:
    """2-D box on every z-plane (Table I 2DBox); coeffs [dy][dx]."""
    a = _f64(inp)
    out = np.zeros_like(a)
    n = 2 * radius + 1
    c = _f64(np.asarray(coeffs).reshape(n, n))
    _load().orc_box2d(_ptr(a), _ptr(out), ctypes.byref(_grid(a, nx, ny, nz, halo)), radius,
                      _ptr(c))
    return out


def _at(fn, inp, nx, ny, nz, radius, coeffs, points, halo, shape):
    a = inp if (inp.dtype == np.float64 and inp.flags.c_contiguous) else None
    if a is None:
        raise ValueError("sampled evaluation needs a contiguous FP64 grid (convert once, reuse)")
    pts = np.ascontiguousarray(points, dtype=np.int64).reshape(-1, 3)
    assert np.all(pts >= 0) and np.all(pts < np.array([nz, ny, nx]))
    c = _f64(np.asarray(coeffs).reshape(shape))
    out = np.zeros(len(pts))
    g = _grid(a, nx, ny, nz, halo)
    fn(_ptr(a), ctypes.byref(g), radius, _ptr(c), len(pts),
       pts.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _ptr(out))
    return out


def star_at(inp, nx, ny, nz, radius, coeffs, points, halo=4):
    """Star definition at the interior points [(z, y, x), ...] of an FP64 padded grid."""
    return _at(_load().orc_star_at, inp, nx, ny, nz, radius, coeffs, points, halo,
               (3, 2 * radius + 1))


def box_at(inp, nx, ny, nz, radius, coeffs, points, halo=4):
    """Box definition at the interior points [(z, y, x), ...] of an FP64 padded grid."""
    n = 2 * radius + 1
    return _at(_load().orc_box_at, inp, nx, ny, nz, radius, coeffs, points, halo, (n, n, n))


def sponge_1d(n: int, width: int, alpha: float, damp_lo: bool, damp_hi: bool) -> np.ndarray:
    g = np.zeros(n, dtype=np.float64)
    _load().orc_sponge_1d(n, width, alpha, int(damp_lo), int(damp_hi), _ptr(g))
    return g


def star2d_at(inp, nx, ny, nz, radius, coeffs, points, halo=4):
    return _at(_load().orc_star2d_at, inp, nx, ny, nz, radius, coeffs, points, halo,
               (2, 2 * radius + 1))


def box2d_at(inp, nx, ny, nz, radius, coeffs, points, halo=4):
    n = 2 * radius + 1
    return _at(_load().orc_box2d_at, inp, nx, ny, nz, radius, coeffs, points, halo, (n, n))


class Wave:
    """Acoustic problem description for the oracle (all arrays promoted to FP64)."""

    def __init__(self, nx, ny, nz, c2, lap_half, src, src_dt2f, nt, sponge_width=0,
                 sponge_alpha=0.0, sponge_faces=0, halo=4):
        self.nx, self.ny, self.nz, self.halo = nx, ny, nz, halo
        self.c2 = _f64(c2)
        self.lap = _f64(lap_half)
        self.src_dt2f = _f64(src_dt2f)
        self.shape = self.c2.shape
        self.nt = nt
        g = _grid(self.c2, nx, ny, nz, halo)
        self._s = _Wave(g, len(lap_half) - 1, _ptr(self.lap), _ptr(self.c2), sponge_width,
                        sponge_alpha, sponge_faces, src[0], src[1], src[2],
                        _ptr(self.src_dt2f), nt)

    @classmethod
    def from_setup(cls, s, lap_half, nt=None):
        return cls(s.nx, s.ny, s.nz, s.c2, lap_half, s.src, s.src_dt2f,
                   s.nt if nt is None else nt, s.sponge_width, s.sponge_alpha, s.sponge_faces)

    def zeros(self):
        return np.zeros(self.shape, dtype=np.float64)

    def step(self, n, uprev, ucur, image=None):
        """u^{n+1} from (u^{n-1}, u^n); returns (u^{n+1}, d^n)."""
        up, uc = _f64(uprev), _f64(ucur)
        un = self.zeros()
        tr = np.zeros((self.ny, self.nx))
        _load().orc_wave_step(ctypes.byref(self._s), n, _ptr(up), _ptr(uc), _ptr(un),
                              _ptr(tr), _ptr(image))
        return un, tr

    def forward(self, u0, u1, keep_states=False, image=False):
        """Returns dict(traces [nt][ny][nx], last (u^{nt-1}, u^nt), states?, image?)."""
        a, b = _f64(u0), _f64(u1)
        tr = np.zeros((self.nt, self.ny, self.nx))
        states = np.zeros((self.nt + 1,) + self.shape) if keep_states else None
        last = np.zeros((2,) + self.shape)
        img = self.zeros() if image else None
        _load().orc_wave_forward(ctypes.byref(self._s), _ptr(a), _ptr(b), _ptr(tr),
                                 _ptr(states), _ptr(last), _ptr(img))
        return {"traces": tr, "last": last, "states": states, "image": img}

    def adjoint_step(self, n, lam2, lam1, resid_n, u_n, grad):
        """lam^n from (lam^{n+2}, lam^{n+1}); adds the step's term to grad in place."""
        l2, l1 = _f64(lam2), _f64(lam1)
        l0 = self.zeros()
        r = None if resid_n is None else _f64(resid_n)
        u = None if u_n is None else _f64(u_n)
        assert grad is None or (grad.dtype == np.float64 and grad.flags.c_contiguous)
        _load().orc_adjoint_step(ctypes.byref(self._s), n, _ptr(l2), _ptr(l1), _ptr(l0),
                                 _ptr(r), _ptr(u), _ptr(grad))
        return l0

    def adjoint(self, states, resid):
        """Full adjoint over stored states; returns (grad_c2, dJ/du0, dJ/du1, dJ/dsrc)."""
        st = _f64(states)
        rs = _f64(resid)
        assert st.shape[0] >= self.nt and rs.shape == (self.nt, self.ny, self.nx)
        g, l0, l1 = self.zeros(), self.zeros(), self.zeros()
        gs = np.zeros(self.nt)
        _load().orc_wave_adjoint(ctypes.byref(self._s), _ptr(st), _ptr(rs), _ptr(g), _ptr(l0),
                                 _ptr(l1), _ptr(gs))
        return g, l0, l1, gs

    def vti_step(self, n, a, b, hp, hc, vp, vc):
        """VTI pair (Sec. II-A): returns (H^{n+1}, V^{n+1}, receiver plane of H^n)."""
        A, B = _f64(a), _f64(b)
        arrs = [_f64(t) for t in (hp, hc, vp, vc)]
        hn, vn = self.zeros(), self.zeros()
        tr = np.zeros((self.ny, self.nx))
        _load().orc_vti_step(ctypes.byref(self._s), n, _ptr(A), _ptr(B), _ptr(arrs[0]),
                             _ptr(arrs[1]), _ptr(hn), _ptr(arrs[2]), _ptr(arrs[3]), _ptr(vn),
                             _ptr(tr))
        return hn, vn, tr

    def tti(self, eps, delta, theta, phi, sigma, alpha, d1):
        """Bind TTI medium fields (padded) and parameters; returns the handle for tti_*."""
        keep = [_f64(a) for a in (eps, delta, theta, phi)] + [_f64(d1)]
        t = _Tti(_ptr(keep[0]), _ptr(keep[1]), _ptr(keep[2]), _ptr(keep[3]), float(sigma),
                 float(alpha), _ptr(keep[4]))
        return (t, keep)

    def tti_operators(self, tti, f):
        """(L f, H1 f) on the interior (Sec. II-A operators, Sec. IV-G mixed derivatives)."""
        ff = _f64(f)
        lf, h1 = self.zeros(), self.zeros()
        _load().orc_tti_operators(ctypes.byref(self._s), ctypes.byref(tti[0]), _ptr(ff), _ptr(lf),
                                  _ptr(h1))
        return lf, h1

    def tti_step(self, tti, n, pp, pc, qp, qc):
        """TTI pair (Sec. II-A): returns (p^{n+1}, q^{n+1}, receiver plane of p^n)."""
        arrs = [_f64(t) for t in (pp, pc, qp, qc)]
        pn, qn = self.zeros(), self.zeros()
        tr = np.zeros((self.ny, self.nx))
        _load().orc_tti_step(ctypes.byref(self._s), ctypes.byref(tti[0]), n, _ptr(arrs[0]),
                             _ptr(arrs[1]), _ptr(pn), _ptr(arrs[2]), _ptr(arrs[3]), _ptr(qn),
                             _ptr(tr))
        return pn, qn, tr

    def tti_forward(self, tti, p0, p1, q0, q1):
        """Returns dict(traces of p [nt][ny][nx], last = (p^{nt-1}, p^nt, q^{nt-1}, q^nt))."""
        arrs = [_f64(t) for t in (p0, p1, q0, q1)]
        tr = np.zeros((self.nt, self.ny, self.nx))
        last = np.zeros((4,) + self.shape)
        _load().orc_tti_forward(ctypes.byref(self._s), ctypes.byref(tti[0]),
                                *[_ptr(t) for t in arrs], _ptr(tr), _ptr(last))
        return {"traces": tr, "last": last}

    def vti_forward(self, a, b, h0, h1, v0, v1):
        """Returns dict(traces of H [nt][ny][nx], last = (H^{nt-1}, H^nt, V^{nt-1}, V^nt))."""
        A, B = _f64(a), _f64(b)
        arrs = [_f64(t) for t in (h0, h1, v0, v1)]
        tr = np.zeros((self.nt, self.ny, self.nx))
        last = np.zeros((4,) + self.shape)
        _load().orc_vti_forward(ctypes.byref(self._s), _ptr(A), _ptr(B), *[_ptr(t) for t in arrs],
                                _ptr(tr), _ptr(last))
        return {"traces": tr, "last": last}
