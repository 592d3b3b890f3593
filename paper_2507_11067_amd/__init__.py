"""MI355X (gfx950) library for the MMStencil hot path: 3-D high-order stencil
sweeps (star and box, radius 1..4) and the acoustic wave step they drive, with
its exact adjoint and gradient.

This module only marshals arguments for the C ABI of libmmstencil.so (declared
in include/mmstencil.h).  PyTorch supplies device memory and the current HIP
stream; every arithmetic step runs in the library's HIP kernels.  There is no
CPU fallback: if the library is not built, the calls raise.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import (MMS_BF16X1, MMS_BF16X3, MMS_BOX, MMS_BOX2D, MMS_FP16X3S, MMS_FP32,
                   MMS_REDUCE_WORK, MMS_STAR, MMS_STAR2D, MmsError, check, lib)

__all__ = ["Grid", "stencil_apply", "Wave", "Tti", "dot", "flat_dot", "flat_misfit", "flat_scale",
           "dense_to_grid", "reduce_work", "check_result", "MmsError", "PRECISIONS", "SHAPES"]

PRECISIONS = {"fp32": MMS_FP32, "bf16x3": MMS_BF16X3, "fp16x3s": MMS_FP16X3S, "bf16x1": MMS_BF16X1}
SHAPES = {"star": MMS_STAR, "box": MMS_BOX, "star2d": MMS_STAR2D, "box2d": MMS_BOX2D}


@dataclass(frozen=True)
class Grid:
    """Padded FP32 grid layout: interior (z, y, x) at [z+H][y+H][x+H] of a
    (nz+2H, ny+2H, sy) array, x fastest."""
    nx: int
    ny: int
    nz: int
    halo: int = 4
    sy: int | None = None

    def __post_init__(self):
        if self.sy is None:
            need = ((self.nx + 3) // 4) * 4 + 2 * self.halo
            object.__setattr__(self, "sy", ((need + 3) // 4) * 4)

    @classmethod
    def aligned(cls, nx: int, ny: int, nz: int, halo: int = 4) -> "Grid":
        """The layout of mms_grid_aligned: rows padded to 32 elements, so that with
        zeros()'s placement every interior row starts on a 128-byte boundary."""
        need = ((nx + 3) // 4) * 4 + 2 * halo
        return cls(nx, ny, nz, halo, ((need + 31) // 32) * 32)

    @property
    def lead(self) -> int:
        """Elements zeros() places in front of an FP32 array: (32 - H % 32) % 32 when
        sy is a multiple of 32 (interior rows then start on 128-byte boundaries), else 0."""
        return (32 - self.halo % 32) % 32 if self.sy % 32 == 0 else 0

    @property
    def shape(self):
        return (self.nz + 2 * self.halo, self.ny + 2 * self.halo, self.sy)

    @property
    def sz(self):
        return (self.ny + 2 * self.halo) * self.sy

    @property
    def points(self):
        return self.nx * self.ny * self.nz

    def c(self) -> _lib.MmsGrid:
        return _lib.MmsGrid(self.nx, self.ny, self.nz, self.halo, 0, self.sy, self.sz)

    def zeros(self, device="cuda", dtype=torch.float32) -> torch.Tensor:
        lead = self.lead if dtype == torch.float32 else 0
        if lead == 0:
            return torch.zeros(self.shape, device=device, dtype=dtype)
        n = self.shape[0] * self.shape[1] * self.shape[2]
        return torch.zeros(lead + n, device=device, dtype=dtype)[lead:].view(self.shape)

    def interior(self, t: torch.Tensor) -> torch.Tensor:
        H = self.halo
        return t[H:H + self.nz, H:H + self.ny, H:H + self.nx]


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _grid_ptr(t: torch.Tensor | None, grid: Grid, name: str, dtype=torch.float32):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name}: need a contiguous {dtype} CUDA tensor")
    if tuple(t.shape) != grid.shape:
        raise ValueError(f"{name}: shape {tuple(t.shape)} does not match grid {grid.shape}")
    return ctypes.c_void_p(t.data_ptr())


def _dev_ptr(t: torch.Tensor | None, name: str, dtype, numel: int | None = None):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name}: need a contiguous {dtype} CUDA tensor")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name}: needs {numel} elements, has {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def stencil_apply(inp: torch.Tensor, out: torch.Tensor, grid: Grid, shape: str, radius: int,
                  coeffs, precision: str = "fp32", stream=None) -> torch.Tensor:
    """One sweep out = S(inp) (star, box, star2d or box2d, radius 1..4), see mms_stencil_apply."""
    c = torch.as_tensor(coeffs, dtype=torch.float32).detach().cpu().contiguous().reshape(-1)
    g = grid.c()
    rc = lib().mms_stencil_apply(_grid_ptr(inp, grid, "inp"), _grid_ptr(out, grid, "out"),
                                 ctypes.byref(g), SHAPES[shape], int(radius),
                                 ctypes.cast(c.data_ptr(), ctypes.POINTER(ctypes.c_float)),
                                 c.numel(), PRECISIONS[precision], _stream(stream))
    check(rc, "mms_stencil_apply")
    return out


class Wave:
    """Acoustic problem (mms_wave) bound to device tensors.

    c2: padded grid tensor; C2 = c2_scale * c2 (c2_scale = 1 for a C2 field,
    dt^2/h^2 for a v^2 field).  src_dt2f: device [nt] FP32 or None.
    traces: device [nt, ny, nx] FP32 or None.  image: device [nz, ny, nx] FP64 or None.
    """

    def __init__(self, grid: Grid, c2: torch.Tensor, lap, nt: int, c2_scale: float = 1.0,
                 sponge_width: int = 0, sponge_alpha: float = 0.0, sponge_faces: int = 0,
                 src=(0, 0, 0), src_dt2f: torch.Tensor | None = None,
                 traces: torch.Tensor | None = None, image: torch.Tensor | None = None):
        self.grid = grid
        self.c2 = c2
        self.src_dt2f = src_dt2f
        self.traces = traces
        self.image = image
        self.nt = nt
        lapf = (ctypes.c_float * 5)(*([float(v) for v in lap] + [0.0] * (5 - len(lap))))
        self._w = _lib.MmsWave(grid.c(), len(lap) - 1, lapf, _grid_ptr(c2, grid, "c2"),
                               float(c2_scale), int(sponge_width), float(sponge_alpha),
                               int(sponge_faces), int(nt), int(src[0]), int(src[1]), int(src[2]),
                               _dev_ptr(src_dt2f, "src_dt2f", torch.float32, nt),
                               _dev_ptr(traces, "traces", torch.float32, nt * grid.ny * grid.nx),
                               _dev_ptr(image, "image", torch.float64, grid.points))

    def set_c2(self, c2: torch.Tensor, c2_scale: float | None = None):
        self.c2 = c2
        self._w.c2 = _grid_ptr(c2, self.grid, "c2")
        if c2_scale is not None:
            self._w.c2_scale = float(c2_scale)

    def set_traces(self, traces: torch.Tensor | None):
        self.traces = traces
        self._w.traces = _dev_ptr(traces, "traces", torch.float32,
                                  self.nt * self.grid.ny * self.grid.nx)

    def set_image(self, image: torch.Tensor | None, part: torch.Tensor | None = None,
                  block: int = 1):
        """FP64 image; with block K > 1 the terms of K consecutive steps are summed in the
        FP32 workspace `part` ([nz, ny, nx]) and added to the image at each block's end."""
        self.image = image
        self._w.image = _dev_ptr(image, "image", torch.float64, self.grid.points)
        self.set_accumulation(part, block)

    def set_accumulation(self, part: torch.Tensor | None, block: int):
        """Block size K of the FP64 accumulations (image in forward steps, gradient in
        adjoint steps) and their FP32 workspace ([nz, ny, nx]; needed when K > 1)."""
        self.acc_part = part
        self._w.acc_part = _dev_ptr(part, "acc_part", torch.float32, self.grid.points)
        self._w.acc_block = int(block)

    def set_source(self, src_dt2f: torch.Tensor | None, src=None):
        self.src_dt2f = src_dt2f
        self._w.src_dt2f = _dev_ptr(src_dt2f, "src_dt2f", torch.float32, self.nt)
        if src is not None:
            self._w.src_z, self._w.src_y, self._w.src_x = (int(v) for v in src)

    def step(self, n, u_prev, u_cur, u_next, stream=None):
        g = self.grid
        check(lib().mms_wave_step(ctypes.byref(self._w), int(n), _grid_ptr(u_prev, g, "u_prev"),
                                  _grid_ptr(u_cur, g, "u_cur"), _grid_ptr(u_next, g, "u_next"),
                                  _stream(stream)), "mms_wave_step")

    def record(self, n, u, stream=None):
        check(lib().mms_wave_record(ctypes.byref(self._w), int(n), _grid_ptr(u, self.grid, "u"),
                                    _stream(stream)), "mms_wave_record")

    def forward(self, n_begin, n_end, states, stream=None):
        """Steps n_begin..n_end-1; states[i] is u^{n_begin-1+i} (see mms_wave_forward)."""
        arr = (ctypes.c_void_p * len(states))(*[_grid_ptr(s, self.grid, "state") for s in states])
        if len(states) < n_end - n_begin + 2:
            raise ValueError("states too short")
        check(lib().mms_wave_forward(ctypes.byref(self._w), int(n_begin), int(n_end), arr,
                                     _stream(stream)), "mms_wave_forward")

    def adjoint_step(self, n, lam_np2, lam_np1, lam_n, resid=None, u_n=None, grad=None,
                     stream=None):
        g = self.grid
        check(lib().mms_wave_adjoint_step(
            ctypes.byref(self._w), int(n), _grid_ptr(lam_np2, g, "lam_np2"),
            _grid_ptr(lam_np1, g, "lam_np1"), _grid_ptr(lam_n, g, "lam_n"),
            _dev_ptr(resid, "resid", torch.float32, self.nt * g.ny * g.nx),
            _grid_ptr(u_n, g, "u_n"), _dev_ptr(grad, "grad", torch.float64, g.points),
            _stream(stream)), "mms_wave_adjoint_step")

    def adjoint(self, n_hi, n_lo, lams, us=None, resid=None, grad=None, stream=None):
        """Adjoint steps n_hi..n_lo; lams[i] is lam^{n_lo+i}, us[i] is u^{n_lo+i}."""
        g = self.grid
        if len(lams) < n_hi - n_lo + 3:
            raise ValueError("lams too short")
        if us is not None and len(us) < n_hi - n_lo + 1:
            raise ValueError("us too short")
        la = (ctypes.c_void_p * len(lams))(*[_grid_ptr(t, g, "lam") for t in lams])
        ua = None
        if us is not None:
            ua = (ctypes.c_void_p * len(us))(*[_grid_ptr(t, g, "u") for t in us])
        check(lib().mms_wave_adjoint(
            ctypes.byref(self._w), int(n_hi), int(n_lo), la, ua,
            _dev_ptr(resid, "resid", torch.float32, self.nt * g.ny * g.nx),
            _dev_ptr(grad, "grad", torch.float64, g.points), _stream(stream)), "mms_wave_adjoint")

    def adjoint_mu(self, n_hi, n_lo, mus, us=None, resid=None, grad=None, stream=None):
        """Adjoint steps n_hi..n_lo in the variable mu = C2 G lam (see mms_wave_adjoint_mu);
        mus[i] is mu^{n_lo+i}, us[i] is u^{n_lo+i}.  Needs c2 > 0 in every cell."""
        g = self.grid
        if len(mus) < n_hi - n_lo + 3:
            raise ValueError("mus too short")
        if us is not None and len(us) < n_hi - n_lo + 1:
            raise ValueError("us too short")
        ma = (ctypes.c_void_p * len(mus))(*[_grid_ptr(t, g, "mu") for t in mus])
        ua = None
        if us is not None:
            ua = (ctypes.c_void_p * len(us))(*[_grid_ptr(t, g, "u") for t in us])
        check(lib().mms_wave_adjoint_mu(
            ctypes.byref(self._w), int(n_hi), int(n_lo), ma, ua,
            _dev_ptr(resid, "resid", torch.float32, self.nt * g.ny * g.nx),
            _dev_ptr(grad, "grad", torch.float64, g.points), _stream(stream)), "mms_wave_adjoint_mu")

    def scale_mu(self, inp, out, direction, stream=None):
        """out = C2 G inp (direction +1, lam -> mu) or inp / (C2 G) (direction -1)."""
        g = self.grid
        check(lib().mms_wave_scale_mu(ctypes.byref(self._w), _grid_ptr(inp, g, "in"),
                                      _grid_ptr(out, g, "out"), int(direction), _stream(stream)),
              "mms_wave_scale_mu")

    def vti_step(self, n, a, b, h_prev, h_cur, h_next, v_prev, v_cur, v_next, stream=None):
        """One pseudo-acoustic VTI step (see mms_vti_step); a = 1 + 2 eps, b = sqrt(1 + 2 delta)."""
        g = self.grid
        check(lib().mms_vti_step(ctypes.byref(self._w), int(n), _grid_ptr(a, g, "a"),
                                 _grid_ptr(b, g, "b"), _grid_ptr(h_prev, g, "h_prev"),
                                 _grid_ptr(h_cur, g, "h_cur"), _grid_ptr(h_next, g, "h_next"),
                                 _grid_ptr(v_prev, g, "v_prev"), _grid_ptr(v_cur, g, "v_cur"),
                                 _grid_ptr(v_next, g, "v_next"), _stream(stream)), "mms_vti_step")

    def tti_step(self, n, tti: "Tti", p_prev, p_cur, p_next, q_prev, q_cur, q_next, stream=None):
        """One pseudo-acoustic TTI step (see mms_tti_step)."""
        g = self.grid
        check(lib().mms_tti_step(ctypes.byref(self._w), ctypes.byref(tti._t), int(n),
                                 _grid_ptr(p_prev, g, "p_prev"), _grid_ptr(p_cur, g, "p_cur"),
                                 _grid_ptr(p_next, g, "p_next"), _grid_ptr(q_prev, g, "q_prev"),
                                 _grid_ptr(q_cur, g, "q_cur"), _grid_ptr(q_next, g, "q_next"),
                                 _stream(stream)), "mms_tti_step")

    def energy_work(self) -> int:
        """Doubles of workspace mms_wave_energy needs for this grid."""
        n = ctypes.c_int64(0)
        check(lib().mms_wave_energy_work(ctypes.byref(self._w), ctypes.byref(n)),
              "mms_wave_energy_work")
        return int(n.value)

    def energy(self, u_n, u_np1, out=None, work=None, stream=None) -> float:
        """Discrete energy (mms_wave_energy); raises MmsError (MMS_EUNSTABLE) if it meets
        NaN or Inf.  `out` (2 FP64 on the device) receives the result pair."""
        if out is None:
            out = torch.zeros(2, dtype=torch.float64, device=u_n.device)
        need = self.energy_work()
        if work is None:
            work = torch.empty(max(need, 1), dtype=torch.float64, device=u_n.device)
        check(lib().mms_wave_energy(ctypes.byref(self._w), _grid_ptr(u_n, self.grid, "u_n"),
                                    _grid_ptr(u_np1, self.grid, "u_np1"),
                                    _dev_ptr(out, "out", torch.float64, 2),
                                    _dev_ptr(work, "work", torch.float64, need), work.numel(),
                                    _stream(stream)), "mms_wave_energy")
        return check_result(out, "mms_wave_energy")


class Tti:
    """TTI medium (mms_tti) bound to device tensors; allocates its 4-grid workspace once."""

    def __init__(self, grid: Grid, eps, delta, theta, phi, sigma: float, alpha: float, d1,
                 device="cuda"):
        self.grid = grid
        self.fields = (eps, delta, theta, phi)
        self.work = torch.empty((4,) + grid.shape, dtype=torch.float32, device=device)
        d = (ctypes.c_float * 4)(*([float(v) for v in d1] + [0.0] * (4 - len(d1))))
        self._t = _lib.MmsTti(_grid_ptr(eps, grid, "eps"), _grid_ptr(delta, grid, "delta"),
                              _grid_ptr(theta, grid, "theta"), _grid_ptr(phi, grid, "phi"),
                              float(sigma), float(alpha), d,
                              ctypes.c_void_p(self.work.data_ptr()))


def reduce_work(device) -> torch.Tensor:
    """A workspace for one FP64 reduction (MMS_REDUCE_WORK doubles).  Taken from torch's
    stream-ordered caching allocator, so a fresh one per call costs no device allocation."""
    return torch.empty(MMS_REDUCE_WORK, dtype=torch.float64, device=device)


def check_result(pair: torch.Tensor, where: str = "reduction") -> float:
    """Copy a reduction's (sum, non-finite count) pair to the host; raise MmsError
    (MMS_EUNSTABLE) if it reports NaN or Inf, else return the sum."""
    host = pair.detach().to("cpu", torch.float64).contiguous()
    check(lib().mms_check_reduction(ctypes.cast(host.data_ptr(), ctypes.POINTER(ctypes.c_double))),
          where)
    return float(host[0])


def _pair(out, device):
    if out is None:
        return torch.zeros(2, dtype=torch.float64, device=device)
    return out


def dot(a: torch.Tensor, b: torch.Tensor | None, grid: Grid, out=None, work=None,
        stream=None) -> float:
    """FP64 interior dot product (mms_dot_f64); raises MmsError on NaN or Inf."""
    out = _pair(out, a.device)
    work = reduce_work(a.device) if work is None else work
    g = grid.c()
    check(lib().mms_dot_f64(_grid_ptr(a, grid, "a"), _grid_ptr(b, grid, "b"), ctypes.byref(g),
                            _dev_ptr(out, "out", torch.float64, 2),
                            _dev_ptr(work, "work", torch.float64, MMS_REDUCE_WORK),
                            _stream(stream)), "mms_dot_f64")
    return check_result(out, "mms_dot_f64")


def flat_dot(a: torch.Tensor, b: torch.Tensor | None = None, out=None, work=None,
             stream=None) -> float:
    """FP64 dot product of two flat FP32 tensors (mms_flat_dot_f64); raises on NaN or Inf."""
    out = _pair(out, a.device)
    work = reduce_work(a.device) if work is None else work
    n = a.numel()
    check(lib().mms_flat_dot_f64(_dev_ptr(a, "a", torch.float32), _dev_ptr(b, "b", torch.float32, n),
                                 n, _dev_ptr(out, "out", torch.float64, 2),
                                 _dev_ptr(work, "work", torch.float64, MMS_REDUCE_WORK),
                                 _stream(stream)), "mms_flat_dot_f64")
    return check_result(out, "mms_flat_dot_f64")


def flat_misfit(a: torch.Tensor, b: torch.Tensor, resid: torch.Tensor | None = None,
                out: torch.Tensor | None = None, work=None, stream=None) -> torch.Tensor:
    """0.5 * sum (a - b)^2 in FP64 on the device, returned as the device result pair
    (sum, non-finite count) without a host synchronisation; writes resid = a - b when
    given."""
    out = _pair(out, a.device)
    work = reduce_work(a.device) if work is None else work
    n = a.numel()
    check(lib().mms_flat_misfit_f64(_dev_ptr(a, "a", torch.float32),
                                    _dev_ptr(b, "b", torch.float32, n),
                                    _dev_ptr(resid, "resid", torch.float32, n), n,
                                    _dev_ptr(out, "out", torch.float64, 2),
                                    _dev_ptr(work, "work", torch.float64, MMS_REDUCE_WORK),
                                    _stream(stream)), "mms_flat_misfit_f64")
    return out


def flat_scale(inp: torch.Tensor, scale: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
    """out = (float)(scale * inp) with the FP64 scale read on the device (mms_flat_scale_f32)."""
    n = inp.numel()
    check(lib().mms_flat_scale_f32(_dev_ptr(inp, "inp", torch.float32),
                                   _dev_ptr(scale, "scale", torch.float64, 1),
                                   _dev_ptr(out, "out", torch.float32, n), n, _stream(stream)),
          "mms_flat_scale_f32")
    return out


def dense_to_grid(dense: torch.Tensor, out: torch.Tensor, grid: Grid, scale: float = 1.0,
                  stream=None) -> torch.Tensor:
    g = grid.c()
    check(lib().mms_dense_to_grid(_dev_ptr(dense, "dense", torch.float64, grid.points),
                                  _grid_ptr(out, grid, "out"), ctypes.byref(g), float(scale),
                                  _stream(stream)), "mms_dense_to_grid")
    return out
