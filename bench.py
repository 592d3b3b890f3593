#!/usr/bin/env python3
"""Benchmark of the MMStencil hot path on one MI355X.

Headline workload (the value of the JSON line): FP32 sweeps of a 512^3 grid
with a 4-cell zero halo and uniform [-1, 1] data (seed 2) through three
stencils -- the radius-4 25-point star (8th-order Laplacian), a radius-2
125-point box and a radius-4 729-point box (uniform [-1, 1] weights with the
mean removed, seeds 3 and 4).  One step = one sweep of each stencil; the value
is interior points swept per second over the timed steps (Gpoints/s).

Besides the headline the same JSON line carries, each measured in this run:
  * "kernels": per-stencil Gpoints/s, achieved GB/s or TFLOP/s and the max /
    RMS error against the FP64 oracle over every interior point;
  * "config0": the 64^3 radius-4 Laplacian star, 10 repeated sweeps (time and error);
  * "split_mfma": the radius-4 and radius-3 boxes three ways (FP32 VALU, BF16x3
    and FP16x3S split MFMA, plus the BF16x1 error report);
  * "rtm": the 400^3, 2000-step acoustic forward model with FP64 imaging;
  * "table1": every kernel of the paper's Table I at 512^3 (the 2-D ones on each
    plane of the 512^3 stack), with HBM and FP32-FMA roofline fractions;
  * "vti": the 400^3, 1000-step pseudo-acoustic VTI forward model (two fields);
  * "tti": the 400^3, 300-step pseudo-acoustic TTI forward model (two fields, tilt);
  * "gradient": the 256^3, 1000-step adjoint gradient with checkpointing,
    with its dot-product test;
  * "roofline" of the dominant kernel and "cpu_baseline" (the FP64 oracle on
    the host cores over one step of the headline workload).

The FP64 oracle runs only in the CPU-baseline leg: it times the oracle on one
headline step and keeps those full-grid outputs (with untimed oracle sweeps of
the other 512^3 kernels) as the references of every error column, so each
error is over all 134,217,728 outputs of a sweep.

Kernels run on torch's current stream; HIP events recorded on that stream
bracket every launch, so per-kernel times come from the same events.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gpoints/s per sweep (FP32 vs split-MFMA at <=1e-5 rel err); % HBM/MFMA peak"
HBM_PEAK_GBS = 8000.0
FP32_VALU_PEAK_TF = 157.3   # published vector FP32 (packed) peak
MFMA_BF16_PEAK_TF = 2516.6  # published dense BF16/FP16 MFMA peak
LAP = None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=100)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--n", type=int, default=512, help="headline grid edge")
    p.add_argument("--only", default="", help="profile one kernel: star|box2|box3|box4|box4_bf16x3|"
                   "box4_fp16x3s|box3_bf16x3|wave|vti|copy|2DStarR2|2DStarR4|2DBoxR2|2DBoxR3|"
                   "3DStarR2|3DBoxR1|tti")
    p.add_argument("--skip", default="", help="comma list of extras to skip: "
                   "config0,split,table1,rtm,vti,tti,gradient,cpu,check")
    p.add_argument("--collect", action="store_true",
                   help="run rocprofv3 (kernel trace, FETCH_SIZE, WRITE_SIZE) as child processes "
                        "over the headline kernels and a plain copy, and write profiles/")
    p.add_argument("--collect-dir", default=os.path.join(ROOT, "rocprof_out"),
                   help="where --collect puts the raw rocprofv3 output and a copy of the summaries")
    return p.parse_args()


class Timer:
    """Per-kernel HIP event pairs on torch's current stream."""

    def __init__(self, torch):
        self.torch = torch
        self.pairs = {}

    def run(self, name, fn):
        t = self.torch
        a, b = t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        self.pairs.setdefault(name, []).append((a, b))

    def ms(self, name):
        return float(np.mean([a.elapsed_time(b) for a, b in self.pairs[name]]))

    def reset(self):
        self.pairs = {}


def time_launches(torch, f, warm_ms=60.0, min_ms=150.0):
    """Mean ms per launch of f on torch's current stream.  The GPU is first kept busy
    for warm_ms (clocks ramp up after idle periods), then launches are timed in one
    event pair over at least min_ms."""
    ev = lambda: torch.cuda.Event(enable_timing=True)
    a, b = ev(), ev()
    a.record()
    f()
    b.record()
    torch.cuda.synchronize()
    est = max(a.elapsed_time(b), 1e-3)
    for _ in range(int(warm_ms / est) + 1):
        f()
    torch.cuda.synchronize()
    reps = max(10, int(min_ms / est))
    a.record()
    for _ in range(reps):
        f()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              "(the multi-GPU z-slab decomposition is a design note, not built)",
              file=sys.stderr)
        sys.exit(2)
    if args.collect:
        return collect_counters(args)
    import torch
    import paper_2507_11067_amd as mms
    import synth

    global LAP
    LAP = [float(v) for v in synth.LAPLACIAN_R4]
    skip = set(s for s in args.skip.split(",") if s)
    dev = torch.device("cuda:0")
    n = args.n
    # rows padded to a multiple of 32 elements and placed so that every interior row
    # starts on a 128-byte boundary (mms_grid_aligned): the output rows of the sweeps
    # cover whole cache lines (measured: star r4 653 -> 717 Gpoints/s at 512^3)
    grid = mms.Grid.aligned(n, n, n)
    log(f"[bench] generating {n}^3 input (seed 2)")
    x_np = synth.uniform_grid(2, n, n, n, sy=grid.sy)
    x = grid.zeros(dev)
    x.copy_(torch.from_numpy(x_np))
    outs = {k: grid.zeros(dev) for k in ("star", "box2", "box4")}
    c_star = synth.star_coeffs_laplacian(4)
    c_box2 = synth.box_coeffs(3, 2)
    c_box4 = synth.box_coeffs(4, 4)
    c_box3 = synth.box_coeffs(6, 3)
    sweeps = {
        "star": lambda: mms.stencil_apply(x, outs["star"], grid, "star", 4, c_star),
        "box2": lambda: mms.stencil_apply(x, outs["box2"], grid, "box", 2, c_box2),
        "box4": lambda: mms.stencil_apply(x, outs["box4"], grid, "box", 4, c_box4),
    }

    if args.only:
        return profile_only(args, torch, mms, synth, grid, x, outs, sweeps, c_box4, c_box3, dev)

    timer = Timer(torch)
    log(f"[bench] warmup {args.warmup} steps")
    for _ in range(args.warmup):
        for f in sweeps.values():
            f()
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps")
    t0 = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        for name, f in sweeps.items():
            timer.run(name, f)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = e0.elapsed_time(e1)
    ms_step = total_ms / args.steps
    pts = grid.points
    value = 3 * pts / (ms_step * 1e-3) / 1e9
    log(f"[bench] {ms_step:.3f} ms/step, {value:.1f} Gpoints/s (wall {wall:.2f} s)")

    kernels = {}
    per = {"star": ("hbm", 8.0, 50.0), "box2": ("alu", 8.0, 250.0), "box4": ("alu", 8.0, 1458.0)}
    for name, (bound, bytes_pt, flop_pt) in per.items():
        ms = timer.ms(name)
        gpts = pts / (ms * 1e-3) / 1e9
        kernels[name] = {"ms": ms, "gpoints_s": gpts, "gbs": gpts * bytes_pt,
                         "tflops": gpts * flop_pt / 1e3,
                         "hbm_frac": gpts * bytes_pt / HBM_PEAK_GBS,
                         "valu_frac": gpts * flop_pt / 1e3 / FP32_VALU_PEAK_TF}
    # dominant kernel of the step: the radius-4 box (FP32 FMA bound)
    dom = max(kernels, key=lambda k: kernels[k]["ms"])
    kd = kernels[dom]
    if per[dom][0] == "hbm":
        roof = {"bound": "hbm", "achieved": kd["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    else:
        roof = {"bound": "alu", "achieved": kd["tflops"], "peak": FP32_VALU_PEAK_TF,
                "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["kernel"] = {"star": "star_kernel<4>", "box2": "box_valu_kernel<2>",
                      "box4": "box_valu_kernel<4>"}[dom]
    roof["traffic"] = traffic_for(dom)
    u = util_for(dom)
    if u:
        roof["rocprof"] = u
    rooflines = {}
    for name, (bound, bytes_pt, flop_pt) in per.items():
        k = kernels[name]
        if bound == "hbm":
            rooflines[name] = {"bound": "hbm", "achieved": k["gbs"], "peak": HBM_PEAK_GBS,
                               "unit": "GB/s", "frac": k["hbm_frac"], "traffic": traffic_for(name)}
        else:
            rooflines[name] = {"bound": "alu", "achieved": k["tflops"], "peak": FP32_VALU_PEAK_TF,
                               "unit": "TFLOP/s", "frac": k["valu_frac"],
                               "traffic": traffic_for(name)}

    # context for the HBM-bound rows: what a plain device copy of the same padded grid
    # moves on this GPU (read + write), timed the same way
    # (two fresh flat buffers of the grid's size, so that torch's copy sees its usual
    # allocator alignment)
    ca = x.reshape(-1).clone()
    cb = torch.empty_like(ca)
    cms = time_launches(torch, lambda: cb.copy_(ca))
    del ca, cb
    copy_gbs = 2.0 * x.numel() * 4 / (cms * 1e-3) / 1e9
    rooflines["star"]["copy_gbs"] = copy_gbs
    rooflines["star"]["frac_of_copy"] = kernels["star"]["gbs"] / copy_gbs
    if rooflines["star"]["traffic"]:
        # bytes the counters saw per sweep, over the live sweep time
        rooflines["star"]["traffic_gbs"] = rooflines["star"]["traffic"] / (kernels["star"]["ms"] * 1e-3) / 1e9
    log(f"[bench] plain copy of the padded grid: {copy_gbs:.0f} GB/s; star at "
        f"{kernels['star']['gbs'] / copy_gbs:.2f} of it (algorithmic bytes)")

    result = {
        "metric": METRIC, "value": value, "unit": "Gpoints/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{n}^3 FP32 sweeps, one step = radius-4 star + radius-2 box + "
                               "radius-4 box (4-cell zero halo, uniform [-1,1] seed 2)",
                   "grid": [n, n, n], "halo": 4, "row_pitch": grid.sy,
                   "interior_rows_128B_aligned": True, "points_per_step": 3 * pts},
        "roofline": roof,
        "rooflines": rooflines,
        "kernels": kernels,
    }
    if "config0" not in skip:
        result["config0"] = bench_config0(torch, mms, synth, dev)
    if "split" not in skip:
        result["split_mfma"] = bench_split(torch, mms, grid, x, c_box4, c_box3, dev)
    if "table1" not in skip:
        result["table1"] = bench_table1(torch, mms, synth, grid, x, dev)
    if "cpu" not in skip:
        result["cpu_baseline"] = cpu_baseline_leg(torch, mms, synth, grid, x, x_np, n, dev, result,
                                                  c_star, c_box2, c_box4, c_box3,
                                                  "check" not in skip)
    del outs
    if "rtm" not in skip:
        result["rtm"] = bench_rtm(torch, mms, synth, dev)
    if "vti" not in skip:
        result["vti"] = bench_vti(torch, mms, synth, dev)
    if "tti" not in skip:
        result["tti"] = bench_tti(torch, mms, synth, dev)
    if "gradient" not in skip:
        result["gradient"] = bench_gradient(torch, mms, synth, dev)
    print(json.dumps(result), flush=True)


def bench_split(torch, mms, grid, x, c_box4, c_box3, dev):
    """Radius-4 and radius-3 boxes at 512^3 three ways (FP32 VALU, BF16x3 and FP16x3S split
    MFMA, plus BF16x1); their errors against the FP64 oracle are added by the CPU leg."""
    out = grid.zeros(dev)
    res = {}
    for r, c in ((4, c_box4), (3, c_box3)):
        for prec in ("fp32", "bf16x3", "fp16x3s", "bf16x1"):
            f = lambda: mms.stencil_apply(x, out, grid, "box", r, c, precision=prec)
            ms = time_launches(torch, f)
            gpts = grid.points / (ms * 1e-3) / 1e9
            e = {"ms": ms, "gpoints_s": gpts}
            flop = 2 * (2 * r + 1) ** 3
            e["algorithmic_tflops"] = gpts * flop / 1e3
            if prec == "fp32":
                e["valu_frac"] = gpts * flop / 1e3 / FP32_VALU_PEAK_TF
            else:
                # the method's 2 (2r+1)^3 flop per point against the MFMA peak, and the
                # issued 16x16x32 MFMA work (Toeplitz band, split products) beside it
                nch = -(-((2 * r + 1) * 24) // 32)
                mfma_per_tile = (3 if prec != "bf16x1" else 1) * (2 * r + 1) * nch
                issued = gpts * 1e9 / 256 * mfma_per_tile * 16 * 16 * 32 * 2 / 1e12
                e["mfma_algorithmic_frac"] = e["algorithmic_tflops"] / MFMA_BF16_PEAK_TF
                e["mfma_issued_tflops"] = issued
                e["mfma_issued_frac"] = issued / MFMA_BF16_PEAK_TF
            u = util_for(f"box{r}_{prec}") if prec != "fp32" else None
            if u:
                e["rocprof_mfma_util_pct"] = u.get("MfmaUtil")
                mops = u.get("SQ_INSTS_VALU_MFMA_MOPS_BF16")
                if mops:
                    e["rocprof_mfma_tflops"] = mops * 512 / (ms * 1e-3) / 1e12
                e["rocprof_lds_bank_conflict_pct"] = u.get("LDSBankConflict")
            res[f"box_r{r}_{prec}"] = e
            log(f"[bench] box r{r} {prec}: {gpts:.1f} Gpoints/s")
        res[f"box_r{r}_speedup_bf16x3_over_fp32"] = (res[f"box_r{r}_bf16x3"]["gpoints_s"] /
                                                     res[f"box_r{r}_fp32"]["gpoints_s"])
        res[f"box_r{r}_speedup_fp16x3s_over_fp32"] = (res[f"box_r{r}_fp16x3s"]["gpoints_s"] /
                                                      res[f"box_r{r}_fp32"]["gpoints_s"])
    return res


def bench_config0(torch, mms, synth, dev, n=64, sweeps=10):
    """The 64^3 radius-4 Laplacian star (4-cell zero halo, uniform [-1, 1], seed 1), 10
    repeated out-of-place sweeps of the same input; its error is added by the CPU leg.
    Timed twice: eager launches from Python (bound by the host side of each call at this
    size) and the 10 sweeps captured once in a HIP graph and replayed (the GPU's time)."""
    grid = mms.Grid(n, n, n)
    x = torch.from_numpy(synth.uniform_grid(1, n, n, n, sy=grid.sy)).to(dev)
    out = grid.zeros(dev)
    c = synth.star_coeffs_laplacian(4)
    f = lambda: mms.stencil_apply(x, out, grid, "star", 4, c)
    for _ in range(3):
        f()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(sweeps):
        f()
    b.record()
    torch.cuda.synchronize()
    ms_eager = a.elapsed_time(b)
    # the same 10 sweeps captured on a side stream and replayed on it
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            for _ in range(sweeps):
                f()
        for _ in range(3):
            graph.replay()
        side.synchronize()
        reps = 20
        a.record(side)
        for _ in range(reps):
            graph.replay()
        b.record(side)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    gpts = sweeps * grid.points / (ms * 1e-3) / 1e9
    gpts_eager = sweeps * grid.points / (ms_eager * 1e-3) / 1e9
    log(f"[bench] config 0 (64^3 star r4, {sweeps} sweeps): {ms * 1e3:.1f} us from a HIP graph, "
        f"{gpts:.1f} Gpoints/s ({ms_eager * 1e3:.1f} us, {gpts_eager:.1f} Gpoints/s eager)")
    return {"grid": [n, n, n], "sweeps": sweeps, "ms_total": ms, "us_per_sweep": ms * 1e3 / sweeps,
            "gpoints_s": gpts, "timing": "the sweeps replayed from a captured HIP graph",
            "ms_total_eager": ms_eager, "us_per_sweep_eager": ms_eager * 1e3 / sweeps,
            "gpoints_s_eager": gpts_eager,
            "note": "1 MB grid: latency-bound small-grid kernel; eager launches are bound by "
                    "the host side of each call"}

def bench_rtm(torch, mms, synth, dev, n=400, nt=2000):
    """Acoustic forward model, 400^3, 2000 steps, FP64 image fused (and without)."""
    log(f"[bench] rtm setup {n}^3 x {nt}")
    s = synth.wave_setup(n, nt, seed=7, sponge_width=32)
    grid = mms.Grid(n, n, n)
    c2 = torch.from_numpy(s.c2).to(dev)
    f = torch.from_numpy(s.src_dt2f).to(dev)
    traces = torch.zeros((nt, n, n), device=dev)
    image = torch.zeros((n, n, n), dtype=torch.float64, device=dev)
    part = torch.empty((n, n, n), device=dev)
    res = {"grid": [n, n, n], "steps": nt - 1, "dt": s.dt, "image_block": IMAGE_BLOCK}
    # with_image: the image summed per block of IMAGE_BLOCK steps in FP32 and added in FP64;
    # with_image_each_step: every step's term added in FP64
    for key, with_image, block in (("with_image", True, IMAGE_BLOCK),
                                   ("with_image_each_step", True, 1), ("no_image", False, 1)):
        w = mms.Wave(grid, c2, LAP, nt, 1.0, s.sponge_width, s.sponge_alpha, s.sponge_faces,
                     s.src, f, traces)
        if with_image:
            w.set_image(image, part if block > 1 else None, block)
        bufs = [grid.zeros(dev) for _ in range(3)]
        image.zero_()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        w.record(0, bufs[0])
        w.forward(1, nt, [bufs[i % 3] for i in range(nt + 1)])
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        gpts = grid.points * (nt - 1) / (ms * 1e-3) / 1e9
        # algorithmic bytes per point-step: u^n, u^{n-1}, C2 read, u^{n+1} written; the FP64
        # image read and written (16 B), or per block of K steps: the FP32 partial written
        # (4 B), updated K-2 times (8 B), then read once with one FP64 read-modify-write
        # (20 B), i.e. 8 + 8/K B per step
        bpp = 16.0 + ((16.0 if block == 1 else 8.0 + 8.0 / block) if with_image else 0.0)
        res[key] = {"ms_total": ms, "ms_per_step": ms / (nt - 1), "gpoints_s": gpts,
                    "algorithmic_bytes_per_point": bpp, "gbs": gpts * bpp,
                    "hbm_frac": gpts * bpp / HBM_PEAK_GBS}
        log(f"[bench] rtm {key}: {gpts:.1f} Gpoints/s ({ms:.0f} ms)")
        if with_image:
            res["trace_max_abs"] = float(traces.abs().max().item())
            res[key]["image_sum"] = float(image.sum().item())
    # context for the step's access mix (three fields read, one written): what a plain
    # streaming op over four grids of the same padded size moves on this GPU, timed the
    # same way (torch.addcmul reads three and writes one)
    st = [grid.zeros(dev) for _ in range(4)]
    for t in st[:3]:
        t.uniform_(-1.0, 1.0)
    sms = time_launches(torch, lambda: torch.addcmul(st[0], st[1], st[2], out=st[3]))
    stream_gbs = 4.0 * st[0].numel() * 4 / (sms * 1e-3) / 1e9
    del st
    res["stream_3r1w_gbs"] = stream_gbs
    res["no_image"]["frac_of_stream"] = res["no_image"]["gbs"] / stream_gbs
    log(f"[bench] rtm: three-read one-write stream of the padded grid {stream_gbs:.0f} GB/s; "
        f"the step (no image) at {res['no_image']['frac_of_stream']:.2f} of it (algorithmic bytes)")
    return res


def table1_kernels(synth):
    """Table I kernels: name -> (shape, radius, coefficients, pattern in the table)."""
    return {
        "2DStarR2": ("star2d", 2, synth.star2d_coeffs_laplacian(2), "memory"),
        "2DStarR4": ("star2d", 4, synth.star2d_coeffs_laplacian(4), "memory"),
        "2DBoxR2": ("box2d", 2, synth.box2d_coeffs(12, 2), "memory"),
        "2DBoxR3": ("box2d", 3, synth.box2d_coeffs(13, 3), "both"),
        "3DStarR2": ("star", 2, synth.star_coeffs_laplacian(2), "memory"),
        "3DStarR4": ("star", 4, synth.star_coeffs_laplacian(4), "memory"),
        "3DBoxR1": ("box", 1, synth.box_coeffs(11, 1), "memory"),
        "3DBoxR2": ("box", 2, synth.box_coeffs(3, 2), "compute"),
    }


def bench_table1(torch, mms, synth, grid, x, dev):
    """Every Table I kernel on the 512^3 grid (2-D kernels on each of its planes), FP32; the
    errors against the FP64 oracle are added by the CPU leg."""
    out = grid.zeros(dev)
    res = {}
    for name, (shape, r, c, pattern) in table1_kernels(synth).items():
        f = lambda: mms.stencil_apply(x, out, grid, shape, r, c)
        ms = time_launches(torch, f)
        gpts = grid.points / (ms * 1e-3) / 1e9
        npts = c.size if shape in ("box", "box2d") else (c.shape[0] * (2 * r + 1) - c.shape[0] + 1)
        flop = 2 * int(npts)
        e = {"shape": shape, "radius": r, "points": int(npts), "table_pattern": pattern,
             "ms": ms, "gpoints_s": gpts, "gbs": gpts * 8.0, "hbm_frac": gpts * 8.0 / HBM_PEAK_GBS,
             "tflops": gpts * flop / 1e3, "valu_frac": gpts * flop / 1e3 / FP32_VALU_PEAK_TF}
        res[name] = e
        log(f"[bench] {name}: {gpts:.1f} Gpoints/s, {e['gbs']:.0f} GB/s ({e['hbm_frac']:.2f} "
            f"HBM), {e['tflops']:.1f} TFLOP/s")
    return res


def vti_problem(torch, mms, synth, dev, n, nt, seed=9):
    """400^3 layered VTI medium: C2 at Courant 0.4 / sqrt(1 + 2 eps_max), Thomsen fields."""
    s = synth.wave_setup(n, nt, seed=seed, sponge_width=32)
    grid = mms.Grid(n, n, n)
    eps, delta = synth.thomsen_fields(n, n, n, seed + 1, sy=grid.sy)
    shrink = 1.0 / (1.0 + 2.0 * float(eps.max()))
    a = torch.from_numpy(1 + 2 * eps).to(dev)
    b = torch.from_numpy(np.sqrt(1 + 2 * delta).astype(np.float32)).to(dev)
    c2 = torch.from_numpy(s.c2).to(dev)
    f = torch.from_numpy(s.src_dt2f).to(dev)
    return s, grid, a, b, c2, f, shrink


def bench_vti(torch, mms, synth, dev, n=400, nt=1000):
    """Pseudo-acoustic VTI forward model, 400^3, 1000 steps, H traces recorded."""
    log(f"[bench] vti setup {n}^3 x {nt}")
    s, grid, a, b, c2, f, shrink = vti_problem(torch, mms, synth, dev, n, nt)
    traces = torch.zeros((nt, n, n), device=dev)
    w = mms.Wave(grid, c2, LAP, nt, shrink, s.sponge_width, s.sponge_alpha, s.sponge_faces,
                 s.src, f, traces)
    H = [grid.zeros(dev) for _ in range(2)]
    V = [grid.zeros(dev) for _ in range(2)]
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    w.record(0, H[0])
    for k in range(1, nt):
        w.vti_step(k, a, b, H[(k - 1) % 2], H[k % 2], H[(k + 1) % 2],
                   V[(k - 1) % 2], V[k % 2], V[(k + 1) % 2])
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    gpts = grid.points * (nt - 1) / (ms * 1e-3) / 1e9
    bpp = 36.0      # reads H, V at n and n-1, C2, a, b; writes H, V
    res = {"grid": [n, n, n], "steps": nt - 1, "ms_total": ms, "ms_per_step": ms / (nt - 1),
           "gpoints_s": gpts, "gbs": gpts * bpp, "hbm_frac": gpts * bpp / HBM_PEAK_GBS,
           "algorithmic_bytes_per_point": bpp,
           "trace_max_abs": float(traces.abs().max().item()),
           "finite": bool(torch.isfinite(H[nt % 2]).all().item())}
    log(f"[bench] vti: {gpts:.1f} Gpoints/s ({ms:.0f} ms, {gpts * bpp:.0f} GB/s)")
    return res


IMAGE_BLOCK = 8   # steps summed in FP32 before each FP64 image update (RTM forward)
TTI_SIGMA = 0.1   # v_sz^2 / v_pz^2: keeps the pseudo-acoustic pair stable under varying tilt


def tti_problem(torch, mms, synth, dev, n, nt, seed=11):
    """400^3 TTI medium: layered velocity, Thomsen fields, smooth tilt (0..45 deg) and
    azimuth; C2 scaled by 1/(1 + 2 eps_max)."""
    s = synth.wave_setup(n, nt, seed=seed, sponge_width=32)
    grid = mms.Grid(n, n, n)
    eps, delta = synth.thomsen_fields(n, n, n, seed + 1, sy=grid.sy)
    theta, phi = synth.tilt_fields(n, n, n, seed + 2, sy=grid.sy)
    shrink = 1.0 / (1.0 + 2.0 * float(eps.max()))
    t = mms.Tti(grid, *[torch.from_numpy(a).to(dev) for a in (eps, delta, theta, phi)],
                TTI_SIGMA, 1.0, [float(v) for v in synth.FIRST_DERIV_R4])
    w = mms.Wave(grid, torch.from_numpy(s.c2).to(dev), LAP, nt, shrink, s.sponge_width,
                 s.sponge_alpha, s.sponge_faces, s.src, torch.from_numpy(s.src_dt2f).to(dev))
    return s, grid, w, t


def bench_tti(torch, mms, synth, dev, n=400, nt=300):
    """Pseudo-acoustic TTI forward model, 400^3, 300 steps, p traces recorded."""
    log(f"[bench] tti setup {n}^3 x {nt}")
    s, grid, w, t = tti_problem(torch, mms, synth, dev, n, nt)
    traces = torch.zeros((nt, n, n), device=dev)
    w.set_traces(traces)
    P = [grid.zeros(dev) for _ in range(2)]
    Q = [grid.zeros(dev) for _ in range(2)]
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    w.record(0, P[0])
    for k in range(1, nt):
        w.tti_step(k, t, P[(k - 1) % 2], P[k % 2], P[(k + 1) % 2],
                   Q[(k - 1) % 2], Q[k % 2], Q[(k + 1) % 2])
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    gpts = grid.points * (nt - 1) / (ms * 1e-3) / 1e9
    bpp = 44.0      # fused minimum: p, q at n and n-1, C2, eps, delta, theta, phi; p, q out
    res = {"grid": [n, n, n], "steps": nt - 1, "ms_total": ms, "ms_per_step": ms / (nt - 1),
           "gpoints_s": gpts, "gbs": gpts * bpp, "hbm_frac": gpts * bpp / HBM_PEAK_GBS,
           "algorithmic_bytes_per_point": bpp, "two_pass_bytes_per_point": 84.0,
           "sigma": TTI_SIGMA, "trace_max_abs": float(traces.abs().max().item()),
           "finite": bool(torch.isfinite(P[nt % 2]).all().item())}
    log(f"[bench] tti: {gpts:.1f} Gpoints/s ({ms:.0f} ms, {gpts * bpp:.0f} GB/s at 44 B/pt)")
    return res


def bench_gradient(torch, mms, synth, dev, n=256, nt=1000, K=50):
    """Adjoint gradient of the receiver misfit w.r.t. v^2, 256^3, 1000 steps."""
    from paper_2507_11067_amd.autograd import Problem, misfit, propagate
    log(f"[bench] gradient setup {n}^3 x {nt}")
    s = synth.wave_setup(n, nt, seed=8, sponge_width=32)
    s0 = synth.wave_setup(n, nt, seed=None, sponge_width=32, dt=s.dt)
    grid = mms.Grid(n, n, n)
    f = torch.from_numpy(s.src_dt2f).to(dev)

    def mgrid(v):
        m = synth.padded_zeros(n, n, n)
        synth.interior(m, n, n, n)[...] = (v ** 2).astype(np.float32)
        return torch.from_numpy(m).to(dev)

    prob = Problem(grid, tuple(LAP), nt, s.h, s.dt, s.src, f, s.sponge_width, s.sponge_alpha,
                   s.sponge_faces, checkpoint_every=K)
    z = grid.zeros(dev)
    with torch.no_grad():
        d_obs = propagate(mgrid(s0.v), z, z, prob)
    # one untimed pass first, so that the timed pass reuses the caching allocator's blocks:
    # the first pass's device allocations (about 7 GB of checkpoints and segment levels)
    # and their first-touch mapping cost 40-110 ms and are not part of a step
    mw = mgrid(s.v).requires_grad_(True)
    misfit(propagate(mw, z, z, prob), d_obs).backward()
    del mw
    m = mgrid(s.v).requires_grad_(True)
    torch.cuda.synchronize()
    a, b, c = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    a.record()
    traces = propagate(m, z, z, prob)
    J = misfit(traces, d_obs)
    b.record()
    J.backward()
    c.record()
    torch.cuda.synchronize()
    fwd_ms, bwd_ms = a.elapsed_time(b), b.elapsed_time(c)
    pts = grid.points * (nt - 1)
    res = {"grid": [n, n, n], "steps": nt - 1, "checkpoint_every": K, "J": float(J.item()),
           "forward_ms": fwd_ms, "backward_ms": bwd_ms,
           "gpoints_s": pts / ((fwd_ms + bwd_ms) * 1e-3) / 1e9,
           "recomputed_steps": prob.stats.get("recomputed_steps"),
           "adjoint_form": prob.stats.get("adjoint_form")}
    log(f"[bench] gradient: fwd {fwd_ms:.0f} ms, bwd {bwd_ms:.0f} ms")
    # the same gradient with every forward level resident (nt + 1 grids in HBM, no recompute):
    # the trade that one GPU's 288 GB allows at this size; one untimed pass first as above
    prob.store_all = True
    mw = mgrid(s.v).requires_grad_(True)
    misfit(propagate(mw, z, z, prob), d_obs).backward()
    mw = mgrid(s.v).requires_grad_(True)
    torch.cuda.synchronize()
    a.record()
    J2 = misfit(propagate(mw, z, z, prob), d_obs)
    b.record()
    J2.backward()
    c.record()
    torch.cuda.synchronize()
    f2, b2 = a.elapsed_time(b), b.elapsed_time(c)
    gdiff = float(((mw.grad - m.grad).abs().max() / m.grad.abs().max()).item())
    res["store_all"] = {"forward_ms": f2, "backward_ms": b2,
                        "gpoints_s": pts / ((f2 + b2) * 1e-3) / 1e9,
                        "resident_gb": (nt + 1) * grid.shape[0] * grid.shape[1] * grid.shape[2] * 4 / 1e9,
                        "recomputed_steps": prob.stats.get("recomputed_steps"),
                        "grad_rel_diff_vs_checkpointed": gdiff}
    prob.store_all = False
    del mw, J2
    log(f"[bench] gradient, all levels resident: fwd {f2:.0f} ms, bwd {b2:.0f} ms "
        f"(gradient rel diff vs checkpointed {gdiff:.1e})")
    # dot-product test of the adjoint at the full size: A (u0, u1) -> traces (no source) at
    # fixed m, x = two smooth random levels.  y = A x + the misfit residual scaled to the norm
    # of A x (gated, 1e-5 relative); y = the residual alone is also reported: x and y are then
    # unrelated, |<A x, y>| is a small fraction of |A x| |y| and the relative error is
    # amplified by its inverse, so that case is measured by |lhs - rhs| / (|A x| |y|)
    r = torch.empty_like(traces)
    mms.flat_misfit(traces.detach(), d_obs, resid=r)
    w = mms.Wave(grid, m.detach(), LAP, nt, (s.dt / s.h) ** 2, s.sponge_width, s.sponge_alpha,
                 s.sponge_faces, s.src, None, torch.zeros((nt, n, n), device=dev))
    u0 = torch.from_numpy(synth.smooth_random_grid(81, n, n, n, sigma=3.0)).to(dev)
    u1 = torch.from_numpy(synth.smooth_random_grid(82, n, n, n, sigma=3.0)).to(dev)
    bufs = [u0.clone(), u1.clone(), grid.zeros(dev)]
    w.record(0, bufs[0])
    w.forward(1, nt, [bufs[i % 3] for i in range(nt + 1)])
    ax = w.traces.clone()
    nax, nr = mms.flat_dot(ax) ** 0.5, mms.flat_dot(r) ** 0.5
    ys = {"ax_plus_residual": (ax + r * (nax / nr)).contiguous(), "residual": r}
    lam = [grid.zeros(dev) for _ in range(3)]
    for form in ("mu", "lam"):
        for yname, y in ys.items():
            for b_ in lam:
                b_.zero_()
            if form == "lam":
                w.adjoint(nt - 1, 0, [lam[i % 3] for i in range(nt + 2)], resid=y)
            else:
                w.adjoint_mu(nt - 1, 0, [lam[i % 3] for i in range(nt + 2)], resid=y)
                w.scale_mu(lam[0], lam[0], -1)
                w.scale_mu(lam[1], lam[1], -1)
            lhs = mms.flat_dot(ax, y)
            rhs = mms.dot(u0, lam[0], grid) + mms.dot(u1, lam[1], grid)
            ny = mms.flat_dot(y) ** 0.5
            e = {"form": form, "y": yname, "lhs": lhs, "rhs": rhs,
                 "rel": abs(lhs - rhs) / abs(lhs), "normalised": abs(lhs - rhs) / (nax * ny),
                 "lhs_over_norms": abs(lhs) / (nax * ny)}
            key = "dot_test" if (form == "mu" and yname == "ax_plus_residual") else \
                  f"dot_test_{form}_{yname}"
            res[key] = e
            log(f"[bench] dot test, {form} form, y = {yname}: rel {e['rel']:.2e}, normalised "
                f"{e['normalised']:.2e} (|lhs|/(|Ax||y|) {e['lhs_over_norms']:.1e})")
    res["dot_test"]["gate"] = 1e-5
    res["dot_test"]["pass"] = res["dot_test"]["rel"] <= 1e-5
    res["finite_differences"], res["taylor"] = gradient_checks(torch, mms, synth, prob, m, d_obs,
                                                               grid, dev)
    return res


def gradient_pass(torch, mms, synth, dev, n=256, nt=1000, K=50):
    """One forward + backward pass of the 256^3 x 1000 gradient workload, as a callable."""
    from paper_2507_11067_amd.autograd import Problem, misfit, propagate
    s = synth.wave_setup(n, nt, seed=8, sponge_width=32)
    s0 = synth.wave_setup(n, nt, seed=None, sponge_width=32, dt=s.dt)
    grid = mms.Grid(n, n, n)
    prob = Problem(grid, tuple(LAP), nt, s.h, s.dt, s.src, torch.from_numpy(s.src_dt2f).to(dev),
                   s.sponge_width, s.sponge_alpha, s.sponge_faces, checkpoint_every=K)

    def mgrid(v):
        m = synth.padded_zeros(n, n, n)
        synth.interior(m, n, n, n)[...] = (v ** 2).astype(np.float32)
        return torch.from_numpy(m).to(dev)

    z = grid.zeros(dev)
    with torch.no_grad():
        d_obs = propagate(mgrid(s0.v), z, z, prob)
    m_val = mgrid(s.v)

    def f():
        m = m_val.clone().requires_grad_(True)
        misfit(propagate(m, z, z, prob), d_obs).backward()
    return f


def gradient_checks(torch, mms, synth, prob, m, d_obs, grid, dev, npts=16, seed=84):
    """Central finite differences of J at 16 points drawn from the top decile of the
    (Gaussian-smoothed) |dJ/dm|, and a Taylor test along a smooth direction."""
    n, nt = grid.nx, prob.nt
    traces = torch.zeros((nt, grid.ny, grid.nx), device=dev)
    bufs = [grid.zeros(dev) for _ in range(3)]
    jout = torch.zeros(2, dtype=torch.float64, device=dev)

    def J_of(mt):
        w = prob.wave(mt, traces)
        for b_ in bufs:
            b_.zero_()
        w.record(0, bufs[0])
        w.forward(1, nt, [bufs[i % 3] for i in range(nt + 1)])
        return mms.check_result(mms.flat_misfit(traces, d_obs, out=jout))

    g = m.grad.detach()
    gi = grid.interior(g).cpu().numpy()
    mi = grid.interior(m.detach()).cpu().numpy()
    rng = np.random.default_rng(seed)
    # points from the top decile of the gradient smoothed at the bump's width, away from
    # the faces, and within two decades of its largest value: the gradient spans many
    # decades (it falls off with distance from source and receivers), and a directional
    # derivative <g, bump> far below the largest one sits at the rounding level of the
    # FP32 traces, where no finite difference can resolve it
    from scipy.ndimage import gaussian_filter
    gs = np.abs(gaussian_filter(gi.astype(np.float64), sigma=2.0, truncate=3.0))
    core = np.zeros_like(gs, dtype=bool)
    core[6:-6, 6:-6, 6:-6] = True
    cut = max(np.quantile(gs[core], 0.9), 1e-2 * float(gs[core].max()))
    cand = np.argwhere(core & (gs >= cut))
    if len(cand) < npts:
        cand = np.argwhere(core & (gs >= np.sort(gs[core])[-npts]))
    pick = cand[rng.choice(len(cand), npts, replace=False)]
    md = m.detach()
    # (a) one cell per point: in FP32 the trace change of a single-cell perturbation sits
    #     near the rounding level of the traces, so these numbers are reported, not gated;
    # (b) a Gaussian bump (sigma = 2 cells, 13^3 support) centred on each point: the
    #     directional derivative <g, bump> is compared with the central difference.
    sig, hw = 2.0, 6
    ax = np.arange(-hw, hw + 1)
    bump = np.exp(-(ax[:, None, None] ** 2 + ax[None, :, None] ** 2 + ax[None, None, :] ** 2)
                  / (2 * sig * sig))
    fd_rows = []
    for z_, y_, x_ in pick:
        z_, y_, x_ = (int(min(max(v, hw), n - 1 - hw)) for v in (z_, y_, x_))
        mi_c = float(mi[z_, y_, x_])
        row = {"point": [z_, y_, x_]}
        idx = (z_ + 4, y_ + 4, x_ + 4)
        eps = 5e-2 * mi_c
        mp = md.clone()
        mp[idx] += eps
        jp = J_of(mp)
        mp[idx] -= 2 * eps
        jm = J_of(mp)
        ga = float(gi[z_, y_, x_])
        row["cell_fd"], row["cell_adjoint"] = (jp - jm) / (2 * eps), ga
        row["cell_rel"] = abs(row["cell_fd"] - ga) / abs(ga)
        sl = (slice(z_ + 4 - hw, z_ + 5 + hw), slice(y_ + 4 - hw, y_ + 5 + hw),
              slice(x_ + 4 - hw, x_ + 5 + hw))
        db = torch.from_numpy((1e-2 * mi_c * bump).astype(np.float32)).to(dev)
        mp = md.clone()
        mp[sl] += db
        jp = J_of(mp)
        mp[sl] -= 2 * db
        jm = J_of(mp)
        fdb = (jp - jm) / 2.0
        gdb = float(np.sum(gi[z_ - hw:z_ + hw + 1, y_ - hw:y_ + hw + 1, x_ - hw:x_ + hw + 1]
                           .astype(np.float64) * db.cpu().numpy().astype(np.float64)))
        row["bump_fd"], row["bump_adjoint"] = fdb, gdb
        row["bump_rel"] = abs(fdb - gdb) / abs(gdb)
        fd_rows.append(row)
    cr = [r["cell_rel"] for r in fd_rows]
    br = [r["bump_rel"] for r in fd_rows]
    fdres = {"points": fd_rows, "selection": "top decile of |smoothed g| and >= 1e-2 of its max",
             "cell_eps_rel": 5e-2, "bump_sigma_cells": sig,
             "bump_amp_rel": 1e-2, "cell_rel_median": float(np.median(cr)),
             "cell_rel_max": float(np.max(cr)), "bump_rel_median": float(np.median(br)),
             "bump_rel_max": float(np.max(br)), "bump_gate": 5e-2,
             "bump_pass": bool(np.max(br) <= 5e-2)}
    log(f"[bench] FD at 16 points of large gradient: single cell rel median {fdres['cell_rel_median']:.2e}"
        f" max {fdres['cell_rel_max']:.2e}; bump rel median {fdres['bump_rel_median']:.2e} "
        f"max {fdres['bump_rel_max']:.2e}")
    # Taylor test along a smooth direction dm (max |dm| = 1 % of mean m)
    dm = torch.from_numpy(synth.smooth_random_grid(85, n, n, n, sigma=4.0)).to(dev)
    scale = 0.01 * float(np.mean(mi))
    dm.mul_(scale)
    gdm = mms.dot(g, dm, grid)
    J0 = J_of(md)
    rows = []
    for eps in (1.0, 0.5, 0.25, 0.125):
        Je = J_of(md + eps * dm)
        rows.append({"eps": eps, "J": Je, "first_order_ratio": (Je - J0) / (eps * gdm),
                     "remainder": abs(Je - J0 - eps * gdm)})
    for a_, b_ in zip(rows, rows[1:]):
        b_["remainder_ratio"] = a_["remainder"] / b_["remainder"] if b_["remainder"] else None
    log("[bench] Taylor: " + ", ".join(f"eps {r['eps']}: J'/gdm {r['first_order_ratio']:.5f}"
                                       for r in rows))
    return fdres, {"J0": J0, "g_dot_dm": gdm, "rows": rows}


def errors_chunked(got, ref, chunk=32):
    """Normwise (max, RMS) errors of two [z][y][x] arrays, accumulated over z chunks in FP64."""
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


def cpu_baseline_leg(torch, mms, synth, grid, x, x_np, n, dev, result, c_star, c_box2, c_box4,
                     c_box3, check):
    """The FP64 oracle on the host cores.  (a) Timed: one step of the headline workload (star
    r4, box r2, box r4) over the full 512^3 grid -- the cpu_baseline figure.  (b) Untimed
    unless already computed: full-grid oracle sweeps of every other 512^3 kernel of this run.
    Each GPU sweep is run again into a scratch grid and compared with its reference at every
    interior point; the errors go into the kernels / split_mfma / table1 / config0 entries."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    x64 = x_np.astype(np.float64)
    I = lambda a: a[4:4 + n, 4:4 + n, 4:4 + n]
    out = grid.zeros(dev)

    def gpu(shape, r, c, prec="fp32"):
        mms.stencil_apply(x, out, grid, shape, r, c, precision=prec)
        torch.cuda.synchronize()
        return I(out.cpu().numpy())

    def record(entry, shape, r, c, ref, prec="fp32"):
        if entry is not None:
            entry["rel_max"], entry["rel_rms"] = errors_chunked(gpu(shape, r, c, prec), ref)
            entry["error_points"] = n ** 3

    log(f"[bench] cpu baseline: oracle, one headline step over {n}^3, {threads} threads")
    t0 = time.perf_counter()
    refs = {"star": oracle.star(x64, n, n, n, 4, c_star)}
    refs["box2"] = oracle.box(x64, n, n, n, 2, c_box2)
    refs["box4"] = oracle.box(x64, n, n, n, 4, c_box4)
    dt = time.perf_counter() - t0
    log(f"[bench] cpu baseline: {dt:.1f} s")
    base = {"value": 3 * n ** 3 / dt / 1e9, "unit": "Gpoints/s", "cores": min(threads, cores),
            "kind": "oracle",
            "sample": f"one headline step (one FP64 sweep each of star r4, box r2, box r4) over "
                      f"the full {n}x{n}x{n} input; {dt:.1f} s"}
    if not check:
        return base
    log("[bench] errors against the oracle at every interior point")
    kern, split, t1 = result["kernels"], result.get("split_mfma", {}), result.get("table1", {})
    for name, shape, r, c in (("star", "star", 4, c_star), ("box2", "box", 2, c_box2),
                              ("box4", "box", 4, c_box4)):
        ref = I(refs.pop(name))
        record(kern.get(name), shape, r, c, ref)
        if name == "box4":
            for prec in ("fp32", "bf16x3", "fp16x3s", "bf16x1"):
                record(split.get(f"box_r4_{prec}"), "box", 4, c, ref, prec)
        if name == "star":
            record(t1.get("3DStarR4"), "star", 4, c, ref)
        if name == "box2":
            record(t1.get("3DBoxR2"), "box", 2, c, ref)
        del ref
    if split:
        ref = I(oracle.box(x64, n, n, n, 3, c_box3))
        for prec in ("fp32", "bf16x3", "fp16x3s", "bf16x1"):
            record(split.get(f"box_r3_{prec}"), "box", 3, c_box3, ref, prec)
        del ref
    fns = {"star": oracle.star, "box": oracle.box, "star2d": oracle.star2d, "box2d": oracle.box2d}
    for name, (shape, r, c, _) in table1_kernels(synth).items():
        if name in t1 and "rel_max" not in t1[name]:
            ref = I(fns[shape](x64, n, n, n, r, c))
            record(t1[name], shape, r, c, ref)
            del ref
    for k in ("star", "box2", "box4"):
        log(f"[bench] {k}: rel_max {kern[k]['rel_max']:.2e} rel_rms {kern[k]['rel_rms']:.2e}")
    for k, e in split.items():
        if isinstance(e, dict) and "rel_max" in e:
            log(f"[bench] {k}: rel_max {e['rel_max']:.2e} rel_rms {e['rel_rms']:.2e}")
    if "config0" in result:
        m = 64
        g0 = mms.Grid(m, m, m)
        x0 = synth.uniform_grid(1, m, m, m, sy=g0.sy)
        o0 = g0.zeros(dev)
        mms.stencil_apply(torch.from_numpy(x0).to(dev), o0, g0, "star", 4, c_star)
        torch.cuda.synchronize()
        ref = oracle.star(x0.astype(np.float64), m, m, m, 4, c_star)
        J = lambda a: a[4:4 + m, 4:4 + m, 4:4 + m]
        result["config0"]["rel_max"], result["config0"]["rel_rms"] = errors_chunked(
            J(o0.cpu().numpy()), J(ref))
    return base


# ---------------------------------------------------------------- counters
PROFILES = os.path.join(ROOT, "profiles")
COUNTERS_JSON = os.path.join(PROFILES, "counters_512.json")
# kernel (bench --only name) -> (source file, kernel symbol substring, algorithmic bytes per point)
COUNTED = {
    "copy": (None, "copyBuffer", 8.0),
    "star": ("star.hip", "star_kernel<4", 8.0),
    "box2": ("box_valu.hip", "box_valu_kernel<2", 8.0),
    "box4": ("box_valu.hip", "box_valu_kernel<4", 8.0),
    "box3": ("box_valu.hip", "box_valu_kernel<3", 8.0),
    "box4_bf16x3": ("box_mfma.hip", "box_mfma_kernel<4, 1,", 8.0),
    "box3_bf16x3": ("box_mfma.hip", "box_mfma_kernel<3, 1,", 8.0),
    "wave": ("wave.hip", "wave_kernel<4, 0, 64", 16.0),   # 400^3 forward step, no image
    "vti": ("vti.hip", "vti_kernel<4", 36.0),                # 400^3 VTI step
    "tti_dz": ("tti.hip", "tti_dz_kernel<4", 24.0),          # 400^3 TTI pass 1 (padded rows)
    "tti": ("tti.hip", "tti_kernel<4", 60.0),                # 400^3 TTI pass 2
    # 256^3 gradient workload: the mu-form adjoint pass (mu^{n+1}, mu^{n+2}, C2 read; mu^n
    # written) and the gradient pass (u^n, mu^{n+1} read; FP32 block partial written at the
    # first step of a block of 8, read and written in the next 6, read at the last, which
    # reads and writes the FP64 sum: (12 + 6 * 16 + 28) / 8 = 17 B per point and launch)
    "adjmu": ("wave.hip", "wave_kernel<4, 4, 64", 16.0),
    "grad": ("wave.hip", "wave_kernel<4, 3, 64", 17.0),
}
COUNTED_POINTS = {"wave": 400 ** 3, "vti": 400 ** 3, "tti_dz": 400 ** 3, "tti": 400 ** 3,
                  "adjmu": 256 ** 3, "grad": 256 ** 3}
# the --only command that launches each counted kernel, and its --steps / --warmup when the
# defaults do not fit (one gradient run is 1000 forward and 1000 adjoint steps)
COUNTED_ONLY = {"tti_dz": "tti", "adjmu": "gradient", "grad": "gradient"}
ONLY_STEPS = {"gradient": ("1", "0")}


def source_sha(fname):
    import hashlib
    if fname is None:
        return None
    path = os.path.join(ROOT, "paper_2507_11067_amd", "csrc", fname)
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def traffic_for(name):
    """HBM bytes per launch from the committed counter summary, if that summary was taken
    on the current source of the kernel (else None)."""
    try:
        d = json.load(open(COUNTERS_JSON))
    except (OSError, ValueError):
        return None
    e = d.get("kernels", {}).get(name)
    if not e or e.get("source_sha") != source_sha(COUNTED[name][0]):
        return None
    return e["hbm_bytes_per_launch"]


# utilisation passes (one rocprofv3 run each; derived counters computed by rocprofv3)
UTIL_PASSES = {
    "box4_bf16x3": "MfmaUtil SQ_INSTS_VALU_MFMA_MOPS_BF16 LDSBankConflict",
    "box3_bf16x3": "MfmaUtil SQ_INSTS_VALU_MFMA_MOPS_BF16 LDSBankConflict",
    "box4": "VALUBusy SQ_INSTS_VALU_FMA_F32 LDSBankConflict",
    "box3": "VALUBusy SQ_INSTS_VALU_FMA_F32 LDSBankConflict",
    "box2": "VALUBusy SQ_INSTS_VALU_FMA_F32 LDSBankConflict",
    "star": "VALUBusy LDSBankConflict",
}


def util_for(name):
    """Utilisation counters of one kernel from the committed summary (None if stale)."""
    try:
        d = json.load(open(COUNTERS_JSON))
    except (OSError, ValueError):
        return None
    e = d.get("util", {}).get(name)
    if not e or e.get("source_sha") != source_sha(COUNTED[name][0]):
        return None
    return {k: v for k, v in e.items() if k not in ("source", "source_sha", "command")}


def _counter_means(csv_path, substr):
    import csv
    acc = {}
    for r in csv.DictReader(open(csv_path)):
        if substr in r["Kernel_Name"]:
            acc.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def _counter_mean(csv_path, substr):
    import csv
    vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(csv_path))
            if substr in r["Kernel_Name"]]
    return (sum(vals) / len(vals), len(vals)) if vals else (None, 0)


def _stats_mean_ns(csv_path, substr):
    import csv
    for r in csv.DictReader(open(csv_path)):
        if substr in r["Name"]:
            return float(r["AverageNs"]), int(r["Calls"])
    return None, 0


def collect_counters(args):
    """rocprofv3 runs (each a child process of this one, which never touches the GPU):
    a kernel trace of the headline bench command, then FETCH_SIZE and WRITE_SIZE per kernel.
    The copy kernel of known size calibrates each counter: bytes = counter * factor."""
    import glob
    import subprocess
    out_root = os.path.abspath(args.collect_dir)
    os.makedirs(out_root, exist_ok=True)
    py = sys.executable

    def prof(tag, extra, bench_args, limit):
        d = os.path.join(out_root, tag)
        cmd = ["timeout", "-s", "KILL", str(limit), "rocprofv3"] + extra + \
              ["--output-format", "csv", "-d", d, "-o", "run", "--", py,
               os.path.join(ROOT, "bench.py")] + bench_args
        log("[collect] " + " ".join(cmd[4:]))
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                           env=dict(os.environ, TMPDIR="/tmp"))
        if r.returncode != 0:
            log(r.stdout[-3000:])
            raise SystemExit(f"rocprofv3 step {tag} failed with status {r.returncode}")
        return d, " ".join(["rocprofv3"] + extra + ["--", "python", "bench.py"] + bench_args)

    def find(d, suffix):
        f = glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)
        if not f:
            raise SystemExit(f"no {suffix} under {d}")
        return f[0]

    summary = {"kernels": {}, "commands": {}}
    # 1. kernel trace of the headline command
    targs = ["--steps", "60", "--warmup", "40", "--skip",
             "config0,split,table1,rtm,vti,tti,gradient,cpu,check"]
    d, cmd = prof("trace_headline", ["--kernel-trace", "--stats"], targs, 300)
    stats = find(d, "_kernel_stats.csv")
    summary["commands"]["trace_headline"] = cmd
    summary["trace_headline"] = {}
    for name in ("star", "box2", "box4"):
        ns, calls = _stats_mean_ns(stats, COUNTED[name][1])
        summary["trace_headline"][name] = {"avg_ns": ns, "calls": calls}
    # 1b. kernel traces of the single-kernel commands (split MFMA boxes, wave, VTI)
    summary["trace_only"] = {}
    traced = {}
    for name in ("box4_bf16x3", "box3_bf16x3", "wave", "vti", "tti_dz", "tti", "adjmu", "grad"):
        only = COUNTED_ONLY.get(name, name)
        if only not in traced:        # one run serves every kernel its command launches
            st, wu = ONLY_STEPS.get(only, ("200", "40"))
            traced[only] = prof(f"trace_{only}", ["--kernel-trace", "--stats"],
                                ["--only", only, "--steps", st, "--warmup", wu], 120)
        d, cmd = traced[only]
        ns, calls = _stats_mean_ns(find(d, "_kernel_stats.csv"), COUNTED[name][1])
        summary["trace_only"][name] = {"avg_ns": ns, "calls": calls, "command": cmd,
                                       "source_sha": source_sha(COUNTED[name][0])}
    # 2. counters per kernel, copy first (calibration)
    n = 512
    sy = ((n + 8 + 31) // 32) * 32                      # the headline layout (Grid.aligned)
    grid_bytes = (n + 8) * (n + 8) * sy * 4             # one padded FP32 grid
    factors = {}
    counted = {}
    for name, (src, sym, bpp) in COUNTED.items():
        e = {"source": src, "source_sha": source_sha(src), "symbol": sym}
        only = COUNTED_ONLY.get(name, name)
        for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
            if (only, ctr) not in counted:
                st, wu = ONLY_STEPS.get(only, ("3", "1"))
                counted[(only, ctr)] = prof(f"{only}_{ctr}", ["--pmc", ctr],
                                            ["--only", only, "--steps", st, "--warmup", wu], 90)
            d, cmd = counted[(only, ctr)]
            kib, cnt = _counter_mean(find(d, "_counter_collection.csv"), sym)
            e[ctr.lower() + "_kib"] = kib
            summary["commands"][f"{name}_{ctr}"] = cmd
            if name == "copy":
                # the copy reads and writes one padded grid
                factors[ctr] = grid_bytes / (kib * 1024.0)
        summary["kernels"][name] = e
    summary["factors"] = factors
    # 3. utilisation counters
    summary["util"] = {}
    for name, ctrs in UTIL_PASSES.items():
        src, sym, _ = COUNTED[name]
        d, cmd = prof(f"{name}_util", ["--pmc"] + ctrs.split(),
                      ["--only", name, "--steps", "3", "--warmup", "1"], 90)
        e = {"source": src, "source_sha": source_sha(src), "command": cmd}
        e.update(_counter_means(find(d, "_counter_collection.csv"), sym))
        summary["util"][name] = e
    for name, e in summary["kernels"].items():
        fb = e["fetch_size_kib"] * 1024.0 * factors["FETCH_SIZE"]
        wb = e["write_size_kib"] * 1024.0 * factors["WRITE_SIZE"]
        e["fetch_bytes"], e["write_bytes"] = fb, wb
        e["hbm_bytes_per_launch"] = fb + wb
        e["algorithmic_bytes_per_launch"] = COUNTED[name][2] * COUNTED_POINTS.get(name, n ** 3) \
            if name != "copy" else 2.0 * grid_bytes
        e["traffic_over_algorithmic"] = (fb + wb) / e["algorithmic_bytes_per_launch"]
    os.makedirs(PROFILES, exist_ok=True)
    json.dump(summary, open(COUNTERS_JSON, "w"), indent=1)
    lines = ["# rocprofv3 summaries behind bench.py's roofline (512^3 headline grid)",
             "# produced by: python bench.py --collect  (runs the commands below as children)",
             ""]
    lines.append("## kernel trace (--kernel-trace --stats) of the headline command")
    lines.append("command: " + summary["commands"]["trace_headline"])
    for k, v in summary["trace_headline"].items():
        lines.append(f"  {k:6s} {COUNTED[k][1]:28s} calls {v['calls']:4d}  avg "
                     f"{(v['avg_ns'] or 0) / 1e3:9.2f} us")
    lines.append("")
    lines.append("## kernel traces (--kernel-trace --stats) of single-kernel commands")
    for k, v in summary["trace_only"].items():
        lines.append(f"  {k:12s} {COUNTED[k][1]:28s} calls {v['calls']:4d}  avg "
                     f"{(v['avg_ns'] or 0) / 1e3:9.2f} us   command: {v['command']}")
    lines.append("")
    lines.append("## HBM counters (per dispatch; KiB as read, bytes after copy calibration)")
    lines.append(f"calibration: plain copy of one {n + 8}x{n + 8}x{sy} FP32 grid ({grid_bytes} B each way): "
                 f"FETCH factor {factors['FETCH_SIZE']:.4f}, WRITE factor "
                 f"{factors['WRITE_SIZE']:.4f}")
    for name, e in summary["kernels"].items():
        lines.append(f"  {name:12s} FETCH {e['fetch_size_kib']:12.1f} KiB  WRITE "
                     f"{e['write_size_kib']:12.1f} KiB  -> {e['hbm_bytes_per_launch'] / 1e6:9.1f} MB"
                     f"  ({e['traffic_over_algorithmic']:.3f} x algorithmic)  src {e['source']} "
                     f"{e['source_sha']}")
        lines.append(f"      commands: {summary['commands'][name + '_FETCH_SIZE']} ; "
                     f"{summary['commands'][name + '_WRITE_SIZE']}")
    lines.append("")
    lines.append("## utilisation counters (per dispatch, derived ones as computed by rocprofv3)")
    for name, e in summary["util"].items():
        vals = "  ".join(f"{k} {v:.4g}" for k, v in e.items()
                         if k not in ("source", "source_sha", "command"))
        lines.append(f"  {name:12s} {vals}  src {e['source']} {e['source_sha']}")
        lines.append(f"      command: {e['command']}")
    open(os.path.join(PROFILES, "counters_512.txt"), "w").write("\n".join(lines) + "\n")
    # copies beside the raw rocprofv3 output, for runs whose tree is not kept
    json.dump(summary, open(os.path.join(out_root, "counters_512.json"), "w"), indent=1)
    open(os.path.join(out_root, "counters_512.txt"), "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def profile_only(args, torch, mms, synth, grid, x, outs, sweeps, c_box4, c_box3, dev):
    """Launch one kernel family repeatedly (for rocprofv3 runs)."""
    k = args.only
    out = outs["box4"]
    if k in sweeps:
        f = sweeps[k]
    elif k.startswith("box4_") or k.startswith("box3_"):
        r = 4 if k.startswith("box4") else 3
        prec = k.split("_", 1)[1]
        c = c_box4 if r == 4 else c_box3
        f = lambda: mms.stencil_apply(x, out, grid, "box", r, c, precision=prec)
    elif k == "box3":
        f = lambda: mms.stencil_apply(x, out, grid, "box", 3, c_box3)
    elif k == "copy":
        ca = x.reshape(-1).clone()      # flat buffers of the grid's size, allocator-aligned
        cb = torch.empty_like(ca)
        f = lambda: cb.copy_(ca)
    elif k in table1_kernels(synth):
        shape, r, c, _ = table1_kernels(synth)[k]
        f = lambda: mms.stencil_apply(x, out, grid, shape, r, c)
    elif k == "tti":
        _, g4, wt, tt = tti_problem(torch, mms, synth, dev, 400, 64)
        P = [g4.zeros(dev) for _ in range(2)]
        Q = [g4.zeros(dev) for _ in range(2)]
        it = [0]

        def f():
            i = it[0] % 60 + 1
            wt.tti_step(i, tt, P[(i - 1) % 2], P[i % 2], P[(i + 1) % 2],
                        Q[(i - 1) % 2], Q[i % 2], Q[(i + 1) % 2])
            it[0] += 1
    elif k == "vti":
        n = 400
        s, g4, ta, tb, c2, fsrc, shrink = vti_problem(torch, mms, synth, dev, n, 64)
        w = mms.Wave(g4, c2, LAP, 64, shrink, s.sponge_width, s.sponge_alpha, s.sponge_faces,
                     s.src, fsrc, None, None)
        H = [g4.zeros(dev) for _ in range(2)]
        V = [g4.zeros(dev) for _ in range(2)]
        it = [0]

        def f():
            i = it[0] % 60 + 1
            w.vti_step(i, ta, tb, H[(i - 1) % 2], H[i % 2], H[(i + 1) % 2],
                       V[(i - 1) % 2], V[i % 2], V[(i + 1) % 2])
            it[0] += 1
    elif k == "gradient":
        f = gradient_pass(torch, mms, synth, dev)
    elif k == "wave":
        n = 400
        s = synth.wave_setup(n, 64, seed=7, sponge_width=32)
        g4 = mms.Grid(n, n, n)
        w = mms.Wave(g4, torch.from_numpy(s.c2).to(dev), LAP, 64, 1.0, s.sponge_width,
                     s.sponge_alpha, s.sponge_faces, s.src,
                     torch.from_numpy(s.src_dt2f).to(dev), None, None)
        bufs = [g4.zeros(dev) for _ in range(3)]
        it = [0]

        def f():
            i = it[0] % 60 + 1
            w.step(i, bufs[(i - 1) % 3], bufs[i % 3], bufs[(i + 1) % 3])
            it[0] += 1
    else:
        raise SystemExit(f"unknown --only {k}")
    for _ in range(args.warmup):
        f()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(args.steps):
        f()
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / args.steps
    print(json.dumps({"only": k, "steps": args.steps, "ms_per_launch": ms}), flush=True)


if __name__ == "__main__":
    main()
