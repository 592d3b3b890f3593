"""Host-side checks of bench.py's profiling tables: every kernel it counts exists in the
source it names, with the template arguments the profiler's symbol match expects, and every
--only command it launches is one bench.py knows (CPU only, no GPU calls)."""
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2507_11067_amd", "csrc")


def load_bench():
    sys.argv = ["bench.py"]
    sys.path.insert(0, ROOT)
    import bench
    return bench


def test_counted_symbols_match_sources():
    bench = load_bench()
    wave = open(os.path.join(CSRC, "wave.hip")).read()
    modes = dict((k, int(v)) for k, v in re.findall(r"(MODE_[A-Z]+) = (\d+)", wave))
    expect_mode = {"wave": "MODE_FWD", "adjmu": "MODE_ADJMU", "grad": "MODE_GRAD"}
    for name, (src, sym, bpp) in bench.COUNTED.items():
        assert bpp > 0
        if src is None:
            continue
        text = open(os.path.join(CSRC, src)).read()
        kernel = sym.split("<")[0]
        assert re.search(r"\b%s\s*\(" % kernel, text), (name, kernel, src)
        if name in expect_mode:
            # symbol "wave_kernel<R, MODE, TX": the mode number of that pass
            args = [a.strip() for a in sym.split("<")[1].split(",")]
            assert int(args[1]) == modes[expect_mode[name]], (name, sym)


def test_only_commands_are_known():
    bench = load_bench()
    src = open(os.path.join(ROOT, "bench.py")).read()
    for name in bench.COUNTED:
        only = bench.COUNTED_ONLY.get(name, name)
        known = (only == "copy" or only in ("star", "box2", "box4") or
                 re.match(r"box[34]_", only) or f'k == "{only}"' in src)
        assert known, (name, only)
    for only, (steps, warmup) in bench.ONLY_STEPS.items():
        assert int(steps) >= 1 and int(warmup) >= 0
