"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two builds go to a temporary directory: the FP64 oracle with gcc -fsanitize=address,undefined,
and libmmstencil.so from the same HIP sources with the sanitizers on the host side only (the
GPU code is built as usual; nothing here launches a kernel).  The oracle pins and the ABI
tests then run against them in child processes with the sanitizer runtime preloaded; any
report fails the child (UBSan halts on the first error, ASan aborts by default)."""
import concurrent.futures as cf
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address", "-fsanitize=undefined"]


def _runtime(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def _child(env_extra, args):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:detect_odr_violation=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["OMP_NUM_THREADS"] = "4"
    probe = ("import sys;m=open('/proc/self/maps').read();"
             "sys.exit(0 if ('asan' in m) else 3)")
    r0 = subprocess.run([sys.executable, "-c", probe], env=env, cwd=ROOT)
    assert r0.returncode == 0, "sanitizer runtime not loaded in the child"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider"] + args,
                       env=env, cwd=ROOT, capture_output=True, text=True)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail
    return tail


def test_oracle_pins_under_asan_ubsan(tmp_path):
    libasan = _runtime(["gcc", "-print-file-name=libasan.so"])
    if libasan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = str(tmp_path / "libmms_oracle_san.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer"] + SAN +
                          ["-fno-sanitize-recover=undefined", "-fopenmp", "-fPIC", "-shared",
                           "-std=c11", "-Wall", "-o", lib,
                           os.path.join(ROOT, "oracle", "mms_oracle.c"), "-lm"])
    out = _child({"MMS_ORACLE_LIB": lib, "LD_PRELOAD": libasan}, ["tests/test_oracle_pins.py"])
    assert "passed" in out


def test_abi_validation_under_asan_ubsan(tmp_path):
    sys.path.insert(0, ROOT)
    from paper_2507_11067_amd import _build as B
    hipcc = B._hipcc()
    clang = os.path.join(os.path.dirname(os.path.realpath(hipcc)), "..", "lib", "llvm", "bin",
                         "clang")
    rt = _runtime([clang, "-print-file-name=libclang_rt.asan-x86_64.so"]) if os.path.exists(clang) \
        else None
    if rt is None:
        rt = _runtime(["/opt/rocm/llvm/bin/clang", "-print-file-name=libclang_rt.asan-x86_64.so"])
    if rt is None:
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    host_san = []
    for f in SAN:                        # host pass only: the GPU code is built as usual
        host_san += ["-Xarch_host", f]
    flags = B.HIPFLAGS + ["-g", "-fno-omit-frame-pointer"] + host_san

    def comp(src):
        obj = str(tmp_path / (src + ".o"))
        r = subprocess.run([hipcc] + flags + ["-c", os.path.join(B.CSRC, src), "-o", obj],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        return obj

    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(comp, B.SOURCES))
    lib = str(tmp_path / "libmmstencil_san.so")
    subprocess.check_call([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC"] + host_san +
                          ["-o", lib] + objs)
    out = _child({"MMS_SANITIZED_LIB": lib, "LD_PRELOAD": rt},
                 ["-p", "tests.sanitized_lib_plugin", "tests/test_abi.py"])
    assert "passed" in out
