"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only) and run over its entry points on small seeded inputs:
plain and given plans with fallback codes, periodic linearisation, output
tensors, relative volume, the primitives and the argument checks. Any invalid
access, leak or undefined operation aborts the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = tmp_path / "oracle_asan"
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fopenmp", "-o", str(exe),
           os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), os.path.join(ROOT, "oracle", "bernnn_oracle.c"),
           "-lm"]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "all calls clean" in r.stdout


SOURCES = ("api", "affine", "convert", "compose", "mlp", "simplex", "volume", "noalloc", "predictor")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="needs the ROCm compilers")
@pytest.mark.skipif(os.path.exists("/dev/kfd"), reason="host-only build: run where no GPU runtime registers code")
def test_c_abi_host_paths_under_asan_ubsan(tmp_path):
    """The library's host code built without device code (hipcc host pass
    only) and with the sanitizers, linked into a C driver that exercises the
    paths needing no GPU: argument checks, status strings, defaults, and the
    predictor file reader on damaged files. The empty device-code images the
    host pass leaves undefined are supplied as zero-filled arrays (no kernel
    is launched)."""
    csrc = os.path.join(ROOT, "paper_2211_14438_amd", "csrc")
    inc = os.path.join(ROOT, "include")
    procs, objs = [], []
    for s in SOURCES:
        o = str(tmp_path / f"{s}.o")
        objs.append(o)
        procs.append(subprocess.Popen([HIPCC, "--cuda-host-only", "-O1", "-g", "-fno-omit-frame-pointer", *SAN, "-fPIC",
                                       "-std=c++17", "-I", inc, "-c", os.path.join(csrc, f"{s}.hip"), "-o", o],
                                      stdout=subprocess.PIPE, stderr=subprocess.PIPE))
    for p in procs:
        _, err = p.communicate(timeout=600)
        assert p.returncode == 0, err.decode()[-3000:]
    und = subprocess.run(["nm", "-u", *objs], capture_output=True, text=True, check=True).stdout
    images = sorted({w for w in und.split() if w.startswith("__hip_fatbin_")})
    stubs = tmp_path / "images.c"
    stubs.write_text("".join(f"const char {s}[64] __attribute__((aligned(4096))) = {{0}};\n" for s in images))
    drv = str(tmp_path / "driver.o")
    subprocess.run([CLANG, "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-I",
                    inc, "-c", os.path.join(ROOT, "tests", "sanitize", "host_driver.c"), "-o", drv], check=True)
    subprocess.run([CLANG, "-c", str(stubs), "-o", str(tmp_path / "images.o")], check=True)
    exe = str(tmp_path / "host_asan")
    r = subprocess.run([HIPCC, *SAN, "-o", exe, drv, *objs, str(tmp_path / "images.o")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "all calls clean" in r.stdout
