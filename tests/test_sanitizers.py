"""CPU sanitizer runs (AddressSanitizer + UndefinedBehaviorSanitizer) of the
host-side code: the serial oracle and the multi-core CPU baseline built with
g++, and libhf's host code (argument checks, sizing, the batch planner)
built with hipcc, whose device code is untouched (every -fsanitize= goes to
the host pass only).  Each driver exercises its code on seeded inputs and
edge cases; a sanitizer report or a failed check fails the test.  No GPU is
used."""
import os
import shutil
import subprocess
import concurrent.futures as cf

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2010_10039_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
SAN = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


def _clean(r):
    out = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-3000:]


def test_oracle_and_cpu_baseline_under_sanitizers(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not found")
    exe = str(tmp_path / "oracle_and_cpu_check")
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
    oracle_obj = str(tmp_path / "huff_oracle.o")
    _run(["gcc", *flags, "-std=c99", "-c", os.path.join(ROOT, "oracle", "huff_oracle.c"), "-o", oracle_obj])
    _run(["g++", *flags, "-std=c++17", "-fopenmp", f"-I{INCLUDE}", os.path.join(SAN, "oracle_and_cpu_check.cpp"),
          os.path.join(ROOT, "paper_2010_10039_amd", "cpu", "hf_cpu.cpp"), oracle_obj, "-o", exe])
    r = _run([exe], env=ENV, timeout=600)
    _clean(r)
    assert "sanitized run clean" in r.stdout


def test_libhf_host_code_under_sanitizers(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not found")
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    base = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", f"-I{INCLUDE}", f"-I{CSRC}"]
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    srcs.append(os.path.join(SAN, "host_check.cpp"))

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        _run([*base, *host_san, *lang, "-c", src, "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = str(tmp_path / "host_check")
    # link: the sanitizer runtimes for the host code only (no device code is built on this line)
    _run([hipcc, "--offload-arch=gfx950", "-fsanitize=address,undefined", "-fno-gpu-sanitize", *objs, "-o", exe])
    r = _run([exe], env=ENV, timeout=600)
    _clean(r)
    assert "sanitized host run clean" in r.stdout
