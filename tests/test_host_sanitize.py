"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Every source is rebuilt with the sanitizers applied to the host pass only
(``-Xarch_host`` before each ``-fsanitize=``; the gfx950 device code is built as
usual and never runs here), linked into a separate library in a temporary
folder, and driven by ``tests/host_sanitize.c``: the CSR builder against a dense
adjacency matrix on random edge lists with loops and repeats, the workspace and
scratch size queries over a grid of shapes and options, and the argument and
workspace refusals of the entry points.  A sanitizer finding aborts the driver.
Needs no GPU; a few seconds of compilation on eight cores."""
import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2607_11952_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}"


def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm compilers not found")
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    common = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature",
              "-Xclang", "-packed-fp32-ops", "-I", INCLUDE, "-I", CSRC, *HOST_SAN]
    objs = [str(tmp_path / (s + ".o")) for s in srcs]
    jobs = max(1, min(len(srcs), os.cpu_count() or 1, 8))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(_run, [[HIPCC, *common, "-c", os.path.join(CSRC, s), "-o", o] for s, o in zip(srcs, objs)]))
    lib = tmp_path / "libfastalign_san.so"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *HOST_SAN, "-o", str(lib), *objs])
    # the host objects really are instrumented: the library calls the sanitizer runtimes
    syms = subprocess.run(["nm", "-D", "--undefined-only", str(lib)], capture_output=True, text=True).stdout
    assert "__asan_report_load8" in syms and "__ubsan_handle_" in syms
    exe = tmp_path / "host_sanitize"
    _run([CLANG, "-std=c99", "-Wall", "-Werror", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-I", INCLUDE, os.path.join(ROOT, "tests", "host_sanitize.c"), "-o", str(exe),
          "-L", str(tmp_path), "-lfastalign_san", f"-Wl,-rpath,{tmp_path}"])
    env = dict(os.environ, ASAN_OPTIONS="halt_on_error=1:detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120, env=env)
    assert out.returncode == 0, (out.returncode, out.stdout, out.stderr[-4000:])
    assert out.stdout.split() == ["csr:", "ok", "sizes:", "ok", "arguments:", "ok"]
    assert "runtime error" not in out.stderr and "Sanitizer" not in out.stderr, out.stderr[-4000:]
