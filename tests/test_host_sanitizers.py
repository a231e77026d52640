"""CPU: the library's host code (planning, layout, the shared prime table and CRT
cache, the host thread pool, decoding) built from its own sources with
AddressSanitizer + UndefinedBehaviorSanitizer, and separately with
ThreadSanitizer, and driven from several threads by tests/sanitize/host_driver.cpp.

The host pass of every source without kernels is compiled with the sanitizer
(no device code is generated), so the build takes seconds and needs no GPU; the
sources that define kernels or device arrays (their host side is launch
wrappers) are linked from the library's own build.  A sanitizer report fails
the test."""

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1010_1386_amd", "csrc")
DRIVER = os.path.join(HERE, "sanitize", "host_driver.cpp")
SANITIZED = ["api.cpp", "plan.cpp", "job.cpp", "tune.cpp", "server.cpp", "gcd.cpp"]
WITH_KERNELS = ["kernels.hip", "persistent.hip", "noalloc.cpp"]
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

SANITIZERS = {
    "address_undefined": (["address", "undefined"], {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=1",
                                                     "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}),
    "thread": (["thread"], {"TSAN_OPTIONS": "halt_on_error=1:second_deadlock_stack=1"}),
}


def _tools():
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    clang = os.path.join(ROCM, "llvm", "bin", "clang++")
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("ROCm compilers not found")
    return hipcc, clang


def _build(kind, out_dir):
    hipcc, clang = _tools()
    sans, _ = SANITIZERS[kind]
    san_flags = []
    for s in sans:  # host pass only: each -fsanitize= behind -Xarch_host
        san_flags += ["-Xarch_host", f"-fsanitize={s}"]
    if "undefined" in sans:
        san_flags += ["-Xarch_host", "-fno-sanitize-recover=undefined"]
    common = ["-std=c++17", "-x", "hip", "--offload-host-only", "-O1", "-g", "-fno-omit-frame-pointer",
              "-fPIC"] + san_flags

    def compile_one(src):
        obj = os.path.join(out_dir, os.path.basename(src) + ".o")
        r = subprocess.run([hipcc] + common + ["-c", src, "-o", obj], capture_output=True, text=True)
        if r.returncode:
            raise RuntimeError(f"compile {src}:\n{r.stderr[-4000:]}")
        return obj

    srcs = [os.path.join(CSRC, s) for s in SANITIZED] + [DRIVER]
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    objs += _kernel_objects()
    exe = os.path.join(out_dir, "host_driver")
    link = [clang, "-o", exe] + objs + [f"-fsanitize={','.join(sans)}", f"-L{ROCM}/lib", "-lamdhip64",
                                         f"-Wl,-rpath,{ROCM}/lib", "-lpthread"]
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(f"link:\n{r.stderr[-4000:]}")
    return exe


def _kernel_objects():
    """The library build's objects of the sources with kernels, rebuilt if stale."""
    from paper_1010_1386_amd import build as b

    objs = []
    for src in WITH_KERNELS:
        obj = os.path.join(b.BUILD, src + ".o")
        if not os.path.exists(obj) or os.path.getmtime(obj) < max(
                os.path.getmtime(os.path.join(CSRC, f)) for f in os.listdir(CSRC)):
            os.makedirs(b.BUILD, exist_ok=True)
            obj, _ = b._compile(src)
        objs.append(obj)
    return objs


@pytest.mark.parametrize("kind", sorted(SANITIZERS))
def test_host_code_under_sanitizer(kind, tmp_path):
    exe = _build(kind, str(tmp_path))
    env = dict(os.environ)
    env.update(SANITIZERS[kind][1])
    env["RSL_HOST_THREADS"] = "4"  # the library's own pool, beside the driver's threads
    r = subprocess.run([exe, "6", "64"], capture_output=True, text=True, env=env, timeout=600)
    report = (r.stdout + r.stderr)[-6000:]
    assert r.returncode == 0, report
    assert "ERROR: AddressSanitizer" not in report and "runtime error" not in report, report
    assert "WARNING: ThreadSanitizer" not in report, report
    assert ": ok" in r.stdout
