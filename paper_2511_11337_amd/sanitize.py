"""Host-side AddressSanitizer / UndefinedBehaviorSanitizer build of libboa and
a run of the library's host-only tests against it (no GPU needed).

    python -m paper_2511_11337_amd.sanitize          # build libboa_asan.so, run tests/test_lib_host.py

Only the host half of every source is instrumented (each sanitizer flag is
given to the host compilation alone); device code is built as usual.
Undefined behaviour traps (no runtime library); address errors are reported
by clang's ASan runtime, preloaded into the Python process that runs the
tests.  Leak checking is off: the interpreter and the HIP runtime keep
allocations alive until exit.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

from paper_2511_11337_amd.build import CSRC, COMMON, DEVICE_ONLY, HIPCC, PKG, SOURCES

OUT = os.path.join(PKG, "libboa_asan.so")
HOST_SAN = ("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
            "-Xarch_host -fsanitize-trap=undefined -Xarch_host -fno-omit-frame-pointer -g").split()


def asan_runtime() -> str:
    libs = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not libs:
        raise FileNotFoundError("clang ASan runtime not found under /opt/rocm/llvm")
    return libs[0]


def _compile(src: str) -> str:
    obj = os.path.join(CSRC, "_build_asan", src + ".o")
    os.makedirs(os.path.dirname(obj), exist_ok=True)
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    extra = DEVICE_ONLY if src.endswith(".hip") else []
    cmd = [HIPCC, *COMMON, *extra, *HOST_SAN, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr[-6000:]}")
    return obj


def build() -> str:
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fsanitize-trap=undefined", "-shared-libasan",
           "-o", OUT, "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-6000:]}")
    return OUT


def run_host_tests(extra_args=()) -> int:
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:alloc_dealloc_mismatch=0:detect_odr_violation=0:abort_on_error=1"
    env["BOA_LIB_PATH"] = OUT
    cmd = [sys.executable, "-m", "pytest", os.path.join(PKG, "..", "tests", "test_lib_host.py"), "-q", "-p",
           "no:cacheprovider", *extra_args]
    return subprocess.run(cmd, env=env).returncode


if __name__ == "__main__":
    print("built", build(), flush=True)
    sys.exit(run_host_tests(sys.argv[1:]))
