"""Sanitizer builds for the CPU tests (not used by any GPU run).

The oracle is built by gcc with AddressSanitizer and UndefinedBehaviorSanitizer;
the HIP library with both on its host code only (the device code of a
gfx950 build is not instrumented), every finding fatal.  The tests load
these builds in a child Python with the matching sanitizer runtime
preloaded (ORACLE_LIB / DVM_LIB select them)."""
import glob
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2501_00923_amd import build as hipbuild  # noqa: E402


def build_oracle(path: str) -> str:
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           *oracle.FLAGS, "-o", path, oracle._SRC, "-lm"])
    return path


def gcc_asan_runtime() -> str:
    return subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()


def build_library(path: str) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    flags = [f for f in hipbuild.FLAGS if f not in ("-O3",)]
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=all"]
    cmd = [hipcc, "-O1", "-g", "-fno-omit-frame-pointer", *flags, *host_san, "-shared-libsan",
           "-o", path, *hipbuild.SOURCES]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(res.stdout + res.stderr)
    return path


def clang_asan_runtime() -> str:
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else ""


def run_pytest(args, env_extra, timeout=900):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               **env_extra)
    return subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *args],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)


def loaded_in_child(module_call: str, path: str, env_extra) -> bool:
    """Whether a child Python with the same environment maps `path` after
    `module_call` (so the test above ran the sanitized build)."""
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", **env_extra)
    code = f"{module_call}\nimport sys\nsys.exit(0 if {path!r} in open('/proc/self/maps').read() else 3)"
    return subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, timeout=300).returncode == 0
