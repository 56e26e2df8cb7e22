"""Sanitizer build of the library's host code, for the host-side ABI checks.

AddressSanitizer and UndefinedBehaviorSanitizer instrument the host code of
api.hip (argument validation, handle life cycle, error strings); the device
code is compiled as usual (-Xarch_host keeps the sanitizers off the GPU
side).  The other objects come from the normal build.  tests/abi_host_check.c
is compiled with the same sanitizers and linked against the result.  Nothing
here runs on a GPU: the check program makes only calls that return before
any device work.

Usage: python -m paper_1309_1656_amd.sanitize_build   (after build.build())
"""
import os
import subprocess

from . import build as B

SAN_DIR = os.path.join(B.BUILD, "san")
SAN_LIB = os.path.join(SAN_DIR, "libmlbm_san.so")
CHECK_SRC = os.path.join(B.ROOT, "tests", "abi_host_check.c")
CHECK_BIN = os.path.join(SAN_DIR, "abi_host_check")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd)}\n{res.stdout}\n{res.stderr}")


def _sanitizer_runtime_dir(clang):
    """Directory of the clang sanitizer runtimes (for the run-time search path)."""
    out = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = out.stdout.strip()
    if not os.path.isabs(path):
        res = subprocess.run([clang, "--print-runtime-dir"], capture_output=True, text=True)
        return res.stdout.strip()
    return os.path.dirname(path)


def build():
    os.makedirs(SAN_DIR, exist_ok=True)
    clang = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang")
    rt = _sanitizer_runtime_dir(clang)
    api_obj = os.path.join(SAN_DIR, "api.o")
    _run([B.hipcc(), *B.compile_flags(), *HOST_SAN, "-c", os.path.join(B.CSRC, "api.hip"), "-o", api_obj])
    others = [os.path.join(B.BUILD, os.path.splitext(s)[0] + ".o") for s in B.SOURCES if s != "api.hip"]
    missing = [o for o in others if not os.path.exists(o)]
    if missing:
        raise RuntimeError(f"normal build missing: {missing}")
    _run([B.hipcc(), "-shared", "-fPIC", f"--offload-arch={B.ARCH}", *HOST_SAN, "-shared-libsan",
          "-Wl,-rpath," + rt, "-o", SAN_LIB, api_obj, *others])
    _run([clang, "-O1", "-g", "-std=c99", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
          "-fno-sanitize-recover=undefined", "-shared-libsan", "-I", os.path.join(B.ROOT, "include"), CHECK_SRC,
          "-L", SAN_DIR, "-lmlbm_san", "-Wl,-rpath," + SAN_DIR, "-Wl,-rpath," + rt, "-o", CHECK_BIN])
    return CHECK_BIN


if __name__ == "__main__":
    print(build())
