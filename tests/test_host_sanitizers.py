"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): tests/abi_host_check.c drives every entry point through the paths
that return before device work (handle life cycle, info, setters, argument
checks), linked against a build of libmlbm whose host code is instrumented
(paper_1309_1656_amd/sanitize_build.py).  Leak detection is on."""
import os
import subprocess


def test_host_code_is_clean_under_sanitizers():
    from paper_1309_1656_amd import build as B
    from paper_1309_1656_amd import sanitize_build
    sources = [sanitize_build.CHECK_SRC, os.path.join(B.CSRC, "api.hip"), os.path.join(B.ROOT, "include", "mlbm.h"),
               B.LIB]
    if not os.path.exists(sanitize_build.CHECK_BIN) or \
            os.path.getmtime(sanitize_build.CHECK_BIN) < max(os.path.getmtime(f) for f in sources):
        sanitize_build.build()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([sanitize_build.CHECK_BIN], capture_output=True, text=True, env=env, timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "host checks passed" in res.stdout
    assert "ERROR: AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr
