"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): csrc/host_check.cpp drives every entry point through its size
queries and argument validation, which finish before any HIP call, in an
executable whose host code is built with both sanitizers; any report fails."""
import os
import subprocess


def test_host_code_is_clean_under_asan_and_ubsan():
    from paper_2503_12749_amd import build
    exe = build.build_host_check()
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host check ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
