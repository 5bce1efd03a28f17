"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The FP64 oracle's C code is rebuilt with gcc's ASan/UBSan instrumentation
(stopping at the first report) and its whole CPU test module runs against
that build in a child process that preloads gcc's ASan runtime: every
out-of-bounds access, use after free, signed overflow or misaligned load
the oracle tests reach ends the child with a report.  The library's host
code (the entry points' argument checks, plan and workspace logic) is built
the same way with hipcc and driven by the host-only ABI tests.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _gcc_runtime(name):
    try:
        path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True,
                              check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return path if os.path.isabs(path) and os.path.exists(path) else None


def _env(preload):
    env = dict(os.environ)
    # the ASan runtime must come first; whatever is preloaded already stays
    prior = env.get("LD_PRELOAD", "").strip()
    env.update(S3_ORACLE_SANITIZE="1", LD_PRELOAD=preload + (":" + prior if prior else ""),
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=86",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    return env


def test_oracle_tests_pass_under_asan_and_ubsan():
    asan = _gcc_runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's libasan is not installed")
    # build first (outside the preloaded child), then check the build is instrumented
    env = _env(asan)
    lib = subprocess.run([sys.executable, "-c", "import oracle.api as a; print(a.build())"], cwd=ROOT,
                         env=env, capture_output=True, text=True, timeout=300)
    assert lib.returncode == 0, lib.stderr[-2000:]
    path = lib.stdout.strip().splitlines()[-1]
    assert path.endswith("libs3oracle_san.so")
    syms = subprocess.run(["nm", "-D", path], capture_output=True, text=True, check=True).stdout
    assert "__asan_report_load8" in syms and "__ubsan_handle_" in syms

    run = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                          os.path.join("tests", "test_oracle.py")], cwd=ROOT, env=env, capture_output=True,
                         text=True, timeout=900)
    out = run.stdout + run.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert run.returncode == 0, out[-4000:]
    assert " passed" in out


def test_abi_host_code_under_asan_and_ubsan(tmp_path):
    """The C ABI's host-only checks (test_abi.py: descriptor validation, state
    errors, workspace sizing, 32-bit range checks) against a build whose
    entry points' host code carries ASan/UBSan instrumentation."""
    from paper_1708_08640_amd import build as b
    try:
        rt = b.asan_runtime()
    except (OSError, subprocess.CalledProcessError):
        pytest.skip("no clang resource directory")
    if not os.path.exists(rt):
        pytest.skip("the compiler's shared ASan runtime is not installed")
    lib = b.build(out=str(tmp_path / "libs3cmtf_san.so"), host_sanitize=True)
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True, check=True).stdout
    assert "__asan_report_load8" in syms and "__ubsan_handle_" in syms

    driver = ("import sys, pytest\n"
              "import paper_1708_08640_amd._abi as a\n"
              f"a.LIB_PATH = {lib!r}\n"
              "sys.exit(pytest.main(['-q', '-x', '-p', 'no:cacheprovider', 'tests/test_abi.py']))\n")
    run = subprocess.run([sys.executable, "-c", driver], cwd=ROOT, env=_env(rt), capture_output=True,
                         text=True, timeout=600)
    out = run.stdout + run.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert run.returncode == 0, out[-4000:]
    assert " passed" in out
