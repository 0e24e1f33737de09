"""The library's host C++ under AddressSanitizer and UndefinedBehaviorSanitizer.

A variant of liblv.so is built with -fsanitize=address,undefined on every
host code path (-Xarch_host for the HIP sources, so device code is
untouched; the float64 fit compiled by clang++ without OpenMP), and the
host-only ABI tests (tests/test_abi.py: argument validation before any
launch, the eigensolver and Brent search of the fits, Frank-Wolfe, the
binding's shape checks) run against it in a subprocess with the sanitizer
runtime preloaded.  Any sanitizer report fails the test.  No GPU is used."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"

pytestmark = pytest.mark.slow


def test_abi_tests_clean_under_asan_and_ubsan():
    if not os.path.exists(CLANG):
        pytest.skip("no clang++")
    rt = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"],
                        capture_output=True, text=True).stdout.strip()
    if not os.path.exists(rt):
        pytest.skip("no ASan runtime")
    sys.path.insert(0, ROOT)
    from paper_2312_16335_amd import build

    san = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-fno-sanitize-recover=undefined"]
    with tempfile.TemporaryDirectory(prefix="lv_asan_") as tmp:
        lib = os.path.join(tmp, "liblv.so")
        hip = []
        for f in san:
            hip += ["-Xarch_host", f]
        build.build(out=lib, extra_flags=hip, host_flags=["-O1"] + san, host_cxx=CLANG,
                    openmp=False)
        # the variant is instrumented: it calls into the sanitizer runtimes
        syms = subprocess.run(["nm", "-D", "--undefined-only", lib], capture_output=True,
                              text=True).stdout
        assert "__asan_report" in syms and "__ubsan_handle" in syms
        code = ("import sys, pytest\n"
                "import paper_2312_16335_amd._lib as L\n"
                f"L.LIB_PATH = {lib!r}\n"
                "sys.exit(pytest.main(['-x', '-q', '-p', 'no:cacheprovider', "
                "'tests/test_abi.py']))\n")
        env = dict(os.environ, LD_PRELOAD=rt,
                   ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                           text=True, timeout=900)
        out = r.stdout + r.stderr
        print(out[-3000:])
        assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out
        assert r.returncode == 0, out[-3000:]
        assert " passed" in out
