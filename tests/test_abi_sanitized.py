"""The host side of the C interface under AddressSanitizer and
UndefinedBehaviorSanitizer, without a GPU.

librcp's host code (C interface, argument checking, workspace layout, batch
program builder) is built with both sanitizers, the kernels being the
ordinary objects; test_abi.py then runs against that build in a child
process with the sanitizer runtime preloaded.  An out-of-bounds access, a
use after free or undefined behaviour in the code those tests reach ends
the child with a report, which fails this test.  Leak checking is off: the
Python interpreter and the HIP runtime keep allocations until exit.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_under_address_and_ub_sanitizers():
    from paper_1703_09074_amd import build_sanitized
    try:
        runtime = build_sanitized.runtime()
    except (OSError, RuntimeError, subprocess.CalledProcessError) as e:
        pytest.skip(f"no sanitizer runtime: {e}")
    lib = build_sanitized.build()
    env = dict(os.environ)
    pre = env.get("LD_PRELOAD", "")
    env["LD_PRELOAD"] = runtime + (" " + pre if pre else "")
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:exitcode=86"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1:exitcode=87"
    env["RCP_TEST_LIBRARY"] = lib
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-x",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout[-3000:] + "\n" + r.stderr[-6000:]
    print(out)
    assert "ERROR: AddressSanitizer" not in r.stderr, out
    assert "runtime error:" not in r.stderr, out
    assert r.returncode == 0, out
    assert " passed" in r.stdout, out
