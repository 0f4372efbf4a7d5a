"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The library's host side (planner, plan checker, layout self-check, tuning
cache, argument validation of every entry point) is rebuilt with ASan and
UBSan on the host compilation only (no device code), the plain-C oracle
likewise, and the CPU tests of those parts run again in a child process that
loads both builds with the sanitizer runtime preloaded.  Any report fails the
run (UBSan does not recover; ASan aborts on its first error).
"""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# CPU tests that drive the host code and the C oracle
SUITES = ["tests/test_abi_cpu.py", "tests/test_oracle_cascade.py",
          "tests/test_oracle_signed.py", "tests/test_narrowing_host.py"]


@pytest.mark.slow
def test_host_code_and_oracle_under_sanitizers(tmp_path):
    import torch
    if torch.cuda.is_available():
        pytest.skip("the sanitizer build has no device code; it runs where no GPU is visible")
    sys.path.insert(0, ROOT)
    from oracle import c_oracle
    from paper_1609_06641_amd import _build
    lib = _build.build_sanitized()
    orc = c_oracle.build_sanitized(str(tmp_path / "liborc_chw_san.so"))
    rt = _build.sanitizer_runtime()
    assert os.path.exists(rt), rt
    env = dict(os.environ)
    env.update({
        "LD_PRELOAD": rt,
        "CHW_LIBRARY": lib,
        "ORC_CHW_LIBRARY": orc,
        # Python itself is not built with ASan: its own allocations are not
        # leak-checked; everything else reports and stops
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:halt_on_error=1",
        "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
        "CUDA_VISIBLE_DEVICES": "", "HIP_VISIBLE_DEVICES": "",
    })
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                          "-m", "not gpu and not slow"] + SUITES,
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (res.stdout + res.stderr)[-4000:]
    assert res.returncode == 0, tail
    assert "AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr, tail
    assert " passed" in res.stdout, tail
