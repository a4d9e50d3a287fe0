"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

`paper_1810_02719_amd/mispectral_sanitized` (built by `build()` from every
source and `tests/native/sanitized_driver.hip`, the sanitizers on the host
pass only) runs the planners, the argument checks and, on a GPU, the chained
tracking with three stream lanes under graph capture and replay, the per-block
path, the event timer, choose_c, encode/decode and the adjoint.  A sanitizer
report makes it exit non-zero."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_1810_02719_amd", "mispectral_sanitized")
SUPP = os.path.join(ROOT, "tests", "native", "lsan.supp")


def _run(mode, timeout):
    assert os.path.exists(EXE), "build() makes the sanitized executable"
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "halt_on_error=1:detect_stack_use_after_return=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["LSAN_OPTIONS"] = f"suppressions={SUPP}:print_suppressions=0"
    r = subprocess.run([EXE, mode], capture_output=True, text=True, timeout=timeout, env=env)
    out = r.stdout + r.stderr
    print(out[-6000:])
    assert "ERROR: AddressSanitizer" not in out and "ERROR: LeakSanitizer" not in out, out[-6000:]
    assert "runtime error" not in out, out[-6000:]
    assert r.returncode == 0 and r.stdout.rstrip().endswith("ok"), out[-6000:]


def test_planner_and_argument_checks_sanitized():
    _run("host", 120)


@pytest.mark.gpu
def test_lanes_capture_replay_sanitized():
    _run("gpu", 240)
