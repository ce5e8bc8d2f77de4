"""The runtime's host code under AddressSanitizer and UndefinedBehaviorSanitizer:
tests/hostsan/hostsan_driver (built by __graft_entry__.build() through
tests/hostsan/build.py; the test itself builds nothing) calls every C-ABI
entry point on three small systems and checks K against the oracle's; any
sanitizer finding ends it with a report."""

import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
DRIVER = os.path.join(HERE, "hostsan", "_build", "hostsan_driver")
sys.path.insert(0, os.path.join(HERE, "hostsan"))


def test_host_code_clean_under_sanitizers(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(DRIVER):
        pytest.skip("sanitizer driver not built (python tests/hostsan/build.py)")
    import make_input

    inp = str(tmp_path / "hs.bin")
    make_input.write(inp)
    print("hostsan driver on", inp, flush=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([DRIVER, inp], env=env, capture_output=True, text=True, timeout=240)
    print(r.stdout[-6000:], r.stderr[-6000:], flush=True)
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    assert r.returncode == 0
    assert "PASSED" in r.stdout
