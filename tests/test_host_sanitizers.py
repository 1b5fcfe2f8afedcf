"""The host code of the library (input validation, engine and server set-up,
error paths) built with AddressSanitizer and UndefinedBehaviorSanitizer
(device code unchanged), driven through every host-side error path of the C
ABI in a child process with the sanitizer runtime preloaded.  A sanitizer
report fails the child.  Library robustness; no passage of the paper."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.slow

CHILD = """
import sys
sys.modules["torch"] = None  # the host paths under test need no device runtime of PyTorch
import paper_1107_1653_amd.shapley as S
S.LIB_PATH = sys.argv[1]
import pytest
sys.exit(pytest.main(["-q", "-p", "no:cacheprovider", "tests/test_abi_errors.py"]))
"""


def test_error_paths_are_clean_under_host_sanitizers(tmp_path):
    from paper_1107_1653_amd import build
    try:
        rt = build.sanitizer_runtime()
    except RuntimeError as e:
        pytest.skip(str(e))
    lib = build.build(verbose=False, sanitize_dir=str(tmp_path))
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:exitcode=23",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1:exitcode=24")
    r = subprocess.run([sys.executable, "-c", CHILD, lib], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
