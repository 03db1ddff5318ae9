"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code only, g++) runs the fast pins without a finding: no
out-of-bounds access, use after free or undefined behaviour in the FP64
renderer, its adjoint, the lifting, the z-buffer splat, the normals or the
blending.  The pins run in a child process with the ASan runtime preloaded
(Python itself is not instrumented)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    r = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_pins_pass_under_the_sanitizers(tmp_path):
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("no AddressSanitizer runtime for g++ here")
    sys.path.insert(0, ROOT)
    from oracle import build as obuild
    lib = obuild.build(out=str(tmp_path / "libtgo_sanitized.so"), sanitize=True)
    env = dict(os.environ, TGO_LIB_OVERRIDE=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_lift_pins.py"),
                        os.path.join(ROOT, "tests", "test_zsplat_pins.py"),
                        os.path.join(ROOT, "tests", "test_blend_pins.py"),
                        "-k", "not fd_cfg3_small"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    assert r.returncode == 0, f"sanitized oracle failed the pins:\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
