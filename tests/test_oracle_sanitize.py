"""The oracle built under AddressSanitizer and UndefinedBehaviorSanitizer
(host code only) runs small cases of every part it implements without a
report: oracle/sanitize_main.cpp (moving interfaces on all three velocity
sets with refill, reinitialisation, walls of each kind and gravity, the
cumulant gas, two bubbles, the tangent, decision record and replay, a
crafted refill, a two-level refinement with sensor and re-mesh)."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host compiler")
def test_oracle_under_address_and_undefined_behaviour_sanitizers():
    src = [os.path.join(ROOT, "oracle", f) for f in ("sanitize_main.cpp", "lsb_oracle.cpp", "refine_oracle.cpp")]
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "orc_sanitize")
        subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=all", "-fopenmp", *src, "-o", exe], check=True)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", OMP_NUM_THREADS="4")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        print(r.stdout[-2000:], r.stderr[-4000:])
        assert r.returncode == 0, r.stderr[-4000:]
        assert "sanitize: ok" in r.stdout
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
