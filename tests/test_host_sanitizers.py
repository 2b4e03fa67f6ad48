"""Host code of the library under AddressSanitizer (leaks included) and
ThreadSanitizer: mesh set-up of 2D and 3D meshes, lattice-index and stencil
queries, and concurrent set-up from three threads (tests/sanitize).  The
sanitized build compiles every source again (a few minutes), so these tests
run only with MF_SANITIZE=1; MF_SANITIZE_BIG=1 adds the cube at level 8."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
pytestmark = pytest.mark.skipif(os.environ.get("MF_SANITIZE") != "1",
                                reason="sanitizer builds are opt-in (MF_SANITIZE=1)")


@pytest.mark.parametrize("san", ["address", "thread"])
def test_mesh_setup_under_sanitizer(san, tmp_path):
    out = subprocess.run([os.path.join(HERE, "sanitize", "build.sh"), san, str(tmp_path)], check=True,
                         capture_output=True, text=True).stdout.strip().splitlines()[-1]
    env = dict(os.environ)
    if os.environ.get("MF_SANITIZE_BIG") == "1":
        env["BIG"] = "1"
    if san == "address":
        env["ASAN_OPTIONS"] = "detect_leaks=1"
    r = subprocess.run([out], capture_output=True, text=True, env=env, timeout=3000)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "sanitizer driver OK" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "WARNING: ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
