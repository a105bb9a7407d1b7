"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

`oracle/sanitize_check.c` runs every exported oracle routine (projection, rendering,
backward in the three pointmap frames, frozen trace and its loss, tile sets, the SE(3)
exponential) over small seeded scenes with the edge cases the method has: Gaussians
behind or in front of the near plane, a zero quaternion, opacity past alpha_max, the
Jacobian clamp, views that are not a whole number of tiles, an empty scene and a
one-pixel view.  Built with gcc and both sanitizers (no recovery, leak check on), it must
exit cleanly, and its sums must match a plain -O2 build of the same file run on the same
thread count: integer counts exactly, floating-point sums to 1e-12 relative (the
frozen-trace loss is an OpenMP reduction whose order may differ between builds).
"""
import os
import re
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "..", "oracle", "sanitize_check.c")
COMMON = ["-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-Wall",
          "-Wno-unused-function"]


def _build(out, extra):
    cmd = ["gcc", *extra, *COMMON, SRC, "-o", out, "-lm"]
    return subprocess.run(cmd, capture_output=True, text=True)


def _parse(text):
    rows = []
    for line in text.strip().splitlines():
        rows.append(dict(re.findall(r"(\w+)=(\S+)", line)))
    return rows


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not on PATH")
def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    san, plain = str(tmp_path / "orc_san"), str(tmp_path / "orc_plain")
    r = _build(san, ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                     "-fno-sanitize-recover=all"])
    if r.returncode != 0 and "asan" in r.stderr.lower():
        pytest.skip("gcc here has no sanitizer runtime: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    assert _build(plain, ["-O2"]).returncode == 0
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    a = subprocess.run([san, "2"], capture_output=True, text=True, env=env, timeout=600)
    assert a.returncode == 0, a.stdout + a.stderr
    assert "runtime error" not in a.stderr and "AddressSanitizer" not in a.stderr, a.stderr
    b = subprocess.run([plain, "2"], capture_output=True, text=True, timeout=600)
    assert b.returncode == 0, b.stderr
    ra, rb = _parse(a.stdout), _parse(b.stdout)
    assert len(ra) == len(rb) == 4
    for x, y in zip(ra, rb):
        assert x.keys() == y.keys()
        for k in x:
            if k in ("img", "grad", "loss", "se3"):
                fx, fy = float(x[k]), float(y[k])
                assert abs(fx - fy) <= 1e-12 * max(1.0, abs(fy)), (k, x, y)
            else:
                assert x[k] == y[k], (k, x, y)
    # The scenes reach what they are meant to: fragments, tile pairs and an empty scene.
    assert int(ra[0]["frags"]) > 0 and int(ra[0]["pairs"]) >= int(ra[0]["exact"]) > 0
    assert ra[2]["n"] == "0" and ra[2]["frags"] == "0" and ra[2]["pairs"] == "0"
