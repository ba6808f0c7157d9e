"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host code only): it is
rebuilt with both and a child Python process, with the ASan runtime preloaded, runs every
step of the path on synthetic frames of three formats, the narrowed search, the stereo maps,
the bilateral filter and the tracker.  Any out-of-bounds access, use after free or undefined
operation (signed overflow, a shift past the width, a misaligned load) ends the child with a
report, which fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import os
import numpy as np
import oracle
from paper_1807_02752_amd import synth
maps = open("/proc/self/maps").read()
assert os.environ["LDREF_SO"] in maps or oracle.lib() is not None
assert os.environ["LDREF_SO"] in open("/proc/self/maps").read() and "libasan" in maps
g, d, sc = synth.make_frame("c1", 3, 0)
r = oracle.detect(g, d, sc.d_max)
assert r is not None
oracle.detect(g, d.astype(np.float32), sc.d_max)
bits = np.zeros((4, 16, g.shape[1]), np.uint8)
oracle.detect_pruned(g, d, sc.d_max, bits)
d16 = np.clip(np.rint(d * 16), 0, 65535).astype(np.uint16)
oracle.detect(g, d16, sc.d_max)
d8 = np.clip(np.rint(d), 0, 255).astype(np.uint8)
oracle.detect(g, d8, sc.d_max)
rng = np.random.default_rng(0)
L = rng.integers(0, 256, (24, 40)).astype(np.uint8)
R = np.roll(L, -4, axis=1)
for rho in (1, 3, 5):
    oracle.stereo(L, R, d_max=12, rho=rho)
oracle.bilateral(g[:40, :64], rho=5)
s = oracle.TrackState()
for t in range(30):
    oracle.track_update(s, list(rng.integers(0, 300, int(rng.integers(0, 20)))))
print("sanitized oracle ok", flush=True)
"""


def _runtime(name):
    p = subprocess.run(["g++", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("no AddressSanitizer runtime for g++ here")
    so = str(tmp_path / "libldref_san.so")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
                           "-fno-fast-math", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fPIC", "-shared", "-o", so, os.path.join(ROOT, "oracle", "ldref.cpp")])
    env = dict(os.environ, LDREF_SO=so, LD_PRELOAD=asan, PYTHONPATH=ROOT,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1:exitcode=24")
    p = subprocess.run([sys.executable, "-c", CHILD], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    report = p.stdout[-3000:] + p.stderr[-6000:]
    assert p.returncode == 0 and "sanitized oracle ok" in p.stdout, report
    assert "AddressSanitizer" not in p.stderr and "runtime error" not in p.stderr, report
