"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

* The plan-time mathematics (csrc/plan_math.cpp: modulus-set constants, CRT
  tables, quantised roots, MFMA operand planes of every substrate, stage and
  direction) is compiled for the host only with both sanitizers and driven
  by tests/sanitize/plan_math_driver.cpp.
* The C oracle (oracle/exact.c, oracle/dd.c) is compiled with both
  sanitizers and run through its Python front end on small transforms, the
  stage checkpoints, sampled lines and the pack, in a child process that
  preloads the ASan runtime.
Any sanitizer report fails the test (recovery is disabled).
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_23698_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (cmd[:3], r.stdout[-2000:], r.stderr[-4000:])
    return r


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_plan_math_under_sanitizers(tmp_path):
    objs = []
    for src in (os.path.join(CSRC, "plan_math.cpp"), os.path.join(ROOT, "tests", "sanitize", "plan_math_driver.cpp")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([HIPCC, "-std=c++17", "-O1", "-g", "-x", "hip", "--offload-arch=gfx950", "--cuda-host-only"] + SAN_HOST +
             ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", src, "-o", obj])
        objs.append(obj)
    exe = str(tmp_path / "plan_math_driver")
    _run([HIPCC] + SAN_HOST + objs + ["-o", exe])
    r = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1"))
    assert "plan math checksum" in r.stdout
    assert "runtime error" not in r.stderr


ORACLE_WORK = r"""
import numpy as np
from oracle import exact as ox
from paper_2606_23698_amd import inputs
for shape, pq in (((8, 8, 8), ((2, 4), (4, 2), (2, 4))), ((4, 6, 12), ((2, 2), (2, 3), (3, 4))),
                  ((1, 5, 3), ((1, 1), (5, 1), (1, 3)))):
    x = inputs.uniform(shape, 7)
    y = ox.fft3_exact(x, pq)
    y32 = ox.fft3_exact(x.astype(np.complex64), pq, precision=1)
    hi, lo = ox.fft3_dd(x)
    assert np.all(np.isfinite(y)) and np.all(np.isfinite(hi))
line = inputs.uniform((1, 32), 8).reshape(32)
for st in (1, 2):
    r = ox.line_stage(line, 32, 4, 8, stage=st)
    assert len(r["re"]) == 32
xb = inputs.uniform((16, 16, 16), 9)
ref = ox.lines_at(xb.reshape(-1, 16), 16, 4, 4, 3)
cone = ox.dd_cone_lines(xb, [(0, 5), (7, 2)])
assert ox.pack(2 ** 53 + 1, 0) == float(2 ** 53)
print("oracle ok")
"""


def _asan_runtime():
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.skipif(_asan_runtime() is None, reason="gcc's ASan runtime not installed")
def test_oracle_under_sanitizers(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    src = [os.path.join(ROOT, "oracle", f) for f in ("exact.c", "dd.c")]
    flags = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    _run(["gcc", "-O1", "-g", "-std=gnu11", "-fPIC", "-shared", "-pthread", "-ffp-contract=off"] + flags +
         ["-o", lib] + src + ["-lm"])
    env = dict(os.environ, LD_PRELOAD=_asan_runtime(), OBFFT_ORACLE_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1", PYTHONPATH=ROOT)
    r = _run([sys.executable, "-c", ORACLE_WORK], env=env, cwd=ROOT)
    assert "oracle ok" in r.stdout
    assert "runtime error" not in r.stderr
