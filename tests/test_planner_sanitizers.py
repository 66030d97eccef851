"""The host planner under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU): planner.cpp is built with g++ and both sanitizers into a driver
(tests/native/planner_sanitize.cpp) that plans seeded matrices under every
type option, round-trips their stages, and runs Lie plans through the
theta-Jacobian and the gradient contraction; any sanitizer report aborts
it.  The matrices: the configs' generator, matrices with a symmetric B,
with a12 = a21 = 0 (the IDFT route), the FT matrix and a pure chirp."""
from __future__ import annotations

import os
import shutil
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1707_03688_amd", "csrc")


def _matrices():
    out = []
    c = synth.symplectic_candidates(77)
    out += [next(c) for _ in range(60)]
    rng = np.random.default_rng(77)
    I2, Z2 = np.eye(2), np.zeros((2, 2))
    for _ in range(10):  # symmetric B: CM-CC-CM
        P1, B, P3 = [0.5 * (x + x.T) for x in rng.normal(size=(3, 2, 2))]
        out.append(np.block([[I2, Z2], [P1, I2]]) @ np.block([[I2, B], [Z2, I2]]) @ np.block([[I2, Z2], [P3, I2]]))
    for _ in range(10):  # a12 = a21 = 0
        A0 = np.diag(rng.uniform(0.5, 1.5, 2) * rng.choice([-1, 1], 2))
        Q, P = [0.5 * (x + x.T) for x in rng.normal(0, 0.4, size=(2, 2, 2))]
        out.append(np.block([[I2, Z2], [P, I2]]) @ np.block([[A0, Z2], [Z2, np.linalg.inv(A0)]])
                   @ np.block([[I2, Q], [Z2, I2]]))
    out.append(np.block([[Z2, I2], [-I2, Z2]]))
    out.append(np.block([[I2, Z2], [np.array([[0.3, 0.1], [0.1, -0.2]]), I2]]))
    return out


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_planner_under_asan_and_ubsan(tmp_path):
    exe = tmp_path / "planner_sanitize"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(CSRC, "planner.cpp"), os.path.join(ROOT, "tests", "native", "planner_sanitize.cpp"),
           "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    mats = tmp_path / "mats.txt"
    mats.write_text("\n".join(" ".join(f"{v:.17g}" for v in np.asarray(M).reshape(16)) for M in _matrices()))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([str(exe), str(mats)], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-4000:]
    fields = dict(zip(r.stdout.split()[0::2], map(int, r.stdout.split()[1::2])))
    assert fields["matrices"] == len(_matrices()) and fields["planned"] > 300 and fields["jacobian"] > 50
