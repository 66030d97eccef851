"""Host-side checks of bench.py: its same-algorithm CPU baseline (a pocketfft
five-slot chain of the plan's stage matrices) equals the FP64 oracle chain,
and a request for more than one GPU is refused."""
from __future__ import annotations

import math
import os
import subprocess
import sys

import numpy as np
import pytest

import synth
from oracle import chain, plan as oplan

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("seed", [1, 2, 5])
def test_cpu_fft_chain_equals_oracle(seed):
    N = 64
    d = math.sqrt(2 * math.pi / N)
    M = next(synth.symplectic_candidates(seed))
    po = oplan.plan(M, N, N, d, d)
    g = synth.complex_normal((N, N), seed=3)
    _, _, out = bench.cpu_fft_chain({"type": po.typ, "mats": list(po.mats)}, g, N, d, budget_s=0.0)
    assert chain.rel_l2(out, chain.forward(po, g)) <= 1e-12


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_host_info_and_ranges():
    info = bench.host_info()
    assert info["os_cpu_count"] >= 1 and info["affinity"] >= 1
    assert bench._ranges([0, 1, 2, 5, 7, 8]) == "0-2,5,7-8"


def test_traffic_is_read_only_for_the_profiled_sources(tmp_path, monkeypatch):
    prof = tmp_path / "p.md"
    h = bench.kernel_source_hash()
    prof.write_text(f"x\\ntraffic-per-launch: rows=17 cols=19 sources={h}\\n")
    monkeypatch.setattr(bench, "PROFILE", str(prof))
    assert bench.traffic_from_profile() == {"rows": 17, "cols": 19}
    prof.write_text("traffic-per-launch: rows=17 cols=19 sources=0123456789abcdef\\n")
    assert bench.traffic_from_profile() == {}
