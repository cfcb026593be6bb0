"""Host-side parts of bench.py (no GPU): the one-GPU rule, the algorithmic
byte count of a contraction launch and the traffic guard on the profiled
kernel source."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_contraction_bytes_counts_library_once_and_spectra_per_object():
    info = {"read_bytes_A": 1_000_000, "read_bytes_AT": 2_000_000}
    nk, nz, nt = 33024, 128, 512
    assert bench.contraction_bytes(info, nk, nz, nt, False) == 1_000_000 + nk * (nz + nt) * 8
    assert bench.contraction_bytes(info, nk, nz, nt, True, B=16) == 2_000_000 + 16 * nk * (nz + nt) * 8


def test_profile_traffic_only_for_the_profiled_source(tmp_path, monkeypatch):
    p = os.path.join(ROOT, "profiles", "contract_fp32_256x256x128x512_traffic.json")
    d = json.load(open(p))
    assert d["commands"] and d["calibration"]["copy_bytes"] == 1 << 30
    # counted traffic of the committed summary is within 2 % of the algorithmic
    # bytes: A's member spectra are staged by both workgroups of a split row
    # (+33.8 MB per A launch, 0.9 % of the mean launch) and nothing else is re-read
    assert abs(d["traffic_bytes_per_launch"] / d["algorithmic_bytes_per_launch"] - 1) < 0.02
    fake = tmp_path / "contract.hip"
    fake.write_text("// not the profiled kernel\n")
    monkeypatch.setattr(bench, "CONTRACT_SRC", str(fake))
    assert bench.profile_traffic(0) is None
