"""Host-side parts of bench.py (no GPU): the one-GPU rule, the algorithmic
byte counts of a contraction launch and of the Gram-based FISTA loop and
the traffic guard on the profiled kernel source."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_contraction_bytes_counts_each_class_slab_once_and_spectra_per_object():
    # the method's bytes: every stored slab once (one per symmetry class),
    # whatever the work items re-read, plus the spectra in and out
    info = {"slab_bytes_A": 1_000_000, "slab_bytes_AT": 2_000_000,
            "read_bytes_A": 1_100_000, "read_bytes_AT": 2_300_000}
    nk, nz, nt = 33024, 128, 512
    assert bench.contraction_bytes(info, nk, nz, nt, False) == 1_000_000 + nk * (nz + nt) * 8
    assert bench.contraction_bytes(info, nk, nz, nt, True, B=16) == 2_000_000 + 16 * nk * (nz + nt) * 8
    assert bench.reread_bytes(info, False) == 100_000 and bench.reread_bytes(info, True) == 300_000


def test_fista_bytes_at_the_big_size():
    # 256^2 x 128 x 512: 5,924 Gram blocks of 128 x 128 floats (388 MB) and
    # 826 MB per iteration in all (blocks, nine spectrum-sized passes, 16
    # bytes per voxel: x and z in and out of the update fused into the
    # inverse transform, which also runs the next forward row pass)
    nk, nz, nt, nxy = 256 * 129, 128, 512, 256 * 256
    info = {"slab_bytes_A": 0, "slab_bytes_AT": 5924 * 512 * 128 * 4, "gram_bytes": 5924 * 128 * 128 * 4}
    one = bench.fista_gram_bytes(info, nk, nz, nt, nxy, 1)
    per = bench.fista_gram_bytes(info, nk, nz, nt, nxy, 2) - one
    assert per == 16 * nz * nxy + 72 * nz * nk + info["gram_bytes"]
    assert 0.82e9 < per < 0.83e9
    setup = one - per
    assert setup == 4 * nt * nxy + 24 * nt * nk + bench.contraction_bytes(info, nk, nz, nt, True) + 12 * nz * nxy
    # the algorithmic floor of the same loop: A^T d once, then per iteration
    # the Gram blocks, (A^T d)^ and the update's 16 bytes per voxel
    a1 = bench.fista_algorithmic_bytes(info, nk, nz, nt, nxy, 1)
    a2 = bench.fista_algorithmic_bytes(info, nk, nz, nt, nxy, 2)
    assert a2 - a1 == info["gram_bytes"] + 8 * nz * nk + 16 * nz * nxy
    assert a2 - a1 < per


def test_profile_traffic_only_for_the_profiled_source(tmp_path, monkeypatch):
    p = os.path.join(ROOT, "profiles", "contract_fp32_256x256x128x512_traffic.json")
    d = json.load(open(p))
    assert d["commands"] and d["calibration"]["copy_bytes"] == 1 << 30
    # counted traffic of the committed summary is within 3 % of the method's
    # bytes (each class slab once): A's member spectra are staged by both
    # workgroups of a split row (+33.8 MB per A launch) and A^T reads about
    # 56 MB beyond its slabs and spectrum (1.4 % of the mean launch together)
    assert abs(d["traffic_bytes_per_launch"] / d["algorithmic_bytes_per_launch"] - 1) < 0.03
    fake = tmp_path / "contract.hip"
    fake.write_text("// not the profiled kernel\n")
    monkeypatch.setattr(bench, "CONTRACT_SRC", str(fake))
    assert bench.profile_traffic(0) is None
