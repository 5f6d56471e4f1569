"""Host logic of bench.py (no GPU): the one-GPU guard, the algorithmic bytes
each launch is priced at, and the rule that a committed HBM-counter summary
only counts while the kernel source it was taken on is unchanged."""
import hashlib
import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.mark.parametrize("csz,rsz", [(16, 8), (8, 4)])
def test_algorithmic_bytes_per_launch(csz, rsz):
    n, R = 128, 1
    npts, face = n ** 3, 6 * R * n * n
    # fused halves: A reads psi, V and the aux, writes u2 and its aux; B also
    # reads u2 and the second aux
    assert bench.alg_bytes("fused2_half_a", n, R, csz, rsz) == npts * (2 * csz + rsz) + face * 32
    assert bench.alg_bytes("fused2_half_b", n, R, csz, rsz) == npts * (3 * csz + rsz) + face * 48
    assert bench.alg_bytes("fused2_half_a", n, R, csz, rsz, first=False) == npts * (2 * csz + rsz)
    # staged sweep: stages 1 and 3 write only their z; 2 starts the running
    # sum, 4 finishes it into psi
    assert bench.alg_bytes("stage_1", n, R, csz, rsz) == npts * (2 * csz + rsz)
    assert bench.alg_bytes("stage_3", n, R, csz, rsz) == npts * (2 * csz + rsz)
    assert bench.alg_bytes("stage_2", n, R, csz, rsz) == npts * (4 * csz + rsz)
    assert bench.alg_bytes("stage_4", n, R, csz, rsz) == npts * (3 * csz + rsz)
    assert bench.alg_bytes("boundary_1", n, R, csz, rsz) == face * (48 + csz)
    assert bench.alg_bytes("meanfield", n, R, csz, rsz) is None


def _write_summary(root, label, src_text, hbm, sha=None):
    csrc = root / "paper_1908_02456_amd" / "csrc"
    csrc.mkdir(parents=True, exist_ok=True)
    (csrc / "fused.hip").write_text(src_text)
    prof = root / "profiles"
    prof.mkdir(exist_ok=True)
    if sha is None:
        sha = hashlib.sha256(src_text.encode()).hexdigest()
    (prof / ("traffic_%s_128_c128.txt" % label)).write_text(
        "kernel: %s\nsource: fused.hip\nsource_sha256: %s\nhbm_bytes_per_launch: %d\n" % (label, sha, hbm))


def test_counter_summary_counts_only_for_its_source(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    args = types.SimpleNamespace(n=128, dtype="c128")
    _write_summary(tmp_path, "fused2_half_b", "kernel source v1\n", 150451431)
    assert bench.measured_traffic("fused2_half_b", args) == 150451431.0
    # the kernel changed since the counters were taken: no traffic figure
    (tmp_path / "paper_1908_02456_amd" / "csrc" / "fused.hip").write_text("kernel source v2\n")
    assert bench.measured_traffic("fused2_half_b", args) is None
    # no summary for this launch, or another workload
    assert bench.measured_traffic("fused2_half_a", args) is None
    assert bench.measured_traffic("fused2_half_b", types.SimpleNamespace(n=96, dtype="c128")) is None


def test_counter_summary_with_a_wrong_hash_is_ignored(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    _write_summary(tmp_path, "fused2_half_b", "kernel source\n", 1, sha="0" * 64)
    assert bench.measured_traffic("fused2_half_b", types.SimpleNamespace(n=128, dtype="c128")) is None
