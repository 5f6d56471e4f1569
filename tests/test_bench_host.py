"""Host logic of bench.py (no GPU): the one-GPU guard, the algorithmic bytes
the roofline prices the dominant launch at (the method's bytes per update
times the updates the launch performs), the launch's own I/O, and the rule
that a committed HBM-counter summary only counts while the kernel source it
was taken on is unchanged."""
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
def test_launch_io_bytes(csz, rsz):
    n, R = 128, 1
    npts, face = n ** 3, 6 * R * n * n
    # fused halves: A reads psi, V and the aux, writes u2 and its aux; B also
    # reads u2 and the second aux
    assert bench.launch_io_bytes("fused2_half_a", n, R, csz, rsz) == npts * (2 * csz + rsz) + face * 32
    assert bench.launch_io_bytes("fused2_half_b", n, R, csz, rsz) == npts * (3 * csz + rsz) + face * 48
    assert bench.launch_io_bytes("fused2_half_a", n, R, csz, rsz, first=False) == npts * (2 * csz + rsz)
    # staged sweep: stages 1 and 3 write only their z; 2 starts the running
    # sum, 4 finishes it into psi
    assert bench.launch_io_bytes("stage_1", n, R, csz, rsz) == npts * (2 * csz + rsz)
    assert bench.launch_io_bytes("stage_3", n, R, csz, rsz) == npts * (2 * csz + rsz)
    assert bench.launch_io_bytes("stage_2", n, R, csz, rsz) == npts * (4 * csz + rsz)
    assert bench.launch_io_bytes("stage_4", n, R, csz, rsz) == npts * (3 * csz + rsz)
    assert bench.launch_io_bytes("boundary_1", n, R, csz, rsz) == face * (48 + csz)
    assert bench.launch_io_bytes("meanfield", n, R, csz, rsz) is None


def test_method_bytes_per_update():
    # psi in and out, V, and the FP64 face aux (32 B per entry, 6 R n^2 entries)
    assert bench.method_bytes_per_update(128, 1, 16, 8) == pytest.approx(41.5)
    assert bench.method_bytes_per_update(128, 1, 8, 4) == pytest.approx(21.5)
    assert bench.method_bytes_per_update(128, 3, 16, 8) == pytest.approx(44.5)
    assert bench.method_bytes_per_update(128, 1, 16, 8, first=False) == 40


def test_roofline_is_priced_on_the_method_bytes():
    # the round-one record: half B 25.70 us, half A 22.38 us, 50.15 us per step
    n = 128
    table = [{"launch": "fused2_half_a", "ms": 0.02238}, {"launch": "fused2_half_b", "ms": 0.02570}]
    r = bench.roofline(table, n, 1, 16, 8, 0.05015, 150451777.0)
    alg = 41.5 * n ** 3 * 0.5                      # half a step of updates
    assert r["kernel"] == "fused2_half_b"
    assert r["alg_bytes_per_launch"] == pytest.approx(alg)
    assert r["achieved"] == pytest.approx(alg / 0.02570e-3 / 1e9)
    assert r["frac"] == pytest.approx(0.2117, abs=5e-4)
    assert r["step_frac"] == pytest.approx(41.5 * n ** 3 / 0.05015e-3 / 8e12)
    assert r["impl_frac"] == pytest.approx((n ** 3 * 56 + 6 * n * n * 48) / 0.02570e-3 / 8e12)
    assert r["traffic_ratio"] == pytest.approx(150451777.0 / alg)
    # face-only launches are never the dominant sweep, however long
    table.append({"launch": "boundary_1", "ms": 1.0})
    assert bench.roofline(table, n, 1, 16, 8, 0.05, None)["kernel"] == "fused2_half_b"
    # a one-pass launch carries the whole step
    r1 = bench.roofline([{"launch": "fused_step", "ms": 0.02}], n, 1, 16, 8, 0.02, None)
    assert r1["frac"] == pytest.approx(r1["step_frac"])
    assert r1["traffic_ratio"] is None


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
