"""The benchmark's command line without a GPU: more than one GPU is refused with a message, and the
entry module exposes build() and smoke()."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_bench_help_lists_the_modes():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--gpus", "--precision-study", "--sweep", "--storage"):
        assert flag in r.stdout


def test_entry_module_exposes_build_and_smoke():
    sys.path.insert(0, ROOT)
    import __graft_entry__ as g
    assert callable(g.build) and callable(g.smoke)


def test_profile_entries_follow_the_kernel_source(tmp_path, monkeypatch):
    """bench.py reads a counter summary only when it was taken on the current kernel source, and
    looks entries up by workload, storage and updates per launch."""
    sys.path.insert(0, ROOT)
    import json
    import bench
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps({
        "w/f32/2": {"bytes_per_launch": 123, "source_digest": "a" * 16},
        "w/f32/1": {"bytes_per_launch": 456, "source_digest": "b" * 16}}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_digest", lambda: "a" * 16)
    assert bench.measured_traffic("w", "f32", 2) == 123
    assert bench.measured_traffic("w", "f32", 1) is None      # taken on other sources
    assert bench.measured_traffic("w", "f16s", 2) is None     # not measured
    assert bench.profile_entry("valu", "w", "f32", 2) is None  # no such summary


def test_cpu_baseline_reports_one_and_all_threads():
    """The oracle leg of the benchmark times one thread and every thread it may use, on each
    sample, and names the host CPU."""
    sys.path.insert(0, ROOT)
    import bench
    from paper_1812_05401_amd import inputs as I
    c = I.cylinder_wake(64, 32, d=8.0, x0=16.0, re=100.0)
    r = bench.cpu_baseline(c, [(c, 2, 4)])
    assert r["kind"] == "oracle" and r["unit"] == "MLUPS" and r["value"] > 0
    assert r["threads_1"]["threads"] == 1 and r["threads_1"]["steps"] == 2
    assert r["threads_all"]["threads"] == bench.host_threads() == r["cores"]
    assert r["cpu_model"] and r["nproc"] >= 1
    assert len(r["legs"]) == 2
