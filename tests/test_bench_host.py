"""Host checks of bench.py's byte accounting (no GPU needed)."""
import bench


def test_schedule_bytes_per_step():
    # two-sweep schedule, k = 3 (q = 6): 2q + 4k^2 + 10k + 6 = 84 elements
    # unrefined; one refinement step forward and adjoint adds 91 more
    assert bench.sched_bytes_per_step(2, "fp64", 0) == 84 * 8
    assert bench.sched_bytes_per_step(2, "fp64r", 1) == 175 * 8
    assert bench.sched_bytes_per_step(2, "fp32r", 1) == 175 * 4
    # k = 4 (q = 10): 20 + 64 + 40 + 6 = 130 unrefined, + 20 + 64 + 52 + 4 = 140
    assert bench.sched_bytes_per_step(3, "fp64", 0) == 130 * 8
    assert bench.sched_bytes_per_step(3, "fp32r", 1) == 270 * 4


def test_counter_traffic_only_for_the_measured_sources(tmp_path, monkeypatch):
    # a committed counter figure is reported only while the kernel sources
    # hash to the digest it was measured on
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "k.md").write_text(
        "header\n"
        "traffic kern/a bytes_per_launch=123 kernel_sources_sha256=aaaa\n"
        "traffic kern/b bytes_per_launch=456 kernel_sources_sha256=bbbb\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_sources_sha256", lambda: "aaaa")
    assert bench.counter_traffic("kern/a") == 123
    assert bench.counter_traffic("kern/b") is None
    assert bench.counter_traffic("kern/c") is None


def test_kernel_sources_digest_is_stable():
    d = bench.kernel_sources_sha256()
    assert len(d) == 64 and d == bench.kernel_sources_sha256()


def test_more_than_one_gpu_is_refused(monkeypatch, capsys):
    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", "2"])
    assert bench.main() == 2
    assert "one GPU" in capsys.readouterr().err
