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
