"""Host logic of the serving loop that needs no GPU: the latency breakdown
(queue wait and time in the pool, by job size)."""
import numpy as np

from paper_1208_2428_amd.serve import latency_breakdown


def test_latency_breakdown_splits_and_thirds():
    rng = np.random.default_rng(3)
    works = rng.permutation(np.arange(1, 31, dtype=np.float64) * 1e8)
    waits = np.full(30, 0.002)                # 2 ms in the queue each
    services = works / 1e10                   # time in the pool proportional to work
    out = latency_breakdown(waits, services, works)
    assert abs(out["queue_p50_ms"] - 2.0) < 1e-9 and abs(out["queue_p99_ms"] - 2.0) < 1e-9
    assert abs(out["pool_p50_ms"] - np.percentile(services, 50) * 1e3) < 1e-9
    small, medium, large = out["by_work"]
    assert [t["count"] for t in out["by_work"]] == [10, 10, 10]
    assert small["work_max"] == 10e8 and medium["work_max"] == 20e8 and large["work_max"] == 30e8
    assert small["latency_p50_ms"] < medium["latency_p50_ms"] < large["latency_p50_ms"]
    assert out["log_latency_log_work_corr"] > 0.9


def test_latency_breakdown_queue_dominated():
    works = np.linspace(1e8, 1e9, 12)
    waits = np.linspace(1.0, 0.0, 12)         # the small jobs waited longest
    services = np.full(12, 0.01)
    out = latency_breakdown(waits, services, works)
    assert out["queue_p99_ms"] > out["pool_p99_ms"]
    assert out["log_latency_log_work_corr"] < 0
