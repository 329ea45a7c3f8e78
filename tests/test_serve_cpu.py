"""Host logic of the serving loop that needs no GPU: the latency breakdown
(queue wait and time in the pool, by job size), and the loop itself (FIFO
admission, the arena budget, result hand-back, release) driven against a
host stand-in for the pool."""
import numpy as np
import pytest

from paper_1208_2428_amd import serve
from paper_1208_2428_amd import workloads as WL
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


# ---- the serving loop against a host-side stand-in for the pool --------------


class FakePool:
    """Host stand-in with the pool's contract: admit returns a slot or None
    (no free slot, or the arena budget would be exceeded); tick advances every
    resident job by up to `passes` passes of K steps; done returns (and
    forgets) the jobs that have run all their steps; a collected result is
    ready on the second query; release frees the slot and its bytes."""
    K = 5

    def __init__(self, budget: int, max_slots: int):
        self.budget, self.max_slots = budget, max_slots
        self.used = self.peak = self.ticks = 0
        self.free = list(range(max_slots))
        self.jobs: dict[int, dict] = {}
        self.admitted: list[int] = []   # seeds, in admission order
        self.stream = None

    def admit(self, steps, width, height, seed, fill, force_rate, walls):
        b = serve.job_bytes(width)
        assert width == height
        if not self.free or self.used + b > self.budget:
            return None
        slot = self.free.pop(0)
        self.used += b
        self.peak = max(self.peak, self.used)
        self.jobs[slot] = dict(left=steps, bytes=b, seed=seed, side=width, state="run", queries=0)
        self.admitted.append(seed)
        return slot

    def tick(self, passes):
        self.ticks += 1
        for j in self.jobs.values():
            if j["state"] == "run" and j["left"] > 0:
                j["left"] = max(0, j["left"] - passes * self.K)

    def done(self):
        out = [s for s, j in self.jobs.items() if j["state"] == "run" and j["left"] == 0]
        for s in out:
            self.jobs[s]["state"] = "done"
        return out

    def collect(self, slot, block):
        j = self.jobs[slot]
        assert j["state"] == "done"
        j["state"] = "collecting"
        n = -(-j["side"] // block)
        return np.full((n, n, 3), j["seed"], dtype=np.int32)

    def collected(self, slot):
        j = self.jobs[slot]
        j["queries"] += 1
        return j["queries"] >= 2

    def release(self, slot):
        j = self.jobs.pop(slot)
        assert j["state"] == "collecting"
        self.used -= j["bytes"]
        self.free.append(slot)

    def sync(self):
        pass


class FakeEvent:
    def record(self, stream):
        pass

    def synchronize(self):
        pass


def fake_server(pool: FakePool, passes: int = 1) -> serve.Server:
    s = serve.Server.__new__(serve.Server)
    s.pool, s.passes, s.block, s.ticks_ahead = pool, passes, 16, 2
    return s


def requests(n, seed=1, arrival_span=0.0):
    rng = np.random.default_rng(seed)
    return [WL.Request(arrival=arrival_span * k / n, side=64 * int(rng.integers(1, 9)),
                       steps=int(rng.integers(1, 120)), seed=1000 + k) for k in range(n)]


@pytest.mark.parametrize("passes", [1, 3])
def test_server_fifo_within_budget(monkeypatch, passes):
    monkeypatch.setattr(serve.torch.cuda, "Event", FakeEvent)
    reqs = requests(60)
    budget = 3 * serve.job_bytes(512)          # room for a few jobs at a time
    pool = FakePool(budget, max_slots=8)
    out = fake_server(pool, passes).run(reqs, realtime=False, keep_results={0, 17, 59})
    assert out["completed"] == len(reqs)
    assert pool.peak <= budget and pool.used == 0 and not pool.jobs
    assert pool.admitted == [r.seed for r in reqs]            # first in, first admitted
    assert out["node_updates"] == sum(r.side * r.side * r.steps for r in reqs)
    assert sorted(out["results"]) == [0, 17, 59]
    for i, blocks in out["results"].items():                 # each result is its own job's
        n = -(-reqs[i].side // 16)
        assert blocks.shape == (n, n, 3) and np.all(blocks == reqs[i].seed)
    assert 1 <= out["max_resident"] <= 8


def test_server_realtime_arrivals(monkeypatch):
    monkeypatch.setattr(serve.torch.cuda, "Event", FakeEvent)
    reqs = requests(20, seed=2, arrival_span=0.05)
    pool = FakePool(8 * serve.job_bytes(512), max_slots=16)
    out = fake_server(pool).run(reqs, realtime=True)
    assert out["completed"] == 20 and pool.used == 0
    assert out["queue_p50_ms"] >= 0 and out["pool_p50_ms"] > 0
    assert out["seconds"] >= 0.05 * 19 / 20              # it waited for the last arrival


def test_server_rejects_job_larger_than_the_empty_pool(monkeypatch):
    monkeypatch.setattr(serve.torch.cuda, "Event", FakeEvent)
    reqs = [WL.Request(arrival=0.0, side=1024, steps=10, seed=1)]
    pool = FakePool(serve.job_bytes(512), max_slots=4)
    with pytest.raises(RuntimeError, match="does not fit the pool"):
        fake_server(pool).run(reqs, realtime=False)
