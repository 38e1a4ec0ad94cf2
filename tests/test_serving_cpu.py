"""Host bookkeeping of the serving replay (paper_1810_06800_amd.serving) with
a scripted stand-in for the request server and a simulated clock: arrivals
are submitted on time, latency is completion minus arrival, requests still
running at the window's end are censored, and percentiles are nearest-rank."""
import pytest

from paper_1810_06800_amd import serving, workloads


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeServer:
    """Each request finishes `cost * n` seconds of simulated time after it
    starts; requests run one at a time in arrival order (a FIFO device)."""

    def __init__(self, clock, cost=0.001):
        self.clock, self.cost = clock, cost
        self.queue, self.done, self.sizes, self.t_submit = [], [], {}, {}
        self.busy_until, self.next_id, self.deposits = 0.0, 1, 0

    def submit(self, descs):
        rid = self.next_id
        self.next_id += 1
        self.sizes[rid] = descs
        self.t_submit[rid] = self.clock.t
        self.queue.append(rid)
        return rid

    def step(self, wait=False):
        self.clock.t += 0.0005   # host time of one step
        n = 0
        while self.queue:
            rid = self.queue[0]
            start = max(self.busy_until, self.t_submit[rid])
            end = start + self.cost * len(self.sizes[rid])
            if end > self.clock.t:
                if not wait:
                    break
                self.clock.t = end
                wait = False   # block for the first completion only
            self.busy_until = end
            self.queue.pop(0)
            self.done.append(rid)
            n += 1
        return n

    def completed(self):
        out, self.done = self.done, []
        return out

    def results(self, rid):
        descs = self.sizes.pop(rid)
        self.deposits += 10 * len(descs)
        return [{"n_jam": 10} for _ in descs]

    def stats(self):
        return {"samples_queued": sum(len(self.sizes[r]) for r in self.queue), "samples_resident": 0,
                "deposits_completed": self.deposits, "deposits_in_progress": 0, "arena_bytes": 0,
                "arena_peak": 0, "launches": 0}


def trace(arrivals, n=2):
    return [{"id": i, "arrival_s": a, "L": 64, "k": 8, "n": n, "seed": i} for i, a in enumerate(arrivals)]


def test_percentile_nearest_rank():
    v = list(range(1, 101))
    assert serving.percentile(v, 50) == 50
    assert serving.percentile(v, 99) == 99
    assert serving.percentile(v, 100) == 100
    assert serving.percentile([7], 99) == 7
    assert serving.percentile([], 50) is None


def test_unsaturated_latency_is_service_time():
    clock = Clock()
    srv = FakeServer(clock, cost=0.001)
    tr = trace([0.1 * i for i in range(20)])
    out = serving.replay(srv, tr, window_s=10.0, clock=clock, sleep=clock.sleep)
    assert out["requests_completed"] == 20 and out["requests_censored"] == 0
    # service 2 ms per request plus at most a few host steps of 0.5 ms
    assert 0.002 <= out["latency_s"]["p50"] <= 0.0045
    assert out["samples_completed"] == 40 and out["deposits_completed"] == 400
    assert out["elapsed_s"] < 2.5   # stops once everything offered is done


def test_overload_censors_and_bounds():
    clock = Clock()
    srv = FakeServer(clock, cost=0.05)   # 0.1 s per request, arrivals every 0.01 s
    tr = trace([0.01 * i for i in range(300)])
    out = serving.replay(srv, tr, window_s=1.0, clock=clock, sleep=clock.sleep)
    assert out["requests_offered"] == 101
    assert out["requests_completed"] + out["requests_censored"] == 101
    assert 9 <= out["requests_completed"] <= 10
    lb = out["latency_lower_bound_s"]
    assert lb["p99"] >= out["latency_s"]["p50"]
    assert out["censored_age_s_max"] <= 1.0 + 1e-9


def test_serving_trace_shape():
    tr = workloads.serving_trace(requests=500)
    assert all(256 <= r["L"] <= 16384 and r["L"] & (r["L"] - 1) == 0 for r in tr)
    assert all(2 <= r["k"] <= r["L"] // 8 and r["k"] & (r["k"] - 1) == 0 for r in tr)
    assert all(1 <= r["n"] <= 64 for r in tr)
    gaps = [b["arrival_s"] - a["arrival_s"] for a, b in zip(tr, tr[1:])]
    assert all(g >= 0 for g in gaps)
    assert 1 / 260 < sum(gaps) / len(gaps) < 1 / 150   # Poisson at 200 per second
    assert workloads.serving_trace(requests=500) == tr   # seeded
    assert [r["seed"] for r in tr] == list(range(500))
