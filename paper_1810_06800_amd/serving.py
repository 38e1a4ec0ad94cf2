"""Open-loop replay of a request trace through the request server.

Request r of the trace is submitted ``arrival_s`` seconds after the start,
whatever the server is doing (open loop), with samples 0..n-1 of seed r.
Latency is completion minus scheduled arrival, observed when the host
collects the request.  Only host bookkeeping lives here: every sample runs in
the library's kernels.
"""
from __future__ import annotations

import time


def percentile(values, q: float):
    """Nearest-rank percentile (q in [0, 100]) of a non-empty list."""
    v = sorted(values)
    if not v:
        return None
    rank = max(1, min(len(v), int(-(-q * len(v) // 100))))
    return v[rank - 1]


def requests_of(trace):
    """(L, k, seed, sample, flags) descriptors of every trace entry."""
    return [[(r["L"], r["k"], r["seed"], s, 0) for s in range(r["n"])] for r in trace]


def replay(srv, trace, window_s: float, clock=time.perf_counter, sleep=time.sleep,
           log=None, idle_s: float = 0.0005):
    """Replay ``trace`` (dicts with arrival_s, L, k, n, seed, sorted by
    arrival) for ``window_s`` seconds of wall time.  Requests arriving after
    the window are not submitted; requests still running when it closes are
    reported as censored (their age is a lower bound on their latency).

    ``srv`` needs submit(descs) -> id, step(wait) -> int, completed() -> ids,
    results(id) -> list of dicts and stats() -> dict (rsa.Server)."""
    reqs = requests_of(trace)
    start = clock()
    nxt = 0
    arrival = {}       # id -> scheduled arrival (s after start)
    meta = {}          # id -> trace index
    latency = []
    done_deposits = 0
    done_samples = 0
    last_log = start
    while True:
        t = clock() - start
        while nxt < len(trace) and trace[nxt]["arrival_s"] <= min(t, window_s):
            rid = srv.submit(reqs[nxt])
            arrival[rid] = trace[nxt]["arrival_s"]
            meta[rid] = nxt
            nxt += 1
        if t >= window_s:
            break
        no_more = nxt >= len(trace) or trace[nxt]["arrival_s"] > window_s
        if no_more and not arrival:
            break
        gap = (trace[nxt]["arrival_s"] - t) if not no_more else window_s - t
        srv.step(wait=gap > 0.002)
        now = clock() - start
        for rid in srv.completed():
            res = srv.results(rid)
            latency.append(now - arrival.pop(rid))
            meta.pop(rid)
            done_samples += len(res)
            done_deposits += sum(r["n_jam"] for r in res)
        st = srv.stats()
        if st["samples_queued"] == 0 and st["samples_resident"] == 0 and gap > idle_s:
            sleep(min(gap, 0.01))
        if log and clock() - last_log > 5.0:
            last_log = clock()
            log(f"serving t={now:.1f}s submitted={nxt} completed={len(latency)} "
                f"resident={st['samples_resident']} queued={st['samples_queued']}")
    elapsed = clock() - start
    st = srv.stats()
    censored_age = [elapsed - a for a in arrival.values()]
    offered = [r for r in trace if r["arrival_s"] <= window_s]
    span = offered[-1]["arrival_s"] if offered else 0.0
    out = {
        "window_s": window_s,
        "elapsed_s": elapsed,
        "requests_offered": len(offered),
        "arrival_span_s": span,
        "offered_req_per_s": len(offered) / span if span > 0 else None,
        "offered_samples": sum(r["n"] for r in offered),
        "requests_completed": len(latency),
        "requests_censored": len(censored_age),
        "latency_s": {
            "p50": percentile(latency, 50),
            "p99": percentile(latency, 99),
            "max": max(latency) if latency else None,
        },
        "censored_age_s_max": max(censored_age) if censored_age else None,
        "samples_completed": done_samples,
        "deposits_completed": done_deposits,
        "deposits_in_progress": st["deposits_in_progress"],
        "served_deposits_per_s": (st["deposits_completed"] + st["deposits_in_progress"]) / elapsed,
        "completed_deposits_per_s": done_deposits / elapsed,
        "arena_bytes": st["arena_bytes"],
        "arena_peak_bytes": st["arena_peak"],
        "launches": st["launches"],
    }
    # the latency over every offered request is at least this when some are
    # censored: censored ones count with their age so far
    if censored_age:
        out["latency_lower_bound_s"] = {
            "p50": percentile(latency + censored_age, 50),
            "p99": percentile(latency + censored_age, 99),
        }
    return out
