"""The serving scheduler's host logic (CPU, stub renderer): open-loop release
times, slot exclusivity, admission by footprint, and the statistics."""
import threading
import time

import numpy as np

from paper_2501_12581_amd.serve import schedule


def _stub(service_s):
    busy = set()
    lock = threading.Lock()
    log = []

    def render(slot, req):
        with lock:
            assert slot not in busy, "slot used twice at once"
            busy.add(slot)
        time.sleep(service_s[req["id"]])
        with lock:
            busy.discard(slot)
            log.append(req["id"])
        return None
    return render, log


def test_requests_start_no_earlier_than_arrival_and_overlap():
    reqs = [{"id": k, "arrival": 0.01 * k, "size": 64, "m": 4} for k in range(12)]
    render, log = _stub({k: 0.03 for k in range(12)})
    st = schedule(reqs, 3, lambda r: 1, 1 << 30, render)
    recs = st["records"]
    assert sorted(log) == list(range(12))
    for r in recs:
        assert r["start"] >= r["arrival"] - 1e-3 and r["end"] > r["start"]
    overlapping = sum(1 for i, a in enumerate(recs) for b in recs[i + 1:] if a["start"] < b["end"] and b["start"] < a["end"])
    assert overlapping > 0
    lat = np.array([r["latency"] for r in recs]) * 1e3
    assert abs(st["p50_ms"] - np.percentile(lat, 50)) < 1e-9 and st["p50_ms"] <= st["p99_ms"]


def test_one_slot_serves_one_at_a_time_in_arrival_order():
    reqs = [{"id": k, "arrival": 0.0, "size": 64, "m": 4} for k in range(6)]
    render, log = _stub({k: 0.01 for k in range(6)})
    st = schedule(reqs, 1, lambda r: 1, 1 << 30, render, mode="fifo")
    recs = st["records"]
    assert log == list(range(6))
    for a, b in zip(recs, recs[1:]):
        assert b["start"] >= a["end"] - 1e-4


def test_admission_by_footprint_limits_concurrency():
    # footprint 6 each, budget 10: never two in flight even with 4 slots
    reqs = [{"id": k, "arrival": 0.0, "size": 64, "m": 4} for k in range(5)]
    render, log = _stub({k: 0.02 for k in range(5)})
    st = schedule(reqs, 4, lambda r: 6, 10, render)
    recs = sorted(st["records"], key=lambda r: r["start"])
    for a, b in zip(recs, recs[1:]):
        assert b["start"] >= a["end"] - 1e-4
    # a request larger than the whole budget still runs (alone)
    st = schedule([{"id": 0, "arrival": 0.0}], 2, lambda r: 100, 10, _stub({0: 0.0})[0])
    assert st["requests"] == 1
