"""The serving scheduler's host logic (CPU, stub renderer): open-loop release
times, slot exclusivity, admission by footprint, and the statistics."""
import threading
import time

import numpy as np
import pytest

from paper_2501_12581_amd.serve import device_overlap, schedule


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


def test_size_aware_slots_take_the_smallest_slot_that_holds_the_request():
    # slots 0, 1 hold 2048^2, slots 2, 3 only 512^2
    sizes = [2048, 2048, 512, 512]
    reqs = [{"id": 0, "arrival": 0.0, "size": 256}, {"id": 1, "arrival": 0.0, "size": 2048},
            {"id": 2, "arrival": 0.0, "size": 512}, {"id": 3, "arrival": 0.0, "size": 1024},
            {"id": 4, "arrival": 0.0, "size": 2048}, {"id": 5, "arrival": 0.2, "size": 256}]
    render, _ = _stub({k: 0.05 for k in range(6)})
    st = schedule(reqs, 4, lambda r: 1, 1 << 30, render, slot_size=sizes)
    by = {r["id"]: r for r in st["records"]}
    for r in st["records"]:
        assert sizes[r["slot"]] >= r["size"]  # a request only runs on a slot that holds it
    assert by[0]["slot"] == 2 and by[2]["slot"] == 3  # small requests go to the small slots first
    assert by[1]["slot"] == 0
    # request 3 (1024^2) needs a large slot: slot 1; request 4 waits for a large slot to free up
    assert by[3]["slot"] == 1 and by[4]["start"] >= min(by[1]["end"], by[3]["end"]) - 1e-3
    assert by[5]["slot"] in (2, 3)


def test_request_larger_than_every_slot_is_rejected_up_front():
    with pytest.raises(ValueError):
        schedule([{"id": 0, "arrival": 0.0, "size": 4096}], 2, lambda r: 1, 1 << 30, _stub({0: 0.0})[0],
                 slot_size=[2048, 1024])


def test_device_overlap_counts_requests_whose_intervals_intersect():
    recs = [{"device_start_ms": a, "device_end_ms": b} for a, b in ((0, 10), (5, 12), (20, 30), (30, 31), (40, 50))]
    assert device_overlap(recs) == 2 / 5  # (0,10) and (5,12); touching intervals do not overlap
    assert device_overlap([]) == 0.0
