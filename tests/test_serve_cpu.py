"""The served-ensemble scheduler with stand-in handles (no GPU): admission in
arrival order by footprint, the memory budget is never exceeded, oversized
requests are rejected, every step is accounted."""
import threading
import time

import pytest

from paper_1808_04338_amd.serve import Request, serve


class FakeSim:
    live = 0
    peak = 0
    lock = threading.Lock()

    def __init__(self, model):
        self.model = model
        with FakeSim.lock:
            FakeSim.live += model["fp"]
            FakeSim.peak = max(FakeSim.peak, FakeSim.live)

    def timestep(self, dt):
        time.sleep(0.002 * self.model["cost"])
        return {"newton_iters": 1, "lin_iters": 2}

    def get_state(self):
        return (self.model["name"],)

    def close(self):
        with FakeSim.lock:
            FakeSim.live -= self.model["fp"]


def _model(name, fp, cost, steps=3):
    return {"name": name, "fp": fp, "cost": cost, "schedule": [1.0] * steps}


def test_admission_respects_budget_and_order():
    FakeSim.live = FakeSim.peak = 0
    reqs = [Request(i, _model("m%d" % i, fp, 1 + i % 3), arrival=0.001 * i, tag=fp)
            for i, fp in enumerate([4, 3, 5, 2, 6, 1, 4, 4])]
    res, summ = serve(reqs, budget_bytes=10, max_active=3, sim_factory=FakeSim,
                      footprint_fn=lambda m: m["fp"], keep_state=True)
    assert summ["completed"] == len(reqs)
    assert summ["timesteps"] == 3 * len(reqs)
    assert FakeSim.peak <= 10
    assert summ["peak_bytes"] <= 10 and summ["peak_active"] <= 3
    # first-in first-out: admission times never decrease with arrival order
    adm = [res[i].admitted for i in range(len(reqs))]
    assert adm == sorted(adm)
    for i in range(len(reqs)):
        assert res[i].state == ("m%d" % i,)
        assert len(res[i].latencies) == 3 and all(x >= 0 for x in res[i].latencies)


def test_oversized_request_rejected_others_served():
    reqs = [Request(0, _model("big", 50, 1), 0.0), Request(1, _model("ok", 5, 1), 0.0)]
    res, summ = serve(reqs, budget_bytes=10, sim_factory=FakeSim, footprint_fn=lambda m: m["fp"])
    assert res[0].status == "rejected"
    assert res[1].status == "ok"
    assert summ["rejected"] == 1 and summ["completed"] == 1


def test_completion_hook_runs_once_per_served_request():
    """on_done sees every admitted request once, after its last step; a rejected
    request never reaches a worker, so it is not reported."""
    seen = []
    lock = threading.Lock()

    def on_done(r):
        with lock:
            seen.append((r.rid, len(r.latencies), r.status))

    reqs = [Request(i, _model("m%d" % i, 2, 1), 0.001 * i) for i in range(6)]
    reqs.append(Request(6, _model("big", 50, 1), 0.0))
    res, summ = serve(reqs, budget_bytes=10, max_active=2, sim_factory=FakeSim,
                      footprint_fn=lambda m: m["fp"], on_done=on_done)
    assert sorted(seen) == [(i, 3, "ok") for i in range(6)]
    assert res[6].status == "rejected"


def test_large_request_cap_lets_small_requests_pass():
    """With max_large = 1, at most one request above large_bytes is resident at
    a time, and a small request that arrives behind a held-back large one is
    admitted before it."""
    FakeSim.live = FakeSim.peak = 0
    live_large = [0]
    peak_large = [0]
    lock = threading.Lock()

    class CountingSim(FakeSim):
        def __init__(self, model):
            super().__init__(model)
            if model["fp"] > 5:
                with lock:
                    live_large[0] += 1
                    peak_large[0] = max(peak_large[0], live_large[0])

        def close(self):
            if self.model["fp"] > 5:
                with lock:
                    live_large[0] -= 1
            super().close()

    fps = [8, 8, 1, 8, 1]
    reqs = [Request(i, _model("m%d" % i, fp, 3 if fp > 5 else 1), arrival=0.0001 * i, tag=fp)
            for i, fp in enumerate(fps)]
    res, summ = serve(reqs, budget_bytes=100, max_active=8, sim_factory=CountingSim,
                      footprint_fn=lambda m: m["fp"], max_large=1, large_bytes=5)
    assert summ["completed"] == len(reqs)
    assert peak_large[0] == 1
    # request 2 (small) arrived after request 1 (large, held back) and got in first
    assert res[2].admitted < res[1].admitted
    assert res[4].admitted < res[3].admitted
