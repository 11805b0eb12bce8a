"""Served ensemble: continuous batching of many simulator handles on one GPU.

Requests (a model and an arrival time) are admitted first-in first-out as
soon as their device footprint fits the HBM budget next to the models already
resident and a slot is free.  Every admitted model owns a handle, a workspace
and a HIP stream (default priority) and is advanced by a worker thread; ctypes
releases the interpreter lock inside library calls, so the models' kernels run
concurrently on the device.  When a model finishes its schedule its memory is
released and waiting requests are admitted, while the others keep running.

Per-timestep latency is measured from the moment a step is ready (the arrival
for the first step, the end of the previous step otherwise) to its completion,
so time spent waiting for admission counts against the first step.
"""
import collections
import threading
import time

import numpy as np

from . import _lib as L
from .sim import Sim, footprint


class Request:
    def __init__(self, rid, model, arrival, steps=None, tag=None):
        self.rid = rid
        self.model = model
        self.arrival = float(arrival)
        self.steps = len(model["schedule"]) if steps is None else int(steps)
        self.tag = tag


class Result:
    def __init__(self, req):
        self.rid = req.rid
        self.tag = req.tag
        self.latencies = []
        self.admitted = None
        self.finished = None
        self.status = "ok"
        self.error = None
        self.state = None
        self.newton = 0
        self.lin = 0


def serve(requests, budget_bytes=200 << 30, max_active=64, precision="fp32", device="cuda:0",
          keep_state=False, clock=time.perf_counter, sim_factory=None, footprint_fn=None, on_done=None,
          max_large=None, large_bytes=4 << 30, **sim_opts):
    """Run the requests; returns (results by rid, summary dict).

    sim_factory(model) -> handle and footprint_fn(model) -> bytes default to the
    library's Sim on its own stream and sim_footprint.  on_done(result), if
    given, is called from the request's worker thread when it finishes.
    max_large, if given, caps the resident requests whose footprint exceeds
    large_bytes; a waiting request that fits may then be admitted ahead of a
    large one held back by the cap."""
    if sim_factory is None:
        import torch

        def sim_factory(model):
            stream = torch.cuda.Stream(device=device)
            return Sim(model, precision=precision, device=device, stream=stream, **sim_opts)

    if footprint_fn is None:
        def footprint_fn(model):
            return footprint(model, precision, **sim_opts)

    reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
    results = {r.rid: Result(r) for r in reqs}
    pending = collections.deque(reqs)
    waiting = collections.deque()
    lock = threading.Condition()
    state = {"used": 0, "active": 0, "peak_active": 0, "peak_used": 0, "large": 0}
    fps = {}
    threads = []
    t0 = clock()

    def now():
        return clock() - t0

    def worker(req, sim, fp):
        res = results[req.rid]
        ready = max(req.arrival, res.admitted)
        try:
            for k in range(req.steps):
                info = sim.timestep(req.model["schedule"][k])
                done = now()
                res.latencies.append(done - ready)
                res.newton += info["newton_iters"]
                res.lin += info["lin_iters"]
                ready = done
            if keep_state:
                res.state = sim.get_state()
        except L.DpError as e:
            res.status = "failed"
            res.error = str(e)
        finally:
            res.finished = now()
            sim.close()
            del sim
            with lock:
                state["used"] -= fp
                state["active"] -= 1
                if fp > large_bytes:
                    state["large"] -= 1
                lock.notify_all()
            if on_done is not None:
                on_done(res)

    while pending or waiting:
        t = now()
        while pending and pending[0].arrival <= t:
            waiting.append(pending.popleft())
        # admission under the lock only reserves memory and a slot; the handles
        # (device allocation, upload, setup of the topology) are made outside it,
        # so finishing workers never wait behind another model's creation
        admitted = []
        with lock:
            i = 0
            while i < len(waiting) and state["active"] < max_active:
                req = waiting[i]
                if req.rid not in fps:
                    fps[req.rid] = footprint_fn(req.model)
                fp = fps[req.rid]
                if fp > budget_bytes:
                    del waiting[i]
                    results[req.rid].status = "rejected"
                    results[req.rid].error = "footprint %d exceeds the budget" % fp
                    continue
                large = fp > large_bytes
                if large and max_large is not None and state["large"] >= max_large:
                    i += 1  # held back by the cap: later requests may pass it
                    continue
                if state["used"] + fp > budget_bytes:
                    break
                del waiting[i]
                state["used"] += fp
                state["active"] += 1
                state["large"] += 1 if large else 0
                state["peak_active"] = max(state["peak_active"], state["active"])
                state["peak_used"] = max(state["peak_used"], state["used"])
                results[req.rid].admitted = now()
                admitted.append((req, fp))
        for req, fp in admitted:
            try:
                sim = sim_factory(req.model)
            except L.DpError as e:
                results[req.rid].status = "failed"
                results[req.rid].error = str(e)
                results[req.rid].finished = now()
                with lock:
                    state["used"] -= fp
                    state["active"] -= 1
                    if fp > large_bytes:
                        state["large"] -= 1
                    lock.notify_all()
                continue
            th = threading.Thread(target=worker, args=(req, sim, fp), daemon=True)
            threads.append(th)
            th.start()
        if not admitted:
            with lock:
                # sleep until the next arrival or until a model frees memory
                timeout = None
                if pending:
                    timeout = max(0.0, pending[0].arrival - now())
                if waiting or pending:
                    lock.wait(timeout=min(timeout, 0.05) if timeout is not None else 0.05)
    for th in threads:
        th.join()
    t_end = now()
    lat = [x for r in results.values() for x in r.latencies]
    steps = len(lat)
    first = reqs[0].arrival if reqs else 0.0
    makespan = max((r.finished or 0.0) for r in results.values()) - first if reqs else 0.0
    by_tag = {}
    for r in results.values():
        by_tag.setdefault(str(r.tag), []).extend(r.latencies)
    summary = {
        "requests": len(reqs),
        "completed": sum(1 for r in results.values() if r.status == "ok"),
        "failed": sum(1 for r in results.values() if r.status == "failed"),
        "rejected": sum(1 for r in results.values() if r.status == "rejected"),
        "timesteps": steps,
        "makespan_s": makespan,
        "timesteps_per_s": steps / makespan if makespan > 0 else 0.0,
        "p50_step_ms": float(np.percentile(lat, 50)) * 1e3 if lat else None,
        "p99_step_ms": float(np.percentile(lat, 99)) * 1e3 if lat else None,
        "peak_active": state["peak_active"],
        "peak_bytes": state["peak_used"],
        "wall_s": t_end,
        "by_class": {k: {"steps": len(v), "p50_ms": float(np.percentile(v, 50)) * 1e3,
                         "p99_ms": float(np.percentile(v, 99)) * 1e3}
                     for k, v in by_tag.items() if v},
    }
    return results, summary
