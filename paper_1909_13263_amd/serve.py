"""Open-loop driver of the batched server: requests arrive on their own clock.

The client side of the served stream: each request of a workloads.served_stream is
submitted to an hjw.Server once its arrival time has passed, while the server runs
chunks of batched RK3 steps over everything admitted.  Latency is measured from the
scheduled arrival (not from the moment the driver got round to submitting) to the
moment the server had copied the result back to host memory.  All arithmetic runs in
the library; this module only keeps time.
"""
from __future__ import annotations

import time

import numpy as np

from . import hjw


def prepare(requests):
    """Initial data of every request, built before the clock starts (phi0 generation is
    the client's work, not the server's).  Grids of the same problem share one array."""
    cache = {}
    out = []
    for rq in requests:
        p = rq.problem
        key = (p.name, p.shape, p.seed if p.name == "levelset2d" else 0)
        if key not in cache:
            cache[key] = np.ascontiguousarray(p.phi0())
        out.append(cache[key])
    return out


def run_stream(server: hjw.Server, requests, phi0s, time_scale=1.0, chunks=1,
               keep_phi=False, on_result=None):
    """Replay `requests` (arrival seconds x time_scale) against `server` in real time.

    Returns {rid: record} with the request's latency, its solve info and, with
    keep_phi, its phi."""
    order = sorted(range(len(requests)), key=lambda k: requests[k].arrival)
    t0 = server.clock()
    ids = {}
    out = {}
    nxt = 0
    while len(out) < len(requests):
        now = server.clock() - t0
        while nxt < len(order) and requests[order[nxt]].arrival * time_scale <= now:
            k = order[nxt]
            ids[server.submit(requests[k].problem, phi0s[k])] = k
            nxt += 1
        active, queued = server.run(chunks)
        for sid in server.completed():
            res = server.result(sid)
            k = ids.pop(sid)
            rq = requests[k]
            arrival = t0 + rq.arrival * time_scale
            rec = {"rid": rq.rid, "status": res.status, "latency": res.t_finish - arrival,
                   "queue_and_run": res.latency, "cells": rq.problem.cells,
                   "steps": res.info.steps, "t": res.info.t, "info": res.info}
            if keep_phi:
                rec["phi"] = res.phi
            out[rq.rid] = rec
            if on_result is not None:
                on_result(rec)
        if active == 0 and queued == 0 and nxt < len(order):
            wait = t0 + requests[order[nxt]].arrival * time_scale - server.clock()
            if wait > 0:
                time.sleep(wait)
    return out


def saturation(server: hjw.Server, requests, phi0s, chunks=4):
    """Closed-loop throughput: submit everything at once and drain.  Returns
    (requests per second, cell-stages per second, wall seconds)."""
    before = server.stats()["node_stages"]
    t0 = time.perf_counter()
    for rq, phi0 in zip(requests, phi0s):
        server.submit(rq.problem, phi0)
    done = server.drain(chunks)
    wall = time.perf_counter() - t0
    bad = [r for r in done if r.status != hjw.OK]
    if bad:
        raise RuntimeError(f"{len(bad)} requests failed while measuring saturation")
    stages = server.stats()["node_stages"] - before
    return len(requests) / wall, stages / wall, wall


def sustained(server: hjw.Server, requests, phi0s, outstanding=128, warm=64, chunks=1):
    """Closed-loop throughput with the server kept full: `outstanding` requests are in the
    server at all times (a new one is submitted as each finishes, in list order).  Timed
    from the `warm`-th completion until the list is exhausted, so that neither the ramp
    nor the final drain (where the last long solves run alone) enters the figure.
    Returns (requests per second, cell-stages per second, wall seconds, requests timed)."""
    if not 0 < warm < len(requests) - outstanding:
        raise ValueError(f"sustained: need 0 < warm < len(requests) - outstanding "
                         f"({warm}, {len(requests)}, {outstanding})")
    nxt = 0
    inflight = 0
    done = 0
    t0 = st0 = None
    done0 = 0
    while nxt < len(requests):
        while inflight < outstanding and nxt < len(requests):
            server.submit(requests[nxt].problem, phi0s[nxt])
            nxt += 1
            inflight += 1
        server.run(chunks)
        for sid in server.completed():
            res = server.result(sid)
            if res.status != hjw.OK:
                raise RuntimeError("a request failed while measuring sustained throughput")
            inflight -= 1
            done += 1
            if t0 is None and done >= warm:
                t0, st0, done0 = time.perf_counter(), server.stats()["node_stages"], done
    if t0 is None:
        raise ValueError("too few requests to time")
    wall = time.perf_counter() - t0
    stages = server.stats()["node_stages"] - st0
    timed = done - done0
    server.drain()
    return timed / wall, stages / wall, wall, timed


def summarize(records, wall):
    lat = np.array([r["latency"] for r in records.values()])
    ok = [r for r in records.values() if r["status"] == hjw.OK]
    return {
        "requests": len(records),
        "failed": len(records) - len(ok),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p90_ms": float(np.percentile(lat, 90) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "max_ms": float(lat.max() * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
        "cell_updates": float(sum(3.0 * r["cells"] * r["steps"] for r in ok)),
        "wall_s": wall,
    }
