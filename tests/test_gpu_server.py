"""GPU tests of the batched server (continuous batching of many solves).

Bars: a solve's phi from the server is bitwise the phi of the same solve run alone
through the server, and bitwise the phi of hjw_step_to on a single grid with the same
precision (the same stage code runs per tile; the dissipation's min/max reductions are
exact, so neither the batch nor the order of workgroups changes a value).  The FP64
server matches the FP64 oracle to 1e-12 of max|phi|.  Admission never holds more pool
bytes than the pool has, nor more solves than max_active; a failing solve is retired
alone.
"""
import dataclasses
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_1909_13263_amd import hjw
from paper_1909_13263_amd import serve as S
from paper_1909_13263_amd import workloads as W

pytestmark = pytest.mark.gpu

FP64, MIXED, FP32 = hjw.FP64, hjw.FP32_MIXED, hjw.FP32


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "these tests need the GPU"
    assert os.path.dirname(hjw.LIB_PATH).endswith("paper_1909_13263_amd")
    yield


def _mix(count, seed, n_min=40, n_max=200, t_lo=0.01, t_hi=0.05):
    """A small stream shaped like the served workload: ragged square and non-square grids,
    the three 2-D Hamiltonians with their phi0, short horizons."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.integers(n_min, n_max + 1))
        ny = n if rng.random() < 0.7 else int(rng.integers(n_min, n_max + 1))
        tf = float(rng.uniform(t_lo, t_hi))
        kind = int(rng.integers(0, 3))
        if kind == 0:
            p = W.burgers2d(n, tf, ny=ny)
        elif kind == 1:
            p = W.negcos2d(n, tf, ny=ny)
        else:
            p = W.levelset2d(n, tf, seed=int(rng.integers(0, 2**31 - 1)), ny=ny)
        out.append(W.Request(i, 0.0, p))
    return out


def _alone(reqs, prec):
    srv = hjw.Server(prec, pool_bytes=64 << 20, max_active=4)
    out = {}
    for rq in reqs:
        srv.submit(rq.problem)
        res = srv.drain()
        assert len(res) == 1 and res[0].status == hjw.OK
        out[rq.rid] = res[0]
    srv.close()
    return out


@pytest.mark.parametrize("prec", [FP64, MIXED, FP32])
def test_server_matches_single_grid_step_to(prec):
    reqs = _mix(5, seed=11 + prec)
    alone = _alone(reqs, prec)
    for rq in reqs:
        pr = rq.problem
        g = hjw.grid_for(pr, prec)
        g.set_phi(pr.phi0())
        info = g.step_to(pr.t_final, pr.cfl)
        ref = g.get_phi()
        g.close()
        res = alone[rq.rid]
        assert res.info.steps == info.steps and res.info.t == info.t, (pr, res.info, info)
        assert np.array_equal(res.phi, ref), (pr.name, pr.shape, np.abs(res.phi - ref).max())


def test_fp64_server_matches_oracle():
    reqs = [W.Request(0, 0.0, W.burgers2d(72, 0.03)), W.Request(1, 0.0, W.levelset2d(90, 0.03)),
            W.Request(2, 0.0, W.negcos2d(100, 0.05, ny=70))]
    alone = _alone(reqs, FP64)
    for rq in reqs:
        pr = rq.problem
        ref, info = O.step_to(O.Problem(pr.shape, pr.spacing, pr.ham, pr.params, pr.bc),
                              pr.phi0(), pr.t_final, pr.cfl)
        res = alone[rq.rid]
        assert res.info.steps == info.steps
        err = float(np.abs(res.phi - ref).max() / np.abs(ref).max())
        assert err <= 1e-12, (pr.name, err)


@pytest.mark.parametrize("prec", [MIXED, FP32])
def test_each_result_is_the_same_alone_and_in_the_mix(prec):
    """40 requests submitted together to a server that holds at most 6 at once and whose
    pool holds about four of the largest: requests wait, are admitted as others retire,
    and share every launch with different neighbours than when run alone."""
    reqs = _mix(40, seed=1909 + prec)
    alone = _alone(reqs, prec)
    big = max(hjw.Server.footprint(rq.problem, prec) for rq in reqs)
    srv = hjw.Server(prec, pool_bytes=4 * big + (1 << 20), max_active=6)
    pool = srv.stats()["pool_bytes"]
    ids = {srv.submit(rq.problem): rq.rid for rq in reqs}
    seen_queue = 0
    results = {}
    while True:
        act, que = srv.run(1)
        assert act <= 6
        seen_queue = max(seen_queue, que)
        st = srv.stats()
        assert st["pool_in_use"] <= pool
        for sid in srv.completed():
            results[ids[sid]] = srv.result(sid)
        if act == 0 and que == 0:
            break
    st = srv.stats()
    assert st["pool_peak"] <= pool and st["pool_in_use"] == 0
    assert seen_queue > 0 and st["done"] == len(reqs) and st["failed"] == 0
    assert len(results) == len(reqs)
    for rq in reqs:
        a, m = alone[rq.rid], results[rq.rid]
        assert m.status == hjw.OK
        assert m.info.steps == a.info.steps and m.info.t == a.info.t
        assert np.array_equal(m.phi, a.phi), (rq.problem.name, rq.problem.shape)
    srv.close()


def test_open_loop_stream_matches_alone():
    """The real-time driver: Poisson arrivals replayed on the server's clock."""
    base = _mix(24, seed=77)
    rng = np.random.default_rng(5)
    arrivals = np.cumsum(rng.exponential(0.004, size=len(base)))
    reqs = [W.Request(rq.rid, float(t), rq.problem) for rq, t in zip(base, arrivals)]
    alone = _alone(reqs, MIXED)
    srv = hjw.Server(MIXED, pool_bytes=256 << 20, max_active=16)
    recs = S.run_stream(srv, reqs, S.prepare(reqs), keep_phi=True)
    summary = S.summarize(recs, 1.0)
    assert summary["failed"] == 0 and summary["requests"] == len(reqs)
    assert 0 < summary["p50_ms"] <= summary["p99_ms"]
    for rq in reqs:
        assert np.array_equal(recs[rq.rid]["phi"], alone[rq.rid].phi)
    srv.close()


def test_failures_are_isolated():
    """A request that blows up is retired alone with ENONFINITE; a non-finite phi0 and a
    request larger than the pool are refused at submission; the rest are unaffected."""
    reqs = _mix(8, seed=3)
    alone = _alone(reqs, MIXED)
    srv = hjw.Server(MIXED, pool_bytes=32 << 20, max_active=8)
    bad = W.burgers2d(64, 50.0)
    bad = dataclasses.replace(bad, cfl=40.0)
    with pytest.raises(hjw.HJWError) as e:
        srv.submit(W.burgers2d(64, 0.1), np.full((64, 64), np.nan))
    assert e.value.code == hjw.ENONFINITE
    with pytest.raises(hjw.HJWError) as e:
        srv.submit(W.burgers2d(2048, 0.1))
    assert e.value.code == hjw.ENOMEM
    ids = {}
    for k, rq in enumerate(reqs):
        ids[srv.submit(rq.problem)] = rq.rid
        if k == 3:
            bad_id = srv.submit(bad, bad.phi0() * 1e3)
    with pytest.raises(hjw.HJWError) as e:
        srv.result(bad_id)                       # not finished yet
    assert e.value.code == hjw.ESTATE
    results = {}
    failed = []
    while True:
        act, que = srv.run(1)
        for sid in srv.completed():
            res = srv.result(sid)
            if sid == bad_id:
                failed.append(res)
            else:
                results[ids[sid]] = res
        if act == 0 and que == 0:
            break
    assert len(failed) == 1 and failed[0].status == hjw.ENONFINITE and failed[0].phi is None
    st = srv.stats()
    assert st["failed"] == 1 and st["done"] == len(reqs) and st["pool_in_use"] == 0
    for rq in reqs:
        assert np.array_equal(results[rq.rid].phi, alone[rq.rid].phi)
    with pytest.raises(KeyError):
        srv.result(bad_id)                       # released
    srv.close()


def test_served_workload_sample_holds_fp32_bound():
    """A few requests of the served stream itself (sides 64..1024, t_final up to 0.5),
    FP32 stencil with FP64 phi, against the FP64 single-grid path: relative L-inf error
    below 2e-5."""
    stream = W.served_stream(count=64)
    pick = [rq for rq in stream if rq.problem.cells <= 300 * 300][:4]
    srv = hjw.Server(MIXED, pool_bytes=256 << 20, max_active=8)
    recs = S.run_stream(srv, pick, S.prepare(pick), time_scale=0.0, keep_phi=True)
    for rq in pick:
        pr = rq.problem
        g = hjw.grid_for(pr, FP64)
        g.set_phi(pr.phi0())
        g.step_to(pr.t_final, pr.cfl)
        ref = g.get_phi()
        g.close()
        err = float(np.abs(recs[rq.rid]["phi"] - ref).max() / np.abs(ref).max())
        assert err < 2e-5, (pr.name, pr.shape, pr.t_final, err)
    srv.close()


def test_mixed_schemes_in_one_batch():
    """WENO-L and WENO-JP requests share the batched launches; each matches hjw_step_to
    with its own scheme bit for bit."""
    reqs = _mix(10, seed=31)
    schemes = [hjw.WENO_JP if k % 2 else hjw.WENO_L for k in range(len(reqs))]
    srv = hjw.Server(MIXED, pool_bytes=128 << 20, max_active=8)
    ids = {srv.submit(rq.problem, scheme=sc): (rq, sc) for rq, sc in zip(reqs, schemes)}
    results = {r.rid: r for r in srv.drain()}
    srv.close()
    assert len(results) == len(reqs)
    for sid, (rq, sc) in ids.items():
        pr = rq.problem
        g = hjw.grid_for(pr, MIXED, scheme=sc)
        g.set_phi(pr.phi0())
        g.step_to(pr.t_final, pr.cfl)
        ref = g.get_phi()
        g.close()
        assert results[sid].status == hjw.OK
        assert np.array_equal(results[sid].phi, ref), (pr.name, pr.shape, sc)


def test_phi0_is_checked_on_both_submission_paths():
    """phi0 is copied at submission either into the pinned inbox (a quarter of the pool) or,
    when it does not fit there, into host memory; both copies test every value.  A single
    infinity at the last node or in the middle is refused on either path, and requests that
    pass solve to their single-grid results."""
    srv = hjw.Server(MIXED, pool_bytes=24 << 20, max_active=2)   # inbox 6 MiB
    small = W.burgers2d(64, 0.01)       # 32 KB of phi0: the inbox
    big = W.burgers2d(900, 0.002)       # 6.5 MB of phi0: host memory
    for pr in (small, big):
        for where in (-1, pr.shape[0] * pr.shape[1] // 2):
            phi = pr.phi0().copy()
            phi.flat[where] = np.inf if where < 0 else -np.inf
            with pytest.raises(hjw.HJWError) as e:
                srv.submit(pr, phi)
            assert e.value.code == hjw.ENONFINITE
    srv.submit(big)
    srv.submit(small)
    done = srv.drain()
    st = srv.stats()
    srv.close()
    assert len(done) == 2 and st["done"] == 2 and st["pool_in_use"] == 0
    for res in done:
        pr = big if res.phi.shape == big.shape else small
        g = hjw.grid_for(pr, MIXED)
        g.set_phi(pr.phi0())
        info = g.step_to(pr.t_final, pr.cfl)
        ref = g.get_phi()
        g.close()
        assert res.status == hjw.OK and res.info.steps == info.steps
        assert np.array_equal(res.phi, ref)


def test_bursts_larger_than_one_staging_step():
    """Forty 1200^2 solves (11.5 MB of phi0 and of result each, 460 MB in all) submitted at
    once: the pinned inbox (a quarter of the 1.4 GB pool) takes the phi0 of the first ~30,
    the rest wait in host memory and are admitted through pinned staging; retirement moves
    at most 256 MiB through staging per step, so the two groups (long horizons first, short
    ones second) finish in the same chunk and retire over two steps.  Every result is the
    single-grid result of its own phi0, bit for bit."""
    n = 1200
    reqs = []
    for k in range(40):
        pr = W.burgers2d(n, 0.004 if k < 23 else 0.001)
        reqs.append((pr, pr.phi0() * (1.0 + 0.01 * k)))
    big = hjw.Server.footprint(reqs[0][0], MIXED)
    srv = hjw.Server(MIXED, pool_bytes=41 * big, max_active=64)
    ids = {srv.submit(pr, phi0): k for k, (pr, phi0) in enumerate(reqs)}
    results = {}
    while True:
        act, que = srv.run(1)
        for sid in srv.completed():
            results[ids[sid]] = srv.result(sid)
        if act == 0 and que == 0:
            break
    st = srv.stats()
    srv.close()
    assert len(results) == len(reqs) and st["done"] == len(reqs) and st["pool_in_use"] == 0
    for k, (pr, phi0) in enumerate(reqs):
        g = hjw.grid_for(pr, MIXED)
        g.set_phi(phi0)
        info = g.step_to(pr.t_final, pr.cfl)
        ref = g.get_phi()
        g.close()
        res = results[k]
        assert res.status == hjw.OK and res.info.steps == info.steps and res.info.t == info.t
        assert np.array_equal(res.phi, ref), (k, np.abs(res.phi - ref).max())


def test_sustained_closed_loop_keeps_the_server_full():
    """The closed-loop throughput driver: a fixed number of requests stays in the server,
    every request completes with its single-grid result, and the figure is positive."""
    reqs = _mix(48, seed=91)
    srv = hjw.Server(MIXED, pool_bytes=128 << 20, max_active=16)
    seen = []
    orig_submit = srv.submit

    def submit(problem, phi0=None, scheme=hjw.WENO_L):
        st = srv.stats()
        seen.append(st["active"] + st["queued"])
        return orig_submit(problem, phi0, scheme)

    srv.submit = submit
    rps, cells, wall, timed = S.sustained(srv, reqs, S.prepare(reqs), outstanding=8, warm=8)
    st = srv.stats()
    srv.close()
    assert rps > 0 and cells > 0 and wall > 0 and 0 < timed <= len(reqs)
    assert max(seen) <= 8
    assert st["done"] == len(reqs) and st["failed"] == 0 and st["pool_in_use"] == 0
