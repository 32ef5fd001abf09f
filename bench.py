"""Benchmark: cell-updates/s per RK3 stage of the WENO-L solver on one MI355X.

One benchmark step is one whole solve of the 2-D Burgers problem of Example 3.3 scaled
to a 1024 x 1024 periodic grid on [-2,2)^2, phi0 = -cos(pi(x+y)/2), CFL 0.5, from t = 0
to t = 0.5/pi^2: every RK3 step (derivative ranges -> dissipation -> time step -> three
fused stages) runs on the GPU, from phi0 already resident in HBM.

value = cells x RK stages / wall time for the FP32-stencil path (FP64 phi, FP64 time step
and accumulation); the FP64 path is timed the same way and reported beside it.  The
roofline object describes the dominant kernel, timed with HIP events on the library's
stream during an instrumented solve that follows the timed region.  cpu_baseline is the
FP64 oracle on the host cores, on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0                     # MI355X HBM3E, 8 TB/s
# Vector ALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39,322 G lane-slots/s
# (one lane-operation per lane per clock, packed FP32 not used).
VALU_PEAK_GSLOTS = 256 * 4 * 16 * 2.4
# Algorithmic vector work of one node-stage in 2-D: about 200 add/mul/FMA plus 28
# square roots, logarithms, divisions and reciprocals (6 + 6 + 12 + 4), the latter at
# quarter rate (4 slots each): 200 + 28 * 4 = 312 lane-slots.
ALGO_SLOTS_PER_CELL = 200 + 28 * 4
METRIC = "cell-updates/s per RK3 stage (FP32 vs FP64, %HBM peak); served p50/p99 latency"

# Compulsory HBM bytes per node of each kernel of a step (read stage inputs once, write
# outputs once) for (phi bytes, flux bytes).
def kernel_bytes_per_cell(phi_b, flux_b):
    return {
        "pre": phi_b + 3 * flux_b,                 # read phi^n; write Hbar, Dx, Dy
        "mid": phi_b + 3 * flux_b + phi_b,         # read phi^n, Hbar, Dx, Dy; write phi_2
        "last": 2 * phi_b + phi_b,                 # read phi^n, phi_2; write phi^{n+1}
    }


# HBM bytes per launch of the FP32-stencil kernels on the benchmark grid, from rocprofv3
# counters: FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (KiB), the factors being what the same
# counters read for a plain 256 MiB copy kernel.  Valid only for the kernel sources whose
# SHA-256 is recorded; any change to them turns the figure into null until re-measured.
MEASURED_TRAFFIC = {"source_sha256": "663aefb64534659ba604393a3e29cff09e1d4a8af198da0478907b0d0c0887f2",
                    "n": 1024, "tile_rows": 16,
                    "bytes": {"pre": 22120000, "mid": 31040000, "last": 26160000}}


def segment(n):
    """Nodes per thread the library picks for the FP32 stencil on an n x n grid (4 on
    grids of at most 640 tiles of 64 x 16, else 8)."""
    tiles = -(-n // 64) * -(-n // 16)
    return 4 if tiles <= 640 else 8


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for f in ("hjw_tile.h", "hjw_kernels.h", "hjw_common.h", "hjw.hip"):
        with open(os.path.join(ROOT, "paper_1909_13263_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1024)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--tile-rows", type=int, default=0, help="16 or 32 (0: library default)")
    ap.add_argument("--no-serve", action="store_true", help="skip the served stream")
    ap.add_argument("--no-jp", action="store_true", help="skip the WENO-JP comparison solve")
    ap.add_argument("--no-families", action="store_true",
                    help="skip the kernel times of the other Hamiltonians and boundaries")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the FP32-vs-FP64 error of the full-size configurations")
    ap.add_argument("--serve-requests", type=int, default=2048)
    ap.add_argument("--serve-load", type=float, default=0.7,
                    help="arrival rate as a fraction of the measured saturation rate")
    ap.add_argument("--serve-pool-gib", type=float, default=4.0)
    ap.add_argument("--serve-max-active", type=int, default=256)
    ap.add_argument("--serve-sat-sample", type=int, default=256,
                    help="requests submitted at once to measure the saturation rate")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 256 MiB device-to-device copy (counter calibration)")
    ap.add_argument("--profile", choices=sorted(PROFILE_PRECS),
                    help="only run the stage kernels of the --workload on an --n grid in this "
                         "precision: --profile-steps real steps, then --profile-reps launches of "
                         "each kernel back to back (a short target for counter collection)")
    ap.add_argument("--workload", default="burgers2d", choices=sorted(PROFILE_WORKLOADS))
    ap.add_argument("--profile-steps", type=int, default=4)
    ap.add_argument("--profile-reps", type=int, default=20)
    return ap.parse_args()


PROFILE_PRECS = {"fp64": 0, "fp32_stencil": 1, "fp32": 2}
PROFILE_WORKLOADS = {"burgers2d": "burgers2d", "negcos2d": "negcos2d", "levelset2d": "levelset2d"}


def profile_target(args):
    """Stage kernels only, for rocprofv3: a grid of the workload, --profile-steps whole steps
    from phi0 (every kernel does a step), then hjw_time_kernels' launches of each kernel."""
    import torch

    from paper_1909_13263_amd import hjw
    from paper_1909_13263_amd import workloads as W
    pr = getattr(W, PROFILE_WORKLOADS[args.workload])(args.n)
    prec = PROFILE_PRECS[args.profile]
    g = hjw.grid_for(pr, prec)
    g.set_phi(torch.from_numpy(pr.phi0()).to("cuda"))
    info = g.step_to(pr.t_final, pr.cfl, max_steps=args.profile_steps)
    times = g.time_kernels(reps=args.profile_reps)
    g.close()
    print(json.dumps({"profile": args.profile, "workload": args.workload, "n": args.n,
                      "cells": pr.cells, "steps": info.steps, "reps": args.profile_reps,
                      "kernel_ms": times}))
    return 0


def calibrate_copy():
    """A plain copy of known size: what FETCH_SIZE / WRITE_SIZE read for 256 MiB."""
    import torch
    n = 256 * 1024 * 1024
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": n, "launches": 3}))
    return 0


def time_solves(hjw, pr, prec, phi_dev, steps, warmup, tile_rows=0, scheme=0):
    import torch
    g = hjw.grid_for(pr, prec, scheme=scheme)
    if tile_rows:
        g.set_option(hjw.OPT_TILE_ROWS, tile_rows)
    info = None
    for _ in range(warmup):
        g.set_phi(phi_dev)
        info = g.step_to(pr.t_final, pr.cfl)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.set_phi(phi_dev)
        info = g.step_to(pr.t_final, pr.cfl)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # kernel durations: each stage kernel launched back to back between HIP events on
    # the library's stream (queued behind a hold kernel, after two untimed launches), on
    # this grid and data, right after the timed region
    g.set_phi(phi_dev)
    times = g.time_kernels(reps=50)
    g.close()
    return wall, info, times


def cpu_baseline(pr, seconds):
    """The FP64 oracle on the host: whole RK3 steps of the same grid until `seconds` pass."""
    import oracle as O
    prob = O.Problem(pr.shape, pr.spacing, pr.ham, pr.params, pr.bc)
    phi = pr.phi0()
    steps = 0
    t = 0.0
    t0 = time.perf_counter()
    while True:
        phi, info = O.rk3_step(prob, phi, t, pr.t_final, pr.cfl)
        t = info.t
        steps += 1
        if time.perf_counter() - t0 >= seconds or t >= pr.t_final:
            break
    wall = time.perf_counter() - t0
    cores = O.threads()   # the OpenMP team the oracle's loops ran on
    out = {"value": pr.cells * 3 * steps / wall, "unit": "cell-updates/s", "cores": cores,
           "kind": "oracle",
           "sample": f"{steps} RK3 steps of the {pr.shape[1]}x{pr.shape[0]} grid from t=0 "
                     f"({wall:.1f} s, FP64 C, OpenMP over grid lines)",
           "cpu_model": cpu_model(),
           "affinity_cpus": len(os.sched_getaffinity(0)),
           "online_cpus": os.cpu_count()}
    one = single_core_rate(pr, max(2.0, seconds / 4))
    if one is not None:
        out["single_core_value"] = one
    return out


def cpu_model():
    """The host CPU as /proc/cpuinfo names it: model name, family/model/stepping, and the
    clock and cache it reports (virtualised hosts may give only a short model name)."""
    info = {}
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if not line.strip():
                    break   # the first processor's block
                k, _, v = line.partition(":")
                info[k.strip()] = v.strip()
    except OSError:
        return None
    parts = [info.get("model name", "unknown")]
    if "cpu family" in info:
        parts.append(f"family {info['cpu family']} model {info.get('model', '?')} "
                     f"stepping {info.get('stepping', '?')}")
    if "cpu MHz" in info:
        parts.append(f"{float(info['cpu MHz']):.0f} MHz")
    if "cache size" in info:
        parts.append(f"cache {info['cache size']}")
    return ", ".join(parts)


def single_core_rate(pr, seconds):
    """The same oracle steps on one thread, in a child process (OMP_NUM_THREADS=1)."""
    import subprocess
    code = (
        "import sys, time, json; sys.path.insert(0, %r)\n"
        "import oracle as O\n"
        "from paper_1909_13263_amd import workloads as W\n"
        "pr = W.burgers2d(%d, %r)\n"
        "prob = O.Problem(pr.shape, pr.spacing, pr.ham, pr.params, pr.bc)\n"
        "phi = pr.phi0(); t = 0.0; n = 0; t0 = time.perf_counter()\n"
        "while time.perf_counter() - t0 < %r and t < pr.t_final:\n"
        "    phi, info = O.rk3_step(prob, phi, t, pr.t_final, pr.cfl); t = info.t; n += 1\n"
        "print(json.dumps({'rate': pr.cells * 3 * n / (time.perf_counter() - t0)}))\n"
    ) % (ROOT, pr.shape[1], pr.t_final, seconds)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                           timeout=seconds * 4 + 60)
        return json.loads(r.stdout.strip().splitlines()[-1])["rate"] if r.returncode == 0 else None
    except (subprocess.SubprocessError, ValueError, IndexError):
        return None


def accuracy_cases():
    """The full-size configurations whose FP32 error is reported: (label, problem, precs)."""
    from paper_1909_13263_amd import workloads as W
    from paper_1909_13263_amd import hjw
    return [
        ("burgers2d 1024^2 t=0.5/pi^2", W.burgers2d(1024, 0.5 / math.pi**2),
         (hjw.FP32_MIXED, hjw.FP32)),
        ("burgers2d 1024^2 t=1.5/pi^2", W.burgers2d(1024, 1.5 / math.pi**2),
         (hjw.FP32_MIXED, hjw.FP32)),
        ("negcos2d 2048^2 t=1.0", W.negcos2d(2048, 1.0), (hjw.FP32_MIXED,)),
        ("levelset2d 4096^2 t=0.2", W.levelset2d(4096, 0.2), (hjw.FP32_MIXED, hjw.FP32)),
    ]


def solve_once(hjw, pr, prec):
    """One whole solve; returns (phi, info, node-stages/s of step_to with phi0 resident)."""
    import torch
    g = hjw.grid_for(pr, prec)
    g.set_phi(pr.phi0())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info = g.step_to(pr.t_final, pr.cfl)   # returns once the solve is done
    wall = time.perf_counter() - t0
    phi = g.get_phi()
    g.close()
    return phi, info, pr.cells * info.steps * 3 / wall


def accuracy(hjw):
    """Error of the FP32 paths against FP64 on the same GPU, whose results match the
    FP64 oracle to 1e-12 of max|phi| (the parity tests): L-inf; L1 as the grid mean of
    |error| and as the domain integral dx dy sum|error|; L-inf and mean L1 also relative
    to max|phi|.  Each whole solve's node-stages/s (phi0 resident, step_to timed) rides
    along: the full-size configurations' throughput in both precisions."""
    out = {}
    for label, pr, precs in accuracy_cases():
        ref, info, rate64 = solve_once(hjw, pr, hjw.FP64)
        scale = float(np.abs(ref).max())
        row = {"fp64_steps": info.steps, "fp64_cell_updates_per_s": rate64}
        for prec in precs:
            phi, pinfo, rate = solve_once(hjw, pr, prec)
            err = np.abs(phi - ref)
            name = {hjw.FP32_MIXED: "fp32_stencil", hjw.FP32: "fp32_storage"}[prec]
            cell = float(np.prod(pr.spacing))
            row[name] = {"linf": float(err.max()), "l1": float(err.mean()),
                         "l1_integral": float(err.sum()) * cell,
                         "linf_rel": float(err.max()) / scale, "l1_rel": float(err.mean()) / scale,
                         "steps": pinfo.steps, "cell_updates_per_s": rate}
        out[label] = row
    return out


def beyond_mall(hjw, W, steps=3):
    """A grid whose working set (phi, stage buffer, flux records: 28 B per node) exceeds
    the 256 MB Infinity Cache: 4096^2 Burgers, FP32 stencil, whole solves to 0.1/pi^2."""
    import torch
    pr = W.burgers2d(4096, 0.1 / math.pi**2)
    phi_dev = torch.from_numpy(pr.phi0()).to("cuda")
    g = hjw.grid_for(pr, hjw.FP32_MIXED)
    g.set_phi(phi_dev)
    info = g.step_to(pr.t_final, pr.cfl)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.set_phi(phi_dev)
        info = g.step_to(pr.t_final, pr.cfl)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    g.close()
    rate = pr.cells * 3 * info.steps / wall
    step_bytes = sum(kernel_bytes_per_cell(8, 4).values()) / 3.0   # per node-stage
    return {"grid": "4096x4096 burgers2d, t=0.1/pi^2", "working_set_MB": pr.cells * 28 / 1e6,
            "rk_steps": info.steps, "ms_per_solve": wall * 1e3, "cell_updates_per_s": rate,
            "sustained_GBps": rate * step_bytes / 1e9,
            "sustained_frac": rate * step_bytes / 1e9 / HBM_PEAK_GBS}


def families(hjw, W, n):
    """Stage-kernel throughput of every Hamiltonian family and boundary the solver has, on
    an n x n grid with the FP32 stencil in the benchmark's launch configuration: each stage
    kernel launched back to back between HIP events.  Node-stages/s = n^2 * 3 / (pre + mid
    + last)."""
    import dataclasses
    cases = [
        ("burgers, periodic (Ex 3.3)", W.burgers2d(n), None),
        ("-cos, periodic (Ex 3.4)", W.negcos2d(n), None),
        ("quartic, periodic (Ex 3.8 in 2-D)",
         dataclasses.replace(W.burgers2d(n), ham=W.H_QUARTIC, params=(1.0, 1.0, 0.0)), None),
        ("sin, Dirichlet (Ex 3.10)", W.ex310_sin2d(n), None),
        ("control, periodic (Ex 3.11)", W.ex311_control(n),
         W.random_smooth_periodic((n, n), seed=3)),
        ("sqrt form, periodic (Ex 3.12)", W.ex312_eikonal(n), None),
        ("curvature eps=0.1, periodic (Ex 3.13)", W.ex313_curvature(n, 0.1), None),
        ("norm, extrapolated (level set)", W.levelset2d(n), None),
        ("H(x,t,phi,Dphi): cos(wt)(au+bv)+lam phi, periodic (eq. 1.1)",
         W.timed2d(n, 0.8, -0.6, 5.0, 0.9), None),
    ]
    out = {}
    base = None
    for label, pr, phi in cases:
        g = hjw.grid_for(pr, hjw.FP32_MIXED)
        phi0 = pr.phi0() if phi is None else phi
        # the first pass brings the clocks up after the host-side set-up; the second counts
        for _ in range(2):
            g.set_phi(phi0)
            t = g.time_kernels(reps=200)
        g.close()
        total = t["pre"] + t["plan"] + t["mid"] + t["last"]
        rate = pr.cells * 3 / (total * 1e-3)
        base = base or rate
        out[label] = {"kernel_ms": t, "node_stages_per_s": rate, "vs_burgers": rate / base}
    return out


def served_stream(args, hjw):
    """The served stream: Poisson arrivals of mixed solves at a fraction of the measured
    saturation rate, continuous batching on one pool; p50/p99 latency and throughput."""
    from paper_1909_13263_amd import serve as S
    from paper_1909_13263_amd import workloads as W
    reqs = W.served_stream(count=args.serve_requests, rate=1.0)
    t0 = time.perf_counter()
    phi0s = S.prepare(reqs)
    prep = time.perf_counter() - t0
    pool = int(args.serve_pool_gib * (1 << 30))
    srv = hjw.Server(hjw.FP32_MIXED, pool_bytes=pool, max_active=args.serve_max_active)
    # warm the graphs and the code paths, then measure the saturation rate: a sample of
    # the stream submitted at once and drained
    S.saturation(srv, reqs[:16], phi0s[:16])
    k = min(args.serve_sat_sample, len(reqs))
    sat_rps, sat_cells, sat_wall = S.saturation(srv, reqs[-k:], phi0s[-k:])
    rate = args.serve_load * sat_rps
    before = srv.stats()
    t1 = time.perf_counter()
    recs = S.run_stream(srv, reqs, phi0s, time_scale=1.0 / rate)
    wall = time.perf_counter() - t1
    after = srv.stats()
    summary = S.summarize(recs, wall)
    srv.close()
    return {
        "requests": summary["requests"], "failed": summary["failed"],
        "precision": "f32 stencil, f64 phi/dt/accumulation",
        "arrival_rate_rps": rate, "load": args.serve_load,
        "saturation_rps": sat_rps, "saturation_cell_updates_per_s": sat_cells,
        "saturation_sample": f"last {k} requests of the stream submitted at once ({sat_wall:.1f} s)",
        "p50_ms": summary["p50_ms"], "p90_ms": summary["p90_ms"], "p99_ms": summary["p99_ms"],
        "max_ms": summary["max_ms"], "mean_ms": summary["mean_ms"],
        "cell_updates_per_s": summary["cell_updates"] / wall,
        "wall_s": wall, "batched_steps": after["batched_steps"] - before["batched_steps"],
        "pool_gib": args.serve_pool_gib, "pool_peak_gib": after["pool_peak"] / (1 << 30),
        "max_active": args.serve_max_active, "phi0_prep_s": prep,
        "latency_from": "scheduled arrival to result in host memory",
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the solver runs each grid on a single device).", file=sys.stderr)
        return 2
    import torch

    from paper_1909_13263_amd import hjw
    from paper_1909_13263_amd import workloads as W

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        return calibrate_copy()
    if args.profile:
        return profile_target(args)
    pr = W.burgers2d(args.n, 0.5 / math.pi**2)
    phi_dev = torch.from_numpy(pr.phi0()).to("cuda")
    cells = pr.cells

    results = {}
    for name, prec in [("fp32", hjw.FP32_MIXED), ("fp64", hjw.FP64)]:
        if name == "fp64" and args.skip_fp64:
            continue
        wall, info, times = time_solves(hjw, pr, prec, phi_dev, args.steps, args.warmup,
                                        args.tile_rows)
        stages = 3 * info.steps
        results[name] = {"wall": wall, "rk_steps": info.steps, "stages": stages,
                         "cell_updates_per_s": cells * stages * args.steps / wall,
                         "ms_per_solve": 1e3 * wall / args.steps, "kernels": times}

    main_res = results["fp32"]
    # dominant kernel of the FP32-stencil path
    ktimes = main_res["kernels"]
    dom = max(("pre", "mid", "last"), key=lambda k: ktimes[k])
    dom_ms = ktimes[dom]
    bpc = kernel_bytes_per_cell(8, 4)[dom]
    hbm_gbs = bpc * cells / (dom_ms * 1e-3) / 1e9
    alu_achieved = ALGO_SLOTS_PER_CELL * cells / (dom_ms * 1e-3) / 1e9
    traffic = None
    if (MEASURED_TRAFFIC["source_sha256"] == kernel_source_sha()
            and args.n == MEASURED_TRAFFIC["n"] and args.tile_rows in (0, MEASURED_TRAFFIC["tile_rows"])):
        traffic = MEASURED_TRAFFIC["bytes"].get(dom)
    # whole-step compulsory bytes per cell-stage: (8 + 8+8 + 8+8 ... ) averaged over stages
    step_bytes = sum(kernel_bytes_per_cell(8, 4).values())
    sustained = step_bytes * cells * main_res["rk_steps"] * args.steps / main_res["wall"] / 1e9

    line = {
        "metric": METRIC,
        "value": main_res["cell_updates_per_s"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_res["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 stencil, f64 phi/dt/accumulation",
        "data": "synthetic",
        "config": {"workload": f"burgers2d {args.n}x{args.n} periodic [-2,2)^2, "
                               "phi0=-cos(pi(x+y)/2), H=(p+q+1)^2/2, LF, TVD-RK3, CFL 0.5, "
                               "t=0.5/pi^2",
                   "cells": cells, "rk_steps": main_res["rk_steps"],
                   "stages_per_solve": main_res["stages"]},
        "roofline": {"bound": "alu", "kernel": f"k_stage2d<float,double,{dom},16,{segment(args.n)}>",
                     "achieved": alu_achieved, "peak": VALU_PEAK_GSLOTS,
                     "unit": "G lane-slots/s", "frac": alu_achieved / VALU_PEAK_GSLOTS,
                     "traffic": traffic, "avg_launch_ms": dom_ms,
                     "algorithmic_slots_per_cell": ALGO_SLOTS_PER_CELL},
        "hbm": {"kernel_GBps": hbm_gbs, "kernel_frac": hbm_gbs / HBM_PEAK_GBS,
                "sustained_GBps": sustained, "sustained_frac": sustained / HBM_PEAK_GBS,
                "peak_GBps": HBM_PEAK_GBS},
        "kernel_ms": ktimes,
    }
    if "fp64" in results:
        r = results["fp64"]
        line["fp64"] = {"value": r["cell_updates_per_s"], "ms_per_step": r["ms_per_solve"],
                        "rk_steps": r["rk_steps"],
                        "kernel_ms": r["kernels"]}
        line["fp32_speedup_over_fp64"] = main_res["cell_updates_per_s"] / r["cell_updates_per_s"]
    if not args.no_jp:
        # the paper's comparison scheme on the same workload (Jiang-Peng indicators)
        wall, info, times = time_solves(hjw, pr, hjw.FP32_MIXED, phi_dev, args.steps, args.warmup,
                                        args.tile_rows, scheme=hjw.WENO_JP)
        line["weno_jp"] = {"value": cells * 3 * info.steps * args.steps / wall,
                           "ms_per_step": 1e3 * wall / args.steps, "rk_steps": info.steps,
                           "kernel_ms": times,
                           "time_ratio_jp_over_l": (1e3 * wall / args.steps) / main_res["ms_per_solve"]}
    if not args.no_families:
        line["families"] = families(hjw, W, args.n)
    if not args.no_accuracy:
        line["fp32_error_vs_fp64"] = accuracy(hjw)
        line["beyond_infinity_cache"] = beyond_mall(hjw, W)
    if not args.no_serve:
        line["served"] = served_stream(args, hjw)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(pr, args.cpu_seconds)
    print(json.dumps(line))
    return 0


if __name__ == "__main__":
    sys.exit(main())
