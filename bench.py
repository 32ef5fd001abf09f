"""Benchmark: cell-updates/s per RK3 stage of the WENO-L solver on one MI355X.

One benchmark step is one whole solve of the 2-D Burgers problem of Example 3.3 scaled
to a 1024 x 1024 periodic grid on [-2,2)^2, phi0 = -cos(pi(x+y)/2), CFL 0.5, from t = 0
to t = 0.5/pi^2: every RK3 step (derivative ranges -> dissipation -> time step -> three
fused stages) runs on the GPU, from phi0 already resident in HBM.

value = cells x RK stages / wall time for the FP32-stencil path (FP64 phi, FP64 time step
and accumulation); the FP64 path is timed the same way and reported beside it.  The
roofline object describes the dominant kernel, timed with HIP events on the library's
stream right after the timed region, against the vector ALU peak (the bound of this path);
counter-derived traffic and instruction mixes ride along while the kernel sources match the
ones they were measured on.  cpu_baseline is the
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
# Vector ALU issue on gfx950, measured with a throughput probe (issue cycles of one wave64
# instruction on a SIMD): FP32 add/mul/FMA and 32-bit integer operations 2 cycles (32 lanes
# a cycle), FP64 operations and FP64 conversions 4 (16 lanes), FP32 transcendentals
# (reciprocal, square root, logarithm) 8.  One lane-slot is one FP32 lane-operation, so the
# FP32 peak is 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz = 78,643 G lane-slots/s (the published
# 157.3 TFLOP/s FP32 vector peak counts an FMA as two flops); the FP64 peak in FP64
# lane-operations is half of it (the published 78.6 TFLOP/s FP64 vector peak).
CYCLE_HZ = 2.4e9
SIMDS = 256 * 4
FP32_PEAK_GSLOTS = SIMDS * 32 * CYCLE_HZ / 1e9
FP64_PEAK_GOPS = SIMDS * 16 * CYCLE_HZ / 1e9
ISSUE_CYCLES = {"f32": 2, "i32": 2, "f64": 4, "cvt": 4, "i64": 4, "trans_f32": 8, "trans_f64": 16,
                "other": 2}
# Algorithmic work of one node-stage in 2-D (the operations of Section 2, Steps 2-5, per
# node, both axes): about 200 add/mul/FMA plus 28 square roots, logarithms, divisions and
# reciprocals (per axis 3 square roots and 3 logarithms for the arc-length antiderivatives,
# 6 quotients of the cell lengths, 2 weight reciprocals).  In the FP32 stencil a
# transcendental takes 4 lane-slots (quarter rate): 200 + 28 * 4 = 312 lane-slots.  The FP64
# path is priced the same way in FP64 lane-operations.
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


# rocprofv3 counters of the stage kernels (Burgers 2-D, bench.py --profile), per launch:
# traffic = FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (KiB; the factors are what the counters read
# for a plain 256 MiB copy kernel), and executed VALU instructions per node by class
# (SQ_INSTS_VALU_* x 64 / nodes).  Valid only while the kernel sources hash to the recorded
# SHA-256; after any change the counter-derived fields are null until re-measured.
MEASURED = {
    "source_sha256": "cfc9faa4c751c743d53d3b32d2b35723fe6daf266cad6743c697fcb608e3db64",
    "runs": {
        "fp32_stencil/1024": {
            "pre": {"fetch_kib": 4562.1, "write_kib": 12416.0, "traffic_bytes": 22057064,
                    "valu_per_node": {"f32": 178.0, "f64": 6.5, "i32": 21.71, "cvt": 4.75, "i64": 2.36, "trans_f32": 13.25, "trans_f64": 0.0, "other": 38.81}},
            "mid": {"fetch_kib": 11013.0, "write_kib": 8192.1, "traffic_bytes": 30943436,
                    "valu_per_node": {"f32": 182.0, "f64": 17.88, "i32": 16.88, "cvt": 10.25, "i64": 3.86, "trans_f32": 13.25, "trans_f64": 0.06, "other": 33.53}},
            "last": {"fetch_kib": 8636.0, "write_kib": 8194.2, "traffic_bytes": 26077440,
                    "valu_per_node": {"f32": 182.0, "f64": 9.5, "i32": 14.34, "cvt": 5.25, "i64": 2.39, "trans_f32": 13.25, "trans_f64": 0.0, "other": 30.55}},
        },
        "fp32_stencil/2048": {
            "pre": {"fetch_kib": 17072.0, "write_kib": 49664.0, "traffic_bytes": 85819359,
                    "valu_per_node": {"f32": 178.0, "f64": 6.5, "i32": 21.39, "cvt": 4.75, "i64": 2.06, "trans_f32": 13.25, "trans_f64": 0.0, "other": 38.38}},
            "mid": {"fetch_kib": 42201.0, "write_kib": 32768.0, "traffic_bytes": 119982123,
                    "valu_per_node": {"f32": 182.0, "f64": 16.0, "i32": 14.25, "cvt": 9.75, "i64": 2.91, "trans_f32": 13.25, "trans_f64": 0.0, "other": 28.02}},
            "last": {"fetch_kib": 33424.3, "write_kib": 32770.2, "traffic_bytes": 102009614,
                    "valu_per_node": {"f32": 182.0, "f64": 9.5, "i32": 13.92, "cvt": 5.25, "i64": 1.83, "trans_f32": 13.25, "trans_f64": 0.0, "other": 29.91}},
        },
        "fp32_stencil/4096": {
            "pre": {"fetch_kib": 66693.6, "write_kib": 198656.0, "traffic_bytes": 340012260,
                    "valu_per_node": {"f32": 178.0, "f64": 6.5, "i32": 21.23, "cvt": 4.75, "i64": 1.91, "trans_f32": 13.25, "trans_f64": 0.0, "other": 38.16}},
            "mid": {"fetch_kib": 166139.6, "write_kib": 131072.0, "traffic_bytes": 474471718,
                    "valu_per_node": {"f32": 182.0, "f64": 16.0, "i32": 14.25, "cvt": 9.75, "i64": 2.7, "trans_f32": 13.25, "trans_f64": 0.0, "other": 27.82}},
            "last": {"fetch_kib": 132151.2, "write_kib": 131074.2, "traffic_bytes": 404865673,
                    "valu_per_node": {"f32": 182.0, "f64": 9.5, "i32": 13.71, "cvt": 5.25, "i64": 1.54, "trans_f32": 13.25, "trans_f64": 0.0, "other": 29.58}},
        },
        "fp64/1024": {
            "pre": {"fetch_kib": 4881.3, "write_kib": 25720.9, "traffic_bytes": 36335066,
                    "valu_per_node": {"f32": 0.25, "f64": 280.0, "i32": 14.33, "cvt": 0.5, "i64": 2.48, "trans_f32": 0.25, "trans_f64": 10.75, "other": 108.94}},
            "mid": {"fetch_kib": 17782.7, "write_kib": 10188.0, "traffic_bytes": 46851518,
                    "valu_per_node": {"f32": 0.25, "f64": 295.5, "i32": 15.22, "cvt": 0.5, "i64": 3.67, "trans_f32": 0.25, "trans_f64": 10.81, "other": 71.4}},
            "last": {"fetch_kib": 8863.4, "write_kib": 9866.1, "traffic_bytes": 28255028,
                    "valu_per_node": {"f32": 0.25, "f64": 287.12, "i32": 13.96, "cvt": 0.5, "i64": 2.52, "trans_f32": 0.25, "trans_f64": 10.75, "other": 61.92}},
        },
        "fp64/2048": {
            "pre": {"fetch_kib": 17992.9, "write_kib": 102877.7, "traffic_bytes": 142196172,
                    "valu_per_node": {"f32": 0.25, "f64": 280.0, "i32": 14.02, "cvt": 0.5, "i64": 2.18, "trans_f32": 0.25, "trans_f64": 10.75, "other": 108.51}},
            "mid": {"fetch_kib": 68805.6, "write_kib": 40944.4, "traffic_bytes": 182840913,
                    "valu_per_node": {"f32": 0.25, "f64": 293.62, "i32": 13.99, "cvt": 0.5, "i64": 2.38, "trans_f32": 0.25, "trans_f64": 10.75, "other": 58.97}},
            "last": {"fetch_kib": 34431.2, "write_kib": 37658.6, "traffic_bytes": 109077438,
                    "valu_per_node": {"f32": 0.25, "f64": 287.12, "i32": 13.55, "cvt": 0.5, "i64": 1.95, "trans_f32": 0.25, "trans_f64": 10.75, "other": 61.28}},
        },
    },
}


def measured(prec, n):
    """The counter record of (precision, grid side) if the kernel sources are unchanged."""
    if not MEASURED or MEASURED["source_sha256"] != kernel_source_sha():
        return None
    return MEASURED["runs"].get(f"{prec}/{n}")


def counter_fields(rec, kernel, cells, launch_ms):
    """Counter-derived fields of one kernel: bytes per launch, executed instructions per
    node, and the VALU busy fraction (issue cycles at the measured rates over the launch)."""
    if not rec or kernel not in rec:
        return {"traffic": None}
    k = rec[kernel]
    issue = sum(k["valu_per_node"][c] * ISSUE_CYCLES[c] for c in ISSUE_CYCLES) * cells / 64
    busy = issue / SIMDS / CYCLE_HZ / (launch_ms * 1e-3)
    return {"traffic": k["traffic_bytes"],
            "traffic_GBps": k["traffic_bytes"] / (launch_ms * 1e-3) / 1e9,
            "executed_valu_per_cell": sum(k["valu_per_node"].values()),
            "executed_by_class": k["valu_per_node"], "valu_busy_frac": busy}


def alu_roofline(kernel, cells, launch_ms, prec, n):
    """The ALU roofline object of one stage kernel: the method's 312 lane-slots per node
    over the launch against the vector peak of its precision, with counter fields."""
    fp64 = prec == "fp64"
    peak = FP64_PEAK_GOPS if fp64 else FP32_PEAK_GSLOTS
    achieved = ALGO_SLOTS_PER_CELL * cells / (launch_ms * 1e-3) / 1e9
    obj = {"bound": "alu", "kernel": kernel, "achieved": achieved, "peak": peak,
           "unit": "G FP64 lane-ops/s" if fp64 else "G lane-slots/s", "frac": achieved / peak,
           "avg_launch_ms": launch_ms, "algorithmic_slots_per_cell": ALGO_SLOTS_PER_CELL}
    obj.update(counter_fields(measured(prec, n), kernel.split(",")[2], cells, launch_ms))
    return obj


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
    ap.add_argument("--serve-fixed-rate", type=float, default=190.0,
                    help="also replay the stream at this fixed arrival rate (requests/s; "
                         "0 skips): a load that does not move with the saturation rate")
    ap.add_argument("--serve-pool-gib", type=float, default=4.0)
    ap.add_argument("--serve-max-active", type=int, default=256)
    ap.add_argument("--serve-sustain-sample", type=int, default=768,
                    help="requests replayed closed-loop to measure the sustained throughput")
    ap.add_argument("--serve-outstanding", type=int, default=0,
                    help="requests kept in the server during the closed-loop replay "
                         "(0: --serve-max-active, the server kept full)")
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
    the 256 MB Infinity Cache: 4096^2 Burgers, FP32 stencil, whole solves to 0.1/pi^2, then
    each stage kernel timed back to back.  Its HBM figures come from the counters (traffic
    per launch) over the live launch time."""
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
    g.set_phi(phi_dev)
    times = g.time_kernels(reps=20)
    g.close()
    rate = pr.cells * 3 * info.steps / wall
    step_bytes = sum(kernel_bytes_per_cell(8, 4).values()) / 3.0   # per node-stage
    dom = max(("pre", "mid", "last"), key=lambda k: times[k])
    roof = alu_roofline(f"k_stage2d<float,double,{dom},16,8>", pr.cells, times[dom],
                        "fp32_stencil", 4096)
    rec = measured("fp32_stencil", 4096)
    hbm = None
    if rec:
        # traffic of a whole step from the counters over the three kernels' launch times
        tb = sum(rec[k]["traffic_bytes"] for k in ("pre", "mid", "last"))
        tt = sum(times[k] for k in ("pre", "plan", "mid", "last")) * 1e-3
        hbm = {"step_traffic_bytes": tb, "step_kernel_ms": tt * 1e3,
               "GBps": tb / tt / 1e9, "frac": tb / tt / 1e9 / HBM_PEAK_GBS,
               "dominant_kernel_GBps": roof["traffic_GBps"],
               "dominant_kernel_frac": roof["traffic_GBps"] / HBM_PEAK_GBS}
    return {"grid": "4096x4096 burgers2d, t=0.1/pi^2", "working_set_MB": pr.cells * 28 / 1e6,
            "rk_steps": info.steps, "ms_per_solve": wall * 1e3, "cell_updates_per_s": rate,
            "sustained_GBps": rate * step_bytes / 1e9,
            "sustained_frac": rate * step_bytes / 1e9 / HBM_PEAK_GBS,
            "kernel_ms": times, "roofline": roof, "hbm_from_counters": hbm}


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
    # the same server kept full (closed loop): the throughput it sustains without the drain
    sus_k = min(args.serve_sustain_sample, len(reqs))
    sus_out = min(args.serve_outstanding or args.serve_max_active, sus_k // 3)
    sus_rps, sus_cells, sus_wall, sus_n = S.sustained(srv, reqs[:sus_k], phi0s[:sus_k],
                                                      outstanding=sus_out,
                                                      warm=min(64, max(1, sus_out // 2)))
    rate = args.serve_load * sat_rps
    before = srv.stats()
    t1 = time.perf_counter()
    recs = S.run_stream(srv, reqs, phi0s, time_scale=1.0 / rate)
    wall = time.perf_counter() - t1
    after = srv.stats()
    summary = S.summarize(recs, wall)
    fixed = None
    if args.serve_fixed_rate > 0:
        t2 = time.perf_counter()
        recs2 = S.run_stream(srv, reqs, phi0s, time_scale=1.0 / args.serve_fixed_rate)
        s2 = S.summarize(recs2, time.perf_counter() - t2)
        fixed = {"arrival_rate_rps": args.serve_fixed_rate, "failed": s2["failed"],
                 "p50_ms": s2["p50_ms"], "p90_ms": s2["p90_ms"], "p99_ms": s2["p99_ms"],
                 "max_ms": s2["max_ms"],
                 "cell_updates_per_s": s2["cell_updates"] / s2["wall_s"]}
    srv.close()
    return {
        "requests": summary["requests"], "failed": summary["failed"],
        "precision": "f32 stencil, f64 phi/dt/accumulation",
        "arrival_rate_rps": rate, "load": args.serve_load,
        "saturation_rps": sat_rps, "saturation_cell_updates_per_s": sat_cells,
        "saturation_sample": f"last {k} requests of the stream submitted at once ({sat_wall:.1f} s)",
        "sustained_rps": sus_rps, "sustained_cell_updates_per_s": sus_cells,
        "sustained_sample": (f"first {sus_k} requests of the stream, {sus_out} kept in the "
                             f"server, {sus_n} timed after the first "
                             f"{min(64, max(1, sus_out // 2))} finished, drain excluded "
                             f"({sus_wall:.1f} s)"),
        "p50_ms": summary["p50_ms"], "p90_ms": summary["p90_ms"], "p99_ms": summary["p99_ms"],
        "max_ms": summary["max_ms"], "mean_ms": summary["mean_ms"],
        "cell_updates_per_s": summary["cell_updates"] / wall,
        "wall_s": wall, "batched_steps": after["batched_steps"] - before["batched_steps"],
        "pool_gib": args.serve_pool_gib, "pool_peak_gib": after["pool_peak"] / (1 << 30),
        "max_active": args.serve_max_active, "phi0_prep_s": prep,
        "latency_from": "scheduled arrival to result in host memory",
        "fixed_rate": fixed,
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
    fabric_gbs = bpc * cells / (dom_ms * 1e-3) / 1e9
    roofline = alu_roofline(f"k_stage2d<float,double,{dom},16,{segment(args.n)}>", cells, dom_ms,
                            "fp32_stencil", args.n) if args.tile_rows in (0, 16) else None
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
        "roofline": roofline,
        "hbm": {"kernel_GBps": fabric_gbs, "kernel_frac": fabric_gbs / HBM_PEAK_GBS,
                "sustained_GBps": sustained, "sustained_frac": sustained / HBM_PEAK_GBS,
                "peak_GBps": HBM_PEAK_GBS,
                "served_from": ("Infinity Cache: the %.0f MB working set fits its 256 MB, so these "
                                "rates are compulsory bytes over time, not HBM traffic"
                                % (cells * 28 / 1e6)) if cells * 28 < 256e6 else "HBM"},
        "kernel_ms": ktimes,
    }
    if "fp64" in results:
        r = results["fp64"]
        d64 = max(("pre", "mid", "last"), key=lambda k: r["kernels"][k])
        line["fp64"] = {"value": r["cell_updates_per_s"], "ms_per_step": r["ms_per_solve"],
                        "rk_steps": r["rk_steps"],
                        "kernel_ms": r["kernels"],
                        "roofline": alu_roofline(f"k_stage2d<double,double,{d64},16,8>", cells,
                                                 r["kernels"][d64], "fp64", args.n)
                        if args.tile_rows in (0, 16) else None}
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
