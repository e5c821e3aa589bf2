#!/usr/bin/env python3
"""HPM throughput on one MI355X: particles/s of one full solve (tree build + P2M + M2M + M2L +
L2L + L2P + P2P) in FP32, next to the FP64 GPU path at the same gridlet order, with the force
error against a direct sum, per-stage times, the M2L roofline and the CPU oracle's rate.

Workload: 2^18 particles from a Plummer sphere (scale radius 0.05, truncated at 0.5, centred),
equal masses, adaptive tree with at most 64 particles per leaf (depth <= 10), Plummer softening
1e-3, gridlet order N_g = 6 (the smallest supported order that reaches 1e-4 RMS force error on
this workload). Inputs are seeded and synthetic and resident in device memory before timing.

  python bench.py [--steps K] [--warmup W] [--ng 6] [--n 262144] [--no-cpu-baseline]

Prints ONE JSON line. Two other workloads run on their own flag, each printing its own line:

  --batch   512 independent FP32 solves (N log-uniform in [2^10, 2^18], half uniform cube and
            half Plummer, N_g 4 or 6, the shared-transform route unless --batch-m2l says
            otherwise) through one hpm_server_run_batch call on a warm server;
  --large   the 2^24-particle clustered set (N_g = 4, at most 32 per leaf) on each of the three
            source-to-target routes;
  --serve   a Poisson stream of solves (N log-uniform in [2^12, 2^20], uniform, Plummer or
            clustered, force tolerance 1e-4, N_g = 6 extended gridlets on the cell route) at
            0.5, 0.7 and 0.9 of the saturated rate:
            p50/p99 latency from submission to completion, particles/s, and every result checked
            against its tolerance and against the same solve alone.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector (published; counts packed two-wide FP32)
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
# the vector issue ceiling of code without packed FP32: 256 CUs x 4 SIMDs, one 64-lane
# instruction per SIMD every 4 cycles, 2.4 GHz
SIMDS, CLOCK_HZ, CYCLES_PER_VALU = 1024, 2.4e9, 4
PEAK_FP32_UNPACKED_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12  # 78.6


def m2l_flops_per_target(ng: int) -> float:
    """Algorithmic flops of one source-to-target FFT: forward and inverse real transforms of an
    n^3 grid (2.5 n^3 log2 n^3 each, the usual real-FFT count) plus the real spectral multiply
    (2 per half-spectrum point)."""
    n = 8 * ng
    n3 = float(n) ** 3
    half = n * n * (n // 2 + 1)
    return 2 * 2.5 * n3 * np.log2(n3) + 2.0 * half


def m2l_bytes_per_target(ng: int, elem: int) -> float:
    """Effective bytes of one source-to-target FFT, the usual FFT bandwidth convention: one read
    and one write of the n^2 (n/2+1) complex half-spectrum per transform pass, two passes each
    way (4 H complex values of 2 * elem bytes)."""
    n = 8 * ng
    half = n * n * (n // 2 + 1)
    return 4.0 * half * 2 * elem


def source_sha(path: str) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def counters_from_profile(name: str, source: str):
    """Per-launch counter figures of one kernel from a committed rocprofv3 counter summary
    (profiles/<name>.json), if they were taken on the current source file; else None."""
    path = os.path.join(ROOT, "profiles", f"{name}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, "paper_1906_10734_amd", "csrc", source)
    if rec.get("source_sha") != source_sha(src):
        return None
    return rec


def cpu_info() -> dict:
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None
    return {"os_cpu_count": os.cpu_count(), "affinity_cpus": aff, "model": model}


def run_path(hpm, torch, parts, prec: str, ng: int, steps: int, warmup: int, kernel="newton",
             screening=0.0, m2l="grid", extended=False, overlap=True, fp32_strict=False):
    """Times `steps` full solves (rebuild + execute); returns timing dict and outputs."""
    p = parts.astype(np.float32 if prec == "f32" else np.float64)
    dt = torch.float32 if prec == "f32" else torch.float64
    x, y, z, m = (torch.tensor(a, dtype=dt, device="cuda") for a in (p.x, p.y, p.z, p.m))
    prob = hpm.Problem(ng=ng, precision=prec, leaf_capacity=64, max_depth=10, softening=1e-3,
                       kernel=kernel, screening=screening, m2l=m2l, extended=extended)
    plan = hpm.Plan(prob, x, y, z)
    plan.set_overlap(overlap)
    if fp32_strict:
        plan.set_fp32_strict(True)
    out = [torch.empty(p.n, dtype=dt, device="cuda") for _ in range(4)]
    for _ in range(warmup):
        plan.rebuild(x, y, z)
        plan.execute(m, *out)
    torch.cuda.synchronize()
    plan.enable_timing(True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record()
        plan.rebuild(x, y, z)
        plan.execute(m, *out)
        ev[k][1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    st = plan.stage_times()
    info = plan.info()
    res = dict(ms_per_step=(t1 - t0) * 1e3 / steps, lat_p50=float(np.percentile(lat, 50)),
               lat_p99=float(np.percentile(lat, 99)), stages=st, info=info)
    plan.close()
    return res, out, (x, y, z, m)


_ORACLE = {}  # the oracle's evaluation object, shared with forked workers (copy on write)


def _oracle_sample(args):
    """Times the oracle's per-target (source-to-target + parent-to-child) or per-leaf (near zone
    + interpolation) work on a random sample until the deadline; returns (items, seconds)."""
    kind, seed, budget = args
    from threadpoolctl import threadpool_limits
    from oracle import hpm as ohpm
    h, targets, leaves, ng = (_ORACLE[k] for k in ("h", "targets", "leaves", "ng"))
    t = h.tree
    rng = np.random.default_rng(seed)
    n_done, spent = 0, 0.0
    deadline = time.perf_counter() + budget
    with threadpool_limits(1):
        if kind == "m2l":
            for k in rng.permutation(len(targets)):
                l, i = targets[k]
                a = time.perf_counter()
                phi = h.m2l(l, t.levels[l].coords[i])
                if l > 2:
                    ohpm.l2l(phi, int(t.levels[l].keys[i] & 7), ng)
                spent += time.perf_counter() - a
                n_done += 1
                if time.perf_counter() > deadline and n_done >= 4:
                    break
        else:
            for k in rng.permutation(len(leaves)):
                l, i = leaves[k]
                lev = t.levels[l]
                if l >= 2:
                    h.local(l, i)  # chain of locals (its targets' work is counted by "m2l")
                a = time.perf_counter()
                h.leaf_fields(l, i, np.arange(lev.pb[i], lev.pe[i]))
                spent += time.perf_counter() - a
                n_done += 1
                if time.perf_counter() > deadline and n_done >= 4:
                    break
    return n_done, spent


def cpu_baseline(parts, ng: int, budget_s: float, workers: int):
    """The FP64 oracle (test infrastructure, as it stands) on a bounded sample of the same
    workload: tree + full up-sweep timed whole on one thread (the oracle's up-sweep is a serial
    loop); source-to-target + parent-to-child on random samples of targets and near zone +
    interpolation on random samples of leaves, run by `workers` forked processes side by side
    (one thread each), their combined rate taken from the wall clock; scaled to the full solve.
    Call it before the process touches the GPU (the workers are forked)."""
    import multiprocessing as mp
    from threadpoolctl import threadpool_limits
    from oracle import hpm as ohpm
    p = parts.as_f64()
    with threadpool_limits(1):
        prob = ohpm.Problem(ng=ng, softening=1e-3, leaf_capacity=64, max_depth=10)
        t0 = time.perf_counter()
        h = ohpm.HPM(p.x, p.y, p.z, p.m, prob, mode="fft")
        t_up = time.perf_counter() - t0
    t = h.tree
    _ORACLE.update(h=h, ng=ng, leaves=list(t.leaves()),
                   targets=[(l, i) for l in range(2, t.max_level + 1) for i in range(len(t.levels[l]))])
    rates = {}
    for kind in ("m2l", "leaf"):
        jobs = [(kind, 7 + 101 * w, budget_s / 2) for w in range(workers)]
        t0 = time.perf_counter()
        if workers == 1:
            res = [_oracle_sample(jobs[0])]
        else:
            with mp.get_context("fork").Pool(workers) as pool:
                res = pool.map(_oracle_sample, jobs)
        wall = time.perf_counter() - t0
        rates[kind] = (sum(r[0] for r in res), wall)
    n_t, n_l = len(_ORACLE["targets"]), len(_ORACLE["leaves"])
    est = t_up + n_t * rates["m2l"][1] / rates["m2l"][0] + n_l * rates["leaf"][1] / rates["leaf"][0]
    _ORACLE.clear()
    return {"value": round(p.n / est, 2), "unit": "particles/s", "cores": workers, "kind": "oracle",
            "sample": (f"tree+P2M+M2M over all {p.n} particles on one thread ({t_up:.1f} s); "
                       f"M2L+L2L on {rates['m2l'][0]} of {n_t} targets and L2P+P2P on "
                       f"{rates['leaf'][0]} of {n_l} leaves by {workers} process(es) in "
                       f"{rates['m2l'][1]:.1f} + {rates['leaf'][1]:.1f} s of wall clock; scaled "
                       f"to the full solve ({est:.1f} s est.)")}


def run_info_targets(hpm, torch, parts, ng):
    """Number of source-to-target targets of a set's tree (one FP32 plan build)."""
    p = parts.astype(np.float32)
    x, y, z, _ = _device_set(torch, p, torch.float32)
    plan = hpm.Plan(hpm.Problem(ng=ng, precision="f32", leaf_capacity=64, max_depth=10,
                                softening=1e-3), x, y, z)
    n_t = plan.info()["n_targets"]
    plan.close()
    return n_t


def _device_set(torch, p, dt):
    return tuple(torch.tensor(a, dtype=dt, device="cuda") for a in (p.x, p.y, p.z, p.m))


def _force_err(torch, out, sub, ref):
    a = torch.stack([o[sub].double() for o in out[1:]], 1)
    e = (a - ref).norm(dim=1) / ref.norm(dim=1)
    return float(e.pow(2).mean().sqrt())


def batch_bench(args):
    """512 independent FP32 solves in one hpm_server_run_batch call (the largest first, `slots`
    in flight at once), on a server whose plans are already resident (one warm-up batch)."""
    import torch
    from paper_1906_10734_amd import hpm
    from synth import batch_requests, random_subset, request_particles
    reqs = batch_requests(args.batch_count)
    probs, sets = [], []
    for r in reqs:
        p = request_particles(r).astype(np.float32)
        sets.append(_device_set(torch, p, torch.float32))
        probs.append(hpm.Problem(ng=r["ng"], precision="f32", leaf_capacity=64, max_depth=10,
                                 softening=1e-3, m2l=args.batch_m2l))
    torch.cuda.synchronize()
    total = sum(r["n"] for r in reqs)
    print(f"[batch] {len(reqs)} solves, {total} particles on the device", file=sys.stderr,
          flush=True)
    times = []
    with hpm.Server(slots=args.slots) as sv:
        st, outs = sv.run_batch(probs, sets)  # warm-up: plans created and grown
        assert all(v == "HPM_OK" for v in st), st
        for k in range(args.steps):
            t0 = time.perf_counter()
            st, outs = sv.run_batch(probs, sets, outs)
            times.append(time.perf_counter() - t0)
            assert all(v == "HPM_OK" for v in st), st
            print(f"[batch] step {k}: {times[-1] * 1e3:.1f} ms", file=sys.stderr, flush=True)
        stats = sv.stats()
    # every 16th solve: its result alone (bit for bit) and its force error on 64 particles
    same, errs = 0, {4: [], 6: []}
    checked = list(range(0, len(reqs), 16))
    for i in checked:
        solo = hpm.solve(probs[i], *sets[i])
        same += int(all(torch.equal(a, b) for a, b in zip(solo, outs[i])))
        x, y, z, m = sets[i]
        sub = torch.tensor(random_subset(reqs[i]["n"], 64, 5000 + i), device="cuda")
        _, rx, ry, rz = hpm.direct_sum(x, y, z, m, sub, 1.0, 1e-3)
        errs[reqs[i]["ng"]].append(_force_err(torch, outs[i], sub, torch.stack([rx, ry, rz], 1)))
    ms = float(np.median(times)) * 1e3
    rec = {"mode": "batch", "metric": "particles/s of a batch of independent solves",
           "value": round(total / (ms * 1e-3), 1), "unit": "particles/s",
           "solves_per_s": round(len(reqs) / (ms * 1e-3), 1), "ms_per_batch": round(ms, 3),
           "ms_per_batch_all": [round(t * 1e3, 3) for t in times], "steps": args.steps,
           "dtype": "f32", "data": "synthetic (seeded uniform cubes and Plummer spheres)",
           "config": {"workload": f"{len(reqs)} solves, N log-uniform 2^10..2^18, half uniform "
                                  "half Plummer, N_g 4 or 6, leaf<=64, eps=1e-3",
                      "m2l": args.batch_m2l,
                      "solves": len(reqs), "particles": total, "slots": args.slots,
                      "ng4_solves": sum(r["ng"] == 4 for r in reqs)},
           "checked": {"solves": len(checked), "identical_to_alone": same,
                       "force_err_rms_median": {f"ng{g}": (float(np.median(v)) if v else None)
                                                for g, v in errs.items()}},
           "server": stats}
    return rec


def serve_bench(args):
    """A Poisson stream of requests drawn from a pool of seeded particle sets, on a server with
    `slots` workers and a memory budget; latency from submission to completion."""
    import torch
    from paper_1906_10734_amd import hpm
    from synth import random_subset, request_particles, serve_requests
    pool = serve_requests(args.serve_pool)
    sets, probs, refs, solos, subs = [], [], [], [], []
    for i, r in enumerate(pool):
        p = request_particles(r).astype(np.float32)
        dev = _device_set(torch, p, torch.float32)
        # the form for the request's 1e-4 tolerance: the extended N_g = 6 gridlet on the cell
        # route (1.7e-5 on the 2^18 Plummer workload, 6x below the tolerance). The standard
        # N_g = 6 gridlet (8e-5) leaves no margin, no N_g = 4 form reaches 1e-4 (2.7e-4 extended),
        # and FP32 at N_g = 8 stops at 1.5e-4 (its rounding, not the method: FP64 gives 4.6e-6)
        ng = 6
        prob = hpm.Problem(ng=6, precision="f32", leaf_capacity=64, max_depth=10,
                           softening=1e-3, m2l="cells", extended=True)
        sub = torch.tensor(random_subset(r["n"], 256, 6000 + i), device="cuda")
        _, rx, ry, rz = hpm.direct_sum(*dev, sub, 1.0, 1e-3)
        solo = hpm.solve(prob, *dev)
        sets.append(dev)
        probs.append(prob)
        subs.append(sub)
        refs.append(torch.stack([rx, ry, rz], 1))
        solos.append([o[sub].clone() for o in solo])
        r["ng"] = ng
        r["force_err_rms"] = _force_err(torch, solo, sub, refs[-1])
    torch.cuda.synchronize()
    print(f"[serve] pool of {len(pool)} request sets ready", file=sys.stderr, flush=True)
    rng = np.random.Generator(np.random.PCG64(1004))

    def run(stream_of, gaps):
        """Submits pool entries `stream_of` at cumulative times `gaps` (s); returns results."""
        tick, t0 = [], time.perf_counter()
        due = np.cumsum(gaps)
        for k, i in enumerate(stream_of):
            while True:
                left = due[k] - (time.perf_counter() - t0)
                if left <= 0:
                    break
                time.sleep(left if left > 2e-3 else 0)
            tick.append(sv.submit(probs[i], *sets[i], sync=False))
        return [sv.wait(t) for t in tick]

    def check(stream_of, res):
        bad_tol, not_same = 0, 0
        for i, (info, out) in zip(stream_of, res):
            assert info["status"] == "HPM_OK", info
            e = _force_err(torch, out, subs[i], refs[i])
            bad_tol += int(e > pool[i]["tolerance"])
            not_same += int(not all(torch.equal(o[subs[i]], s) for o, s in zip(out, solos[i])))
        return bad_tol, not_same

    out = {}
    with hpm.Server(slots=args.slots, hbm_budget=args.serve_budget_gib << 30) as sv:
        # warm-up, then the saturated rate: everything submitted at once
        warm = rng.integers(0, len(pool), 2 * len(pool))
        run(warm, np.zeros(len(warm)))
        sat = rng.integers(0, len(pool), args.serve_requests // 2)
        t0 = time.perf_counter()
        res = run(sat, np.zeros(len(sat)))
        t_sat = time.perf_counter() - t0
        rate_sat = len(sat) / t_sat
        print(f"[serve] saturated: {rate_sat:.1f} solves/s", file=sys.stderr, flush=True)
        out["saturated"] = {"solves_per_s": round(rate_sat, 1),
                            "particles_per_s": round(sum(pool[i]["n"] for i in sat) / t_sat, 1)}
        for frac in (0.5, 0.7, 0.9):
            lam = frac * rate_sat
            picks = rng.integers(0, len(pool), args.serve_requests)
            gaps = rng.exponential(1.0 / lam, args.serve_requests)
            t0 = time.perf_counter()
            res = run(picks, gaps)
            wall = time.perf_counter() - t0
            lat = np.array([i["latency_ms"] for i, _ in res])
            bad_tol, not_same = check(picks, res)
            out[f"load_{frac}"] = {
                "arrival_rate_per_s": round(lam, 1), "requests": len(picks),
                "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                               "p99": round(float(np.percentile(lat, 99)), 3)},
                "particles_per_s": round(sum(pool[i]["n"] for i in picks) / wall, 1),
                "over_tolerance": bad_tol, "differs_from_alone": not_same}
            print(f"[serve] load {frac}: p50 {np.percentile(lat, 50):.2f} ms, "
                  f"p99 {np.percentile(lat, 99):.2f} ms", file=sys.stderr, flush=True)
            del res
        stats = sv.stats()
    rec = {"mode": "serve", "metric": "solve p50/p99 latency under a Poisson request stream",
           "unit": "ms", "dtype": "f32", "data": "synthetic (seeded uniform, Plummer, clustered)",
           "config": {"workload": "Poisson arrivals, N log-uniform 2^12..2^20, uniform/Plummer/"
                                  "clustered, relative force tolerance 1e-4 for every request, "
                                  "N_g = 6 extended gridlets on the cell route, leaf<=64, "
                                  "eps=1e-3", "pool": len(pool), "slots": args.slots,
                      "hbm_budget_gib": args.serve_budget_gib},
           "results": out, "server": stats,
           "pool_over_tolerance": [{k: r[k] for k in ("kind", "n", "ng", "tolerance",
                                                      "force_err_rms")}
                                   for r in pool if r["force_err_rms"] > r["tolerance"]]}
    return rec


def large_bench(args):
    """The large clustered case: 2^24 particles (32 Plummer spheres on a 10% uniform background),
    at most 32 per leaf, N_g = 4, FP32, on each source-to-target route: rebuild + evaluate timed
    over `steps` solves after one untimed solve, force error on 1024 sampled particles against the
    FP64 direct sum over all particles."""
    import torch
    from paper_1906_10734_amd import hpm
    from synth import random_subset, workload
    n = 2 ** 24
    p = workload("clustered2p24_cap32").astype(np.float32)
    x, y, z, m = _device_set(torch, p, torch.float32)
    sub = torch.tensor(random_subset(n, 1024, 4004), device="cuda")
    _, rx, ry, rz = hpm.direct_sum(x.double(), y.double(), z.double(), m.double(), sub, 1.0, 1e-3)
    ref = torch.stack([rx, ry, rz], 1)
    routes = {}
    for route in getattr(args, "large_routes", "grid,shared,cells").split(","):
        plan = hpm.Plan(hpm.Problem(ng=4, precision="f32", leaf_capacity=32, max_depth=10,
                                    softening=1e-3, m2l=route), x, y, z)
        out = [torch.empty_like(m) for _ in range(4)]
        plan.execute(m, *out)
        torch.cuda.synchronize()
        plan.enable_timing(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.rebuild(x, y, z)
            plan.execute(m, *out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        st = plan.stage_times()
        info = plan.info()
        routes[route] = {"ms_per_step": round(dt * 1e3, 3), "particles_per_s": round(n / dt, 1),
                         "force_err_rms": _force_err(torch, out, sub, ref),
                         "m2l_ms": round(st["m2l"] / max(st["n_exec"], 1), 3),
                         "tree_ms": round(st["tree"] / max(st["n_build"], 1), 3)}
        print(f"[large] {route}: {routes[route]['ms_per_step']} ms", file=sys.stderr, flush=True)
        plan.close()
    return {"mode": "large", "metric": "particles/s of one solve", "unit": "particles/s",
            "dtype": "f32", "data": "synthetic (seeded clustered set)", "steps": args.steps,
            "config": {"workload": "2^24 particles, 32 Plummer spheres on a 10% uniform background, "
                                   "leaf<=32, depth<=10, N_g=4, eps=1e-3",
                       "levels": info["n_levels"], "targets": info["n_targets"]},
            "routes": routes}


def _fastest_route(routes):
    """The route with the highest FP32 whole-solve rate on the headline workload (the padded
    grid per target is `value`)."""
    best = None
    for name in ("cells", "shared"):
        r = routes.get(f"{name}_f32")
        if r and (best is None or r["value"] > best["value"]):
            best = {"route": name, "value": r["value"], "ms_per_step": r["ms_per_step"],
                    "force_err_rms": r["force_err_rms"],
                    "fp64_value": routes.get(f"{name}_f64", {}).get("value")}
    return best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--ng", type=int, default=6)
    ap.add_argument("--n", type=int, default=2 ** 18)
    ap.add_argument("--fp64-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="most host processes of the all-core CPU baseline")
    ap.add_argument("--sweep-steps", type=int, default=3,
                    help="timed solves per point of the gridlet-order accuracy sweep")
    ap.add_argument("--profile", action="store_true",
                    help="FP32 steps only, then a device copy of 256 MiB (counter calibration)")
    ap.add_argument("--m2l", choices=("grid", "cells", "shared"), default="grid",
                    help="source-to-target route of the --profile run")
    ap.add_argument("--in-line", action="store_true",
                    help="--profile: near-zone sums in line after the source-to-target step")
    ap.add_argument("--precision", choices=("f32", "f64"), default="f32",
                    help="precision of the --profile run")
    ap.add_argument("--batch", action="store_true", help="the batched workload instead")
    ap.add_argument("--large", action="store_true",
                    help="the 2^24-particle clustered workload on each route instead")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--batch-m2l", choices=("grid", "cells", "shared"), default="shared",
                    help="source-to-target route of the batched solves")
    ap.add_argument("--serve", action="store_true", help="the served workload instead")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-pool", type=int, default=64)
    ap.add_argument("--serve-budget-gib", type=int, default=64)
    ap.add_argument("--slots", type=int, default=8, help="server slots of --batch and --serve")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.batch:
        print(json.dumps(batch_bench(args)))
        return
    if args.large:
        print(json.dumps(large_bench(args)))
        return
    if args.serve:
        print(json.dumps(serve_bench(args)))
        return

    from synth import plummer_sphere, random_subset

    parts = plummer_sphere(args.n, 1001)
    ng = args.ng
    # the CPU oracle first, before this process touches the GPU (its workers are forked)
    cpu = None
    if not args.no_cpu_baseline and not args.profile:
        host = cpu_info()
        share = min(host["affinity_cpus"] or host["os_cpu_count"] or 1, args.cpu_workers)
        cpu = {"all_cores": cpu_baseline(parts, ng, args.cpu_seconds, share),
               "one_core": cpu_baseline(parts, ng, args.cpu_seconds, 1), "host": host}
        print(f"[cpu] {cpu['all_cores']['value']} particles/s on {share} cores, "
              f"{cpu['one_core']['value']} on one", file=sys.stderr, flush=True)

    import torch
    from paper_1906_10734_amd import hpm
    if args.profile:
        r32, _, _ = run_path(hpm, torch, parts, args.precision, ng, args.steps, args.warmup,
                             m2l=args.m2l, overlap=not args.in_line)
        src = torch.empty(64 * 2 ** 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"profile_run": True, "m2l": args.m2l, "precision": args.precision,
                          "ms_per_step": r32["ms_per_step"], "stages": r32["stages"],
                          "copy_bytes": 2 * src.numel() * 4}))
        return
    r32, out32, dev32 = run_path(hpm, torch, parts, "f32", ng, args.steps, args.warmup)
    r64, out64, dev64 = run_path(hpm, torch, parts, "f64", ng, args.fp64_steps, 1)

    # accuracy: FP64 direct sum on a 4096-particle subset of the FP64 positions
    sub = torch.tensor(random_subset(args.n, 4096, 2002), device="cuda")
    x64, y64, z64, m64 = dev64
    rphi, rax, ray, raz = hpm.direct_sum(x64, y64, z64, m64, sub, 1.0, 1e-3)
    ref = torch.stack([rax, ray, raz], 1)

    def ferr(out):
        a = torch.stack([o[sub].double() for o in out[1:]], 1)
        e = (a - ref).norm(dim=1) / ref.norm(dim=1)
        return float(e.pow(2).mean().sqrt()), float(e.max())

    f32_rms, f32_max = ferr(out32)

    # the same FP32 solve with no FP64 arithmetic in the source-to-target step and L2L
    # (float-float inverse x sums, means and constants)
    r32s, out32s, _ = run_path(hpm, torch, parts, "f32", ng, args.steps, 1, fp32_strict=True)
    s_rms, s_max = ferr(out32s)
    fp32_strict = {"value": round(args.n / (r32s["ms_per_step"] * 1e-3), 1),
                   "ms_per_step": round(r32s["ms_per_step"], 4),
                   "m2l_ms": round(r32s["stages"]["m2l"] / max(r32s["stages"]["n_exec"], 1), 4),
                   "force_err_rms": s_rms, "force_err_max": s_max,
                   "phi_max_rel_diff_to_default": float(
                       ((out32s[0] - out32[0]).abs() / out32[0].abs().clamp_min(1e-30)).max()),
                   "note": "FP32 path with the source-to-target step's inverse x sums and means and "
                           "L2L's constants in float-float instead of FP64"}

    # the screened kernel (kernel independence, Sec. 4) on the same workload, FP32, with its
    # own direct-sum reference
    lam = 0.05
    ry, outy, devy = run_path(hpm, torch, parts, "f32", ng, args.steps, 1, "yukawa", lam)
    _, yax, yay, yaz = hpm.direct_sum(x64, y64, z64, m64, sub, 1.0, 1e-3, kernel="yukawa",
                                      screening=lam)
    yref = torch.stack([yax, yay, yaz], 1)
    ya = torch.stack([o[sub].double() for o in outy[1:]], 1)
    ye = (ya - yref).norm(dim=1) / yref.norm(dim=1)
    ry64, outy64, _ = run_path(hpm, torch, parts, "f64", ng, args.fp64_steps, 1, "yukawa", lam)
    ye64 = (torch.stack([o[sub] for o in outy64[1:]], 1) - yref).norm(dim=1) / yref.norm(dim=1)
    yukawa = {"screening": lam, "value": round(args.n / (ry["ms_per_step"] * 1e-3), 1),
              "unit": "particles/s", "ms_per_step": round(ry["ms_per_step"], 4),
              "force_err_rms": float(ye.pow(2).mean().sqrt()), "force_err_max": float(ye.max()),
              "fp64": {"value": round(args.n / (ry64["ms_per_step"] * 1e-3), 1),
                       "ms_per_step": round(ry64["ms_per_step"], 4),
                       "force_err_rms": float(ye64.pow(2).mean().sqrt())}}
    f64_rms, f64_max = ferr(out64)
    phi_f32_vs_f64 = float(((out32[0].double() - out64[0]).norm() / out64[0].norm()))

    n_t = r32["info"]["n_targets"]
    # the M2L stage of the grid route is one launch of the z-slab kernel, bracketed by HIP events on
    # the stream it is launched on (the near-zone sums run beside it on the plan's second stream)
    m2l_ms = r32["stages"]["m2l"] / max(r32["stages"]["n_exec"], 1)
    flops = m2l_flops_per_target(ng) * n_t
    nbytes = m2l_bytes_per_target(ng, 4) * n_t
    gbs = nbytes / (m2l_ms * 1e-3) / 1e9
    tflops = flops / (m2l_ms * 1e-3) / 1e12
    kernel = f"k_m2l_slab<float, {ng}, 0, false>" if ng >= 4 else f"k_m2l<float, {ng}>"
    ctr = counters_from_profile(f"m2l_ng{ng}_f32_plummer2p18_counters", "m2l.hip")
    valu = None
    if ctr and ctr.get("valu_insts_per_launch"):
        issue_s = ctr["valu_insts_per_launch"] * CYCLES_PER_VALU / (SIMDS * CLOCK_HZ)
        valu = {"insts_per_launch": ctr["valu_insts_per_launch"],
                "issue_frac": round(issue_s / (m2l_ms * 1e-3), 4),
                "source": f"profiles/m2l_ng{ng}_f32_plummer2p18_counters.md"}
    # The FP32 source-to-target kernel keeps its whole transform on chip (LDS and registers); its
    # HBM traffic is the source gridlets and the outputs, so the bound is the vector ALU. The
    # algorithmic work is the FFT-convention count of one zero-padded transform per target; the
    # kernel prunes zero lines and does z in real space, so that count is nominal and the
    # executed-instruction share of the vector issue ceiling (valu.issue_frac) is the utilisation.
    roofline = {"bound": "alu", "achieved": round(tflops, 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(tflops / PEAK_FP32_TFLOPS, 4),
                "traffic": ctr.get("bytes_per_launch") if ctr else None, "kernel": kernel,
                "launch_ms": round(m2l_ms, 4), "launches": r32["stages"]["n_exec"],
                "targets_per_launch": n_t, "flops_per_target": m2l_flops_per_target(ng),
                "peak_unpacked_fp32": round(PEAK_FP32_UNPACKED_TFLOPS, 1),
                "frac_unpacked": round(tflops / PEAK_FP32_UNPACKED_TFLOPS, 4), "valu": valu,
                "effective_hbm": {"achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                  "frac": round(gbs / PEAK_HBM_GBS, 4),
                                  "bytes_per_target": m2l_bytes_per_target(ng, 4)}}

    # the near-zone sums (P2P, on the plan's second stream beside M2L): pairs per second and the
    # 20-flop-per-pair N-body convention against the FP32 peaks
    pairs = r32["info"]["p2p_pairs"]
    p2p_ms = r32["stages"]["p2p"] / max(r32["stages"]["n_exec"], 1)
    p2p_tf = pairs * 20.0 / (p2p_ms * 1e-3) / 1e12
    pctr = counters_from_profile("p2p_f32_plummer2p18_counters", "downsweep.hip")
    near_zone = {"kernel": "k_p2p<float, 0>", "pairs": pairs, "launch_ms": round(p2p_ms, 4),
                 "pairs_per_s": round(pairs / (p2p_ms * 1e-3), 1),
                 "achieved_tflops_20_per_pair": round(p2p_tf, 3),
                 "frac": round(p2p_tf / PEAK_FP32_TFLOPS, 4),
                 "frac_unpacked": round(p2p_tf / PEAK_FP32_UNPACKED_TFLOPS, 4),
                 "note": "timed on its own stream while the source-to-target kernel runs beside it"}
    if pctr and pctr.get("valu_insts_per_launch"):
        near_zone["valu"] = {"insts_per_launch": pctr["valu_insts_per_launch"],
                             "alone_ms": pctr.get("alone_ms"),
                             "issue_frac_alone": pctr.get("issue_frac_alone"),
                             "source": "profiles/p2p_f32_plummer2p18_counters.md"}

    value = args.n / (r32["ms_per_step"] * 1e-3)
    v64 = args.n / (r64["ms_per_step"] * 1e-3)
    # the same workload at the other gridlet order the configuration names (N_g = 4): rates and
    # force errors of both paths (the method's own error at N_g = 4 is far above 1e-4)
    ng4 = {}
    if ng != 4:
        r4, o4, _ = run_path(hpm, torch, parts, "f32", 4, args.steps, 1)
        r4d, o4d, _ = run_path(hpm, torch, parts, "f64", 4, args.fp64_steps, 1)
        e4, e4d = ferr(o4), ferr(o4d)
        ng4 = {"ng": 4, "value": round(args.n / (r4["ms_per_step"] * 1e-3), 1),
               "ms_per_step": round(r4["ms_per_step"], 4), "force_err_rms": e4[0],
               "fp64": {"value": round(args.n / (r4d["ms_per_step"] * 1e-3), 1),
                        "ms_per_step": round(r4d["ms_per_step"], 4), "force_err_rms": e4d[0]}}

    # N_g = 8 (the other order the configuration names), on the 2^16-particle Plummer sphere (the
    # library limits N_g = 8 to 2^16 particles), beside N_g = 6 on the same set; force errors
    # against the FP64 direct sum on 4096 sampled particles
    n8 = 2 ** 16
    parts8 = plummer_sphere(n8, 1001)
    sub8 = torch.tensor(random_subset(n8, 4096, 2002), device="cuda")
    p8 = parts8.as_f64()
    d8 = _device_set(torch, p8, torch.float64)
    _, r8x, r8y, r8z = hpm.direct_sum(*d8, sub8, 1.0, 1e-3)
    ref8 = torch.stack([r8x, r8y, r8z], 1)
    ng8 = {"workload": f"plummer sphere N={n8} a=0.05 r_t=0.5, leaf<=64, depth<=10, eps=1e-3"}
    for g in (8, 6):
        for pr, st in (("f32", args.steps), ("f64", args.fp64_steps)):
            r8, o8, _ = run_path(hpm, torch, parts8, pr, g, st, 1)
            ng8[f"ng{g}_{pr}"] = {"value": round(n8 / (r8["ms_per_step"] * 1e-3), 1),
                                  "ms_per_step": round(r8["ms_per_step"], 4),
                                  "m2l_ms": round(r8["stages"]["m2l"] / max(r8["stages"]["n_exec"], 1), 4),
                                  "force_err_rms": _force_err(torch, o8, sub8, ref8)}
    ng8["m2l_kernel_tflops_fft_convention_f32"] = round(
        m2l_flops_per_target(8) * run_info_targets(hpm, torch, parts8, 8)
        / (ng8["ng8_f32"]["m2l_ms"] * 1e-3) / 1e12, 3)

    # the cell-by-cell source-to-target route (Sec. 2.5) on the same workload: whole-solve rate,
    # its source-to-target stage time beside the padded grid's, and the force error
    def stage(r, k):
        return r["stages"][k] / max(r["stages"]["n_exec"], 1)
    rc, oc, _ = run_path(hpm, torch, parts, "f32", ng, args.steps, 1, m2l="cells")
    rcd, ocd, _ = run_path(hpm, torch, parts, "f64", ng, args.fp64_steps, 1, m2l="cells")
    rs_, os__, _ = run_path(hpm, torch, parts, "f32", ng, args.steps, 1, m2l="shared")
    rsd, osd, _ = run_path(hpm, torch, parts, "f64", ng, args.fp64_steps, 1, m2l="shared")
    pg = float(np.log2(ng))
    routes = {"cells_f32": {"value": round(args.n / (rc["ms_per_step"] * 1e-3), 1),
                            "ms_per_step": round(rc["ms_per_step"], 4),
                            "m2l_ms": round(stage(rc, "m2l"), 4), "force_err_rms": ferr(oc)[0]},
              "cells_f64": {"value": round(args.n / (rcd["ms_per_step"] * 1e-3), 1),
                            "ms_per_step": round(rcd["ms_per_step"], 4),
                            "m2l_ms": round(stage(rcd, "m2l"), 4), "force_err_rms": ferr(ocd)[0]},
              "shared_f32": {"value": round(args.n / (rs_["ms_per_step"] * 1e-3), 1),
                             "ms_per_step": round(rs_["ms_per_step"], 4),
                             "m2l_ms": round(stage(rs_, "m2l"), 4), "force_err_rms": ferr(os__)[0]},
              "shared_f64": {"value": round(args.n / (rsd["ms_per_step"] * 1e-3), 1),
                             "ms_per_step": round(rsd["ms_per_step"], 4),
                             "m2l_ms": round(stage(rsd, "m2l"), 4), "force_err_rms": ferr(osd)[0]},
              "grid_m2l_ms": {"f32": round(stage(r32, "m2l"), 4), "f64": round(stage(r64, "m2l"), 4)},
              "paper_count_ratio_grid_over_cells": round(0.34 * (pg + 3) / (pg + 1), 3)}
    # the route autotuner on the same tree (one plan built with the cell spectra, every route
    # timed on it, the fastest kept)
    for pr in ("f32", "f64"):
        q = parts.astype(np.float32 if pr == "f32" else np.float64)
        dq = torch.float32 if pr == "f32" else torch.float64
        xq, yq, zq, mq = _device_set(torch, q, dq)
        tplan = hpm.Plan(hpm.Problem(ng=ng, precision=pr, leaf_capacity=64, max_depth=10,
                                     softening=1e-3, m2l="shared"), xq, yq, zq)
        best, per = tplan.autotune(mq, reps=3)
        routes[f"autotuned_{pr}"] = {"route": best,
                                     "ms_per_evaluation": {k: round(v, 4) for k, v in per.items()}}
        tplan.close()
    # the extended target gridlet (Sec. 2.5, N_g + 2 nodes per axis) on the cell route, at this
    # order and at N_g = 4: rate and force error beside the standard gridlet's
    for g in sorted({ng, 4}):
        for route in ("cells", "grid"):
            for pr, st in (("f32", args.steps), ("f64", args.fp64_steps)):
                re_, oe, _ = run_path(hpm, torch, parts, pr, g, st, 1, m2l=route, extended=True)
                routes[f"{route}_extended_ng{g}_{pr}"] = {
                    "value": round(args.n / (re_["ms_per_step"] * 1e-3), 1),
                    "ms_per_step": round(re_["ms_per_step"], 4),
                    "m2l_ms": round(stage(re_, "m2l"), 4),
                    "leaf_ms": round(stage(re_, "leaf"), 4), "force_err_rms": ferr(oe)[0]}

    # accuracy sweep over the gridlet order (the paper's accuracy-versus-cost comparison, Sec. 3.2):
    # force error against the direct sum and time per solve, both precisions on the padded grid,
    # and the extended gridlet on the cell route (FP32)
    sweep = {}
    for g in (2, 3, 4, 6):
        point = {}
        for pr in ("f32", "f64"):
            rs, os_, _ = run_path(hpm, torch, parts, pr, g, args.sweep_steps, 1)
            point[pr] = {"ms_per_step": round(rs["ms_per_step"], 4), "force_err_rms": ferr(os_)[0]}
        rs, os_, _ = run_path(hpm, torch, parts, "f32", g, args.sweep_steps, 1, m2l="cells",
                              extended=True)
        point["f32_cells_extended"] = {"ms_per_step": round(rs["ms_per_step"], 4),
                                       "force_err_rms": ferr(os_)[0]}
        sweep[f"ng{g}"] = point
    meets = [g for g in (2, 3, 4, 6) if sweep[f"ng{g}"]["f32"]["force_err_rms"] < 1e-4]
    sweep["smallest_ng_at_1e-4"] = meets[0] if meets else None

    # latency of the small uniform problem (4096 particles, uniform depth 3, N_g = 4, FP64)
    from synth import uniform_cube
    pu = uniform_cube(4096, 1000)
    xu, yu, zu, mu = (torch.tensor(a_, dtype=torch.float64, device="cuda")
                      for a_ in (pu.x, pu.y, pu.z, pu.m))
    planu = hpm.Plan(hpm.Problem(ng=4, precision="f64", uniform_depth=3, softening=1e-3),
                     xu, yu, zu)
    outu = [torch.empty(pu.n, dtype=torch.float64, device="cuda") for _ in range(4)]
    lat_u = []
    for k in range(220):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        planu.rebuild(xu, yu, zu)
        planu.execute(mu, *outu)
        e1.record()
        e1.synchronize()
        if k >= 20:
            lat_u.append(e0.elapsed_time(e1))
    planu.close()
    small = {"workload": "uniform cube N=4096, uniform depth 3, N_g=4, eps=1e-3, FP64",
             "solves": len(lat_u), "latency_ms": {"p50": round(float(np.percentile(lat_u, 50)), 4),
                                                  "p99": round(float(np.percentile(lat_u, 99)), 4)}}

    rec = {
        "metric": "HPM particles/s (FP32 vs FP64 GPU) at 1e-4 force err; solve p50/p99 latency",
        "value": round(value, 1), "unit": "particles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(r32["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "precision_note": "f32 path: FP32 arithmetic and storage except the source-to-target "
                          "step's inverse-x sums and per-target means (FP64; the inverse-y sum "
                          "too at N_g = 8), the FP64 sum of the local constants in L2L, and "
                          "tables built in FP64",
        "data": "synthetic (seeded Plummer sphere)",
        "config": {"workload": f"plummer sphere N={args.n} a=0.05 r_t=0.5, leaf<=64, depth<=10, "
                               f"N_g={ng}, eps=1e-3", "n": args.n, "ng": ng,
                   "leaf_capacity": 64, "max_depth": 10, "softening": 1e-3,
                   "levels": r32["info"]["cells_per_level"], "targets": n_t,
                   "leaves": r32["info"]["n_leaves"]},
        "latency_ms": {"p50": round(r32["lat_p50"], 4), "p99": round(r32["lat_p99"], 4)},
        "fp64": {"value": round(v64, 1), "ms_per_step": round(r64["ms_per_step"], 4),
                 "latency_ms": {"p50": round(r64["lat_p50"], 4), "p99": round(r64["lat_p99"], 4)},
                 "force_err_rms": f64_rms, "force_err_max": f64_max},
        "fp32_over_fp64": round(value / v64, 3),
        "force_err_rms": f32_rms, "force_err_max": f32_max,
        "fp32_strict": fp32_strict,
        "phi_rel_rms_f32_vs_f64": phi_f32_vs_f64,
        "stage_ms_per_step": {k: round(v / max(r32["stages"]["n_exec"], 1), 4)
                              for k, v in r32["stages"].items() if k not in ("n_exec", "n_build")},
        "roofline": roofline,
        "near_zone": near_zone,
        "kernels": {"yukawa_f32": yukawa},
        "other_orders": {"ng4": ng4, "ng8": ng8},
        "m2l_routes": routes,
        "fastest_route": _fastest_route(routes),
        "accuracy_sweep": sweep,
        "small_solve": small,
    }
    rec["stage_ms_per_step"]["tree"] = round(r32["stages"]["tree"] / max(r32["stages"]["n_build"], 1), 4)
    # the large clustered set (2^24 particles), and the batched and served workloads (the batch
    # shortened to two timed batches; their own flags run them in full)
    for key, fn, kw in (("large", large_bench, dict(steps=3, large_routes="grid,shared,cells")),
                        ("batched", batch_bench, dict(steps=2)),
                        ("served", serve_bench, dict())):
        try:
            sub_args = argparse.Namespace(**{**vars(args), **kw})
            rec[key] = fn(sub_args)
        except Exception as e:  # a failure here must not hide the main measurement
            rec[key] = {"error": f"{type(e).__name__}: {e}"}
    if cpu is not None:
        rec["cpu_baseline"] = dict(cpu["all_cores"])
        rec["cpu_baseline"]["one_core"] = cpu["one_core"]
        rec["cpu_baseline"]["host"] = cpu["host"]
    else:
        rec["cpu_baseline"] = None
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
