"""An evaluation of a plan (hpm_plan_execute) launches kernels only: no allocation, no memory set,
no host synchronisation (those all belong to the tree build). So it can be captured in a HIP
graph once per tree and replayed for new masses. From 2^16 particles on, the capture includes
the fork of the near-zone sums onto the plan's second stream and their join, through events.

Each test captures one evaluation, then replays it three times with new masses copied into the
captured mass buffer, with ordinary eager work and a synchronisation between replays, and
checks every replay against an eager evaluation of the same masses, bit for bit (the kernels
take no decision that depends on timing)."""
import time

import numpy as np
import pytest

from tests.hpmcase import log

pytestmark = pytest.mark.gpu


def _set(kind, n, prec):
    import torch
    from synth import plummer_sphere, uniform_cube
    p = uniform_cube(n, 1000) if kind == "uniform" else plummer_sphere(n, 1001)
    dt = torch.float32 if prec == "f32" else torch.float64
    npdt = np.float32 if prec == "f32" else np.float64
    return [torch.tensor(a.astype(npdt), dtype=dt, device="cuda") for a in (p.x, p.y, p.z, p.m)]


@pytest.mark.parametrize("kind,n,ng,prec,kw,route", [
    ("uniform", 4096, 4, "f64", dict(uniform_depth=3), "grid"),
    ("uniform", 4096, 4, "f32", dict(uniform_depth=3), "shared"),
    ("plummer", 1 << 17, 6, "f32", dict(leaf_capacity=64), "grid"),
    ("plummer", 1 << 17, 6, "f32", dict(leaf_capacity=64), "cells"),
    ("plummer", 1 << 17, 6, "f64", dict(leaf_capacity=64), "shared"),
])
def test_captured_evaluation_replays_equal_eager(kind, n, ng, prec, kw, route):
    import torch
    from paper_1906_10734_amd import hpm
    log(f"[graph] {kind} n={n} ng={ng} {prec} {route}")
    x, y, z, m = _set(kind, n, prec)
    prob = hpm.Problem(ng=ng, precision=prec, softening=1e-3, m2l=route, **kw)
    plan = hpm.Plan(prob, x, y, z)
    m_cap = m.clone()
    out_cap = [torch.empty_like(m) for _ in range(4)]
    # warm-up on a side stream, as torch's capture expects
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.execute(m_cap, *out_cap)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.execute(m_cap, *out_cap)
    rng = np.random.default_rng(17)
    for rep in range(3):
        new_m = torch.tensor(rng.random(n) * (2.0 / n), dtype=m.dtype, device="cuda")
        m_cap.copy_(new_m)
        g.replay()
        torch.cuda.synchronize()
        eager = plan(new_m)
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(out_cap, eager)), rep
        assert torch.isfinite(out_cap[0]).all()
        _ = float((new_m * 3.0).sum())  # eager work between replays
    # launch cost: eager evaluations against replays of the same work (reported, not asserted)
    reps = 50
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.execute(m_cap, *out_cap)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    log(f"   eager {1e3 * (t1 - t0) / reps:.3f} ms, replay {1e3 * (t2 - t1) / reps:.3f} ms per evaluation")
    del g
    plan.close()

