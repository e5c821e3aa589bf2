"""Route switching and the route autotuner (hpm_plan_set_route, hpm_plan_autotune): the three
source-to-target routes compute the same sums, so a plan built with the cell spectra may
evaluate with any of them, and the autotuner keeps the one it measures fastest on the plan's own
tree."""
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


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_route_switch_and_autotune(prec):
    """A plan built with the cell spectra evaluates by any of the three routes; they agree to the
    parity bar (FP64 1e-10, FP32 1e-5 relative RMS in potential). The autotuner keeps the
    route it measured fastest, and an evaluation after it equals one with that route set by
    hand, bit for bit."""
    import torch
    from paper_1906_10734_amd import hpm
    from tests.hpmcase import rel_rms
    x, y, z, m = _set("plummer", 1 << 15, prec)
    plan = hpm.Plan(hpm.Problem(ng=6, precision=prec, softening=1e-3, m2l="shared",
                                leaf_capacity=32), x, y, z)
    res = {}
    for route in ("grid", "cells", "shared"):
        plan.set_route(route)
        res[route] = [t.double().cpu().numpy() for t in plan(m)]
    tol = 1e-10 if prec == "f64" else 1e-5
    for route in ("cells", "shared"):
        assert rel_rms(res[route][0], res["grid"][0]) < tol, route
        acc = np.stack(res[route][1:], 1)
        assert rel_rms(acc, np.stack(res["grid"][1:], 1)) < 100 * tol, route
    best, ms = plan.autotune(m, reps=2)
    log(f"[autotune] {prec}: {best} {ms}")
    assert best in ms and set(ms) == {"grid", "cells", "shared"}
    assert ms[best] == min(ms.values())
    tuned = plan(m)
    plan.set_route(best)
    manual = plan(m)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(tuned, manual))
    # a plan made for the padded grid has only that route
    g = hpm.Plan(hpm.Problem(ng=6, precision=prec, softening=1e-3, leaf_capacity=32), x, y, z)
    with pytest.raises(hpm.HpmError):
        g.set_route("cells")
    assert g.autotune(m, reps=1)[0] == "grid"
    g.close()
    plan.close()


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_near_zone_in_line_equals_overlapped(prec):
    # from 2^16 particles the near-zone sums run on the plan's second stream beside the
    # source-to-target step; in line (hpm_plan_set_overlap 0) they give the same bits, and the
    # near-zone stage is timed either way
    import torch
    from paper_1906_10734_amd import hpm
    x, y, z, m = _set("plummer", 1 << 17, prec)
    plan = hpm.Plan(hpm.Problem(ng=4, precision=prec, softening=1e-3), x, y, z)
    plan.enable_timing(True)
    a = [t.clone() for t in plan(m)]
    plan.set_overlap(False)
    b = plan(m)
    torch.cuda.synchronize()
    assert all(torch.equal(u, v) for u, v in zip(a, b))
    st = plan.stage_times()
    log(f"[overlap] {prec}: near zone {st['p2p'] / st['n_exec']:.3f} ms per evaluation")
    assert st["n_exec"] == 2 and st["p2p"] > 0
    assert hpm._lib.hpm_plan_set_overlap(plan._h, 2) == 1  # HPM_ERR_INVALID_ARG
    plan.close()
