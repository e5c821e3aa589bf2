"""Serving and batches (hpm_server_*): many independent solves in flight on the device at once.

Each request's result must be the one the same problem and particles give alone (hpm_solve on
a fresh plan): the server reuses resident plans, whose buffers keep the previous request's
contents, and runs requests on several streams at once, and neither may change a result. The
kernels take no decision that depends on timing, so the comparison is exact. Around that: a
request that can never fit the memory budget fails alone, a request with particles outside the
box fails alone, the budget bounds the memory held, and tickets are reported once."""
import numpy as np
import pytest

from tests.hpmcase import log

pytestmark = pytest.mark.gpu


def _parts(kind: str, n: int, seed: int):
    from synth import clustered_spheres, plummer_sphere, uniform_cube
    if kind == "uniform":
        return uniform_cube(n, seed)
    if kind == "plummer":
        return plummer_sphere(n, seed)
    return clustered_spheres(n, seed, n_spheres=8)


def _device(p, prec):
    import torch
    dt = torch.float32 if prec == "f32" else torch.float64
    npdt = np.float32 if prec == "f32" else np.float64
    return tuple(torch.tensor(a.astype(npdt), dtype=dt, device="cuda") for a in (p.x, p.y, p.z, p.m))


# (kind, n, seed, N_g, precision, route)
MIX = [
    ("plummer", 1 << 17, 11, 6, "f32", "grid"),
    ("uniform", 1024, 12, 4, "f32", "grid"),
    ("clustered", 20000, 13, 4, "f32", "grid"),
    ("plummer", 70000, 14, 6, "f64", "grid"),
    ("uniform", 5000, 15, 6, "f32", "grid"),
    ("plummer", 3000, 16, 4, "f64", "grid"),
    ("clustered", 90000, 17, 6, "f32", "cells"),
    ("uniform", 40000, 18, 4, "f32", "grid"),
    ("plummer", 9000, 19, 6, "f32", "grid"),
    ("uniform", 2048, 20, 6, "f32", "grid"),
    ("plummer", 30000, 21, 4, "f32", "grid"),
    ("clustered", 4096, 22, 6, "f64", "grid"),
    ("plummer", 60000, 23, 6, "f32", "shared"),
    ("uniform", 12000, 24, 4, "f64", "shared"),
]


def _problem(ng, prec, route):
    from paper_1906_10734_amd import hpm
    return hpm.Problem(ng=ng, precision=prec, m2l=route, leaf_capacity=64, max_depth=10,
                       softening=1e-3)


@pytest.fixture(scope="module")
def mix():
    """Inputs on the device and each request's result alone (hpm_solve, fresh plan)."""
    from paper_1906_10734_amd import hpm
    cases = []
    for kind, n, seed, ng, prec, route in MIX:
        dev = _device(_parts(kind, n, seed), prec)
        prob = _problem(ng, prec, route)
        solo = hpm.solve(prob, *dev)
        cases.append((prob, dev, solo))
    import torch
    torch.cuda.synchronize()
    return cases


def _same(a, b) -> bool:
    import torch
    return all(torch.equal(u, v) for u, v in zip(a, b))


def test_results_in_the_mix_equal_results_alone(mix):
    """Requests arriving while others run (two waves, the second submitted before the first has
    finished), four slots, plans reused across requests of different sizes: every output equal
    to the solve alone, bit for bit."""
    from paper_1906_10734_amd import hpm
    with hpm.Server(slots=4) as sv:
        tickets = [sv.submit(prob, *dev) for prob, dev, _ in mix[:6]]
        tickets += [sv.submit(prob, *dev) for prob, dev, _ in mix[6:]]
        # the same requests again: now every one is served by a resident, reused plan
        tickets += [sv.submit(prob, *dev) for prob, dev, _ in mix]
        res = [sv.wait(t) for t in tickets]
        st = sv.stats()
    log(f"[server] stats {st}")
    for k, (info, out) in enumerate(res):
        prob, dev, solo = mix[k % len(mix)]
        assert info["status"] == "HPM_OK", (k, info)
        assert _same(out, solo), (k, MIX[k % len(MIX)])
    assert st["completed"] == len(tickets) and st["failed"] == 0
    assert st["plans"] <= 4 * len({(c[3], c[4], c[5]) for c in MIX})
    overlap = sum(1 for a, _ in res for b, _ in res
                  if a is not b and a["start_ms"] < b["done_ms"] and b["start_ms"] < a["done_ms"])
    log(f"[server] overlapping request pairs: {overlap // 2}")
    assert overlap > 0


def test_batch_equals_results_alone(mix):
    from paper_1906_10734_amd import hpm
    with hpm.Server(slots=8) as sv:
        statuses, outs = sv.run_batch([c[0] for c in mix], [c[1] for c in mix])
    assert statuses == ["HPM_OK"] * len(mix)
    for k, (prob, dev, solo) in enumerate(mix):
        assert _same(outs[k], solo), MIX[k]


def test_memory_budget_bounds_the_plans_held(mix):
    """A budget just above the largest request's estimate, so that it runs with little else beside
    it: everything still completes, equal to the solves alone; the memory held never exceeds the
    budget, since each plan's measured size stays within its estimate; idle plans are released
    to make room."""
    from paper_1906_10734_amd import hpm
    est = [hpm.plan_bytes_estimate(prob, int(dev[0].numel())) for prob, dev, _ in mix]
    budget = int(1.1 * max(est))
    with hpm.Server(slots=4, hbm_budget=budget) as sv:
        tickets = [sv.submit(prob, *dev) for prob, dev, _ in mix + mix]
        res = [sv.wait(t) for t in tickets]
        st = sv.stats()
    log(f"[server] budget {budget}: stats {st}")
    # a reused plan has grown to the largest request of its problem that it served
    most = {}
    for (prob, _, _), e in zip(mix, est):
        most[repr(prob)] = max(most.get(repr(prob), 0), e)
    for j, (info, out) in enumerate(res):
        k = j % len(mix)
        assert info["status"] == "HPM_OK", info
        log(f"[server] {MIX[k]}: plan {info['plan_bytes']} estimate {info['estimate_bytes']}")
        assert info["plan_bytes"] <= most[repr(mix[k][0])], (MIX[k], info)
        assert _same(out, mix[k][2]), MIX[k]
    assert st["peak_held_bytes"] <= budget
    assert st["plans_released"] > 0


def test_request_beyond_the_budget_fails_alone(mix):
    from paper_1906_10734_amd import hpm
    small = mix[1]  # 1024 particles
    big = mix[0]    # 2^17 particles
    budget = int(1.05 * hpm.plan_bytes_estimate(small[0], int(small[1][0].numel())))
    with hpm.Server(slots=2, hbm_budget=budget) as sv:
        t_big = sv.submit(big[0], *big[1])
        t_small = sv.submit(small[0], *small[1])
        info_big, _ = sv.wait(t_big)
        info_small, out_small = sv.wait(t_small)
    assert info_big["status"] == "HPM_ERR_NO_MEMORY" and info_big["slot"] == -1
    assert info_small["status"] == "HPM_OK"
    assert _same(out_small, small[2])


def test_request_out_of_the_box_fails_alone(mix):
    import torch
    from paper_1906_10734_amd import hpm
    prob, dev, solo = mix[4]
    bad = tuple(t.clone() for t in dev)
    bad[0][17] = 1.5  # outside [0, 1]
    torch.cuda.synchronize()
    with hpm.Server(slots=2) as sv:
        t1 = sv.submit(prob, *bad)
        t2 = sv.submit(prob, *dev)
        t3 = sv.submit(prob, *bad)
        t4 = sv.submit(prob, *dev)
        r = [sv.wait(t) for t in (t1, t2, t3, t4)]
    assert [i["status"] for i, _ in r] == ["HPM_ERR_OUT_OF_BOX", "HPM_OK",
                                          "HPM_ERR_OUT_OF_BOX", "HPM_OK"]
    assert _same(r[1][1], solo) and _same(r[3][1], solo)


def test_tickets_are_reported_once(mix):
    from paper_1906_10734_amd import hpm
    prob, dev, solo = mix[1]
    with hpm.Server(slots=1) as sv:
        t = sv.submit(prob, *dev)
        got = None
        while got is None:
            got = sv.poll(t)
        assert got[0]["status"] == "HPM_OK" and _same(got[1], solo)
        with pytest.raises(hpm.HpmError):
            sv.wait(t)
        with pytest.raises(hpm.HpmError):
            sv.poll(t + 1000)


def test_submissions_from_several_host_threads(mix):
    """Six host threads submit and wait for their own requests on one server at once: every
    result is the solve alone."""
    import threading
    from paper_1906_10734_amd import hpm
    results, errors = {}, []
    with hpm.Server(slots=4) as sv:
        def client(k):
            try:
                got = []
                for j in range(3):
                    i = (k + 5 * j) % len(mix)
                    t = sv.submit(mix[i][0], *mix[i][1])
                    got.append((i, sv.wait(t)))
                results[k] = got
            except Exception as e:  # reported below, in the test's thread
                errors.append(e)
        threads = [threading.Thread(target=client, args=(k,)) for k in range(6)]
        for t in threads:
            t.start()
        for t in threads:
            t.join(timeout=120)
        st = sv.stats()
    assert not errors, errors
    assert len(results) == 6 and st["completed"] == 18 and st["failed"] == 0
    for got in results.values():
        for i, (info, out) in got:
            assert info["status"] == "HPM_OK"
            assert _same(out, mix[i][2]), MIX[i]
