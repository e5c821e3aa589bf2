"""The all-FP32 source-to-target step (hpm_plan_set_fp32_strict: float-float instead of FP64 in
the padded-grid route's inverse x sums and target means, and in L2L's constants) against the FP64
oracle on the same seeded inputs, with the FP32 parity bars, and against the default FP32 path
(which forms those sums in FP64): both round the same float inputs, so they agree to FP32
rounding. Also the full-size 2^18 Plummer workload against its stored oracle values."""
import os

import numpy as np
import pytest

from tests.hpmcase import device, gpu_problem, log, oracle, particles, rel_max, rel_rms

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _solve(plan, m, torch):
    phi, ax, ay, az = plan(m)
    torch.cuda.synchronize()
    return phi.double().cpu().numpy(), torch.stack([ax, ay, az], 1).double().cpu().numpy()


@pytest.mark.parametrize("extended", [False, True])
@pytest.mark.parametrize("name,ng", [("plummer3000_cap16", 4), ("clustered5000_cap8", 4),
                                     ("plummer3000_cap64", 6)])
def test_strict_fp32_matches_oracle_and_default(name, ng, extended):
    import torch
    from paper_1906_10734_amd import hpm
    log(f"[strict] {name} ng={ng} extended={extended}")
    h, ophi, oacc = oracle(name, "f32", ng, extended=extended)
    p, kw = particles(name, "f32")
    x, y, z, m = device(p, torch)
    plan = hpm.Plan(gpu_problem(ng, "f32", kw, extended=extended), x, y, z)
    phi0, acc0 = _solve(plan, m, torch)
    plan.set_fp32_strict(True)
    phi, acc = _solve(plan, m, torch)
    locs = h.all_locals()
    for l in range(2, h.tree.max_level + 1):
        assert rel_max(plan.locals(l), locs[l]) < 2e-5, ("locals", l)
    e_phi, e_acc = rel_rms(phi, ophi), rel_rms(acc, oacc)
    d_phi, d_acc = rel_rms(phi, phi0), rel_rms(acc, acc0)
    log(f"   vs oracle: phi {e_phi:.2e} acc {e_acc:.2e}; vs default FP32: phi {d_phi:.2e} acc {d_acc:.2e}")
    assert e_phi < 1e-5
    assert e_acc < 1e-4
    assert d_phi < 1e-6
    assert d_acc < 1e-5
    plan.set_fp32_strict(False)
    phi1, _ = _solve(plan, m, torch)
    assert np.array_equal(phi1, phi0)  # switching back restores the default exactly
    plan.close()


def test_strict_fp32_rejected_where_not_built():
    import torch
    from paper_1906_10734_amd import hpm
    p, kw = particles("plummer3000_cap16", "f64")
    x, y, z, m = device(p, torch)
    plan = hpm.Plan(gpu_problem(4, "f64", kw), x, y, z)
    with pytest.raises(Exception):
        plan.set_fp32_strict(True)
    plan.close()


def test_strict_fp32_full_size_matches_oracle():
    import torch
    from paper_1906_10734_amd import hpm
    from synth import plummer_sphere
    gold = np.load(os.path.join(HERE, "golden", "plummer2p18_ng6_f32.npz"))
    log("[strict] plummer 2^18 ng=6 f32")
    p = plummer_sphere(2 ** 18, 1001).astype(np.float32)
    x, y, z, m = (torch.tensor(a, dtype=torch.float32, device="cuda") for a in (p.x, p.y, p.z, p.m))
    plan = hpm.Plan(hpm.Problem(ng=6, precision="f32", leaf_capacity=64, max_depth=10,
                                softening=1e-3), x, y, z)
    plan.set_fp32_strict(True)
    out = [torch.empty(p.n, dtype=torch.float32, device="cuda") for _ in range(4)]
    for _ in range(2):
        plan.rebuild(x, y, z)
        plan.execute(m, *out)
    torch.cuda.synchronize()
    s = torch.tensor(gold["sample"], device="cuda")
    phi = out[0][s].double().cpu().numpy()
    acc = torch.stack([o[s].double() for o in out[1:]], 1).cpu().numpy()
    e_phi, e_acc = rel_rms(phi, gold["phi"]), rel_rms(acc, gold["acc"])
    log(f"   sampled phi rel rms {e_phi:.2e}  acc rel rms {e_acc:.2e}")
    assert e_phi < 1e-5
    assert e_acc < 1e-4
    plan.close()
