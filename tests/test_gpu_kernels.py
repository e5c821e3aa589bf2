"""The screened (Yukawa) interaction kernel on the HIP path against the FP64 oracle. The method is
kernel independent (Abstract; Sec. 4): only the lattice Green function of the source-to-target
step and the near-zone pair sum change, so the parity bar is the Newtonian one: FP64 to 1e-10
relative, FP32 to 1e-5 relative RMS in potential."""
import numpy as np
import pytest

from oracle.direct import direct_sum as oracle_direct_sum
from tests.hpmcase import device, gpu_problem, log, oracle, particles, rel_max, rel_rms

pytestmark = pytest.mark.gpu

LAM = 0.05
TOL = {"f64": dict(local=1e-10, phi=1e-10, acc=1e-9), "f32": dict(local=2e-5, phi=1e-5, acc=1e-4)}


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name,ng", [("plummer3000_cap16", 4), ("clustered5000_cap8", 4),
                                     ("plummer3000_cap64", 6)])
def test_screened_kernel_matches_oracle(name, ng, prec):
    import torch
    from paper_1906_10734_amd import hpm
    log(f"[yukawa] {name} ng={ng} {prec}")
    h, ophi, oacc = oracle(name, prec, ng, kernel="yukawa", screening=LAM)
    p, kw = particles(name, prec)
    x, y, z, m = device(p, torch)
    plan = hpm.Plan(gpu_problem(ng, prec, kw, kernel="yukawa", screening=LAM), x, y, z)
    phi, ax, ay, az = plan(m)
    torch.cuda.synchronize()
    tol = TOL[prec]
    locs = h.all_locals()
    for lvl in range(2, h.tree.max_level + 1):
        assert rel_max(plan.locals(lvl), locs[lvl]) < tol["local"], ("locals", lvl)
    phi = phi.double().cpu().numpy()
    acc = torch.stack([ax, ay, az], 1).double().cpu().numpy()
    e_phi, e_acc = rel_rms(phi, ophi), rel_rms(acc, oacc)
    log(f"   phi rel rms {e_phi:.2e}  acc rel rms {e_acc:.2e}")
    assert e_phi < tol["phi"]
    assert e_acc < tol["acc"]
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_screened_direct_sum_matches_oracle(prec):
    # the GPU reference sum itself, against the oracle's O(N^2) sum
    import torch
    from paper_1906_10734_amd import hpm
    p, _ = particles("plummer3000_cap16", prec)
    x, y, z, m = device(p, torch)
    tg = torch.arange(0, p.n, 7, device="cuda", dtype=torch.int32)
    phi, ax, ay, az = hpm.direct_sum(x, y, z, m, tg, 1.0, 1e-3, kernel="yukawa", screening=LAM)
    rphi, racc = oracle_direct_sum(p.x, p.y, p.z, p.m, 1.0, 1e-3, targets=tg.cpu().numpy(),
                                   kernel="yukawa", screening=LAM)
    acc = torch.stack([ax, ay, az], 1).cpu().numpy()
    assert rel_max(phi.cpu().numpy(), rphi) < 1e-12
    assert rel_max(acc, racc) < 1e-11


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_screened_lattice_equals_direct_sum(prec):
    # gridlet-node lattice: HPM equals the direct sum for any kernel
    import torch
    from paper_1906_10734_amd import hpm
    p, kw = particles("lattice_d2", prec)
    x, y, z, m = device(p, torch)
    phi, _, _, _ = hpm.solve(gpu_problem(4, prec, kw, kernel="yukawa", screening=LAM), x, y, z, m)
    tg = torch.arange(p.n, device="cuda", dtype=torch.int32)
    rphi, _, _, _ = hpm.direct_sum(x, y, z, m, tg, 1.0, 1e-3, kernel="yukawa", screening=LAM)
    e = rel_rms(phi.double().cpu().numpy(), rphi.cpu().numpy())
    log(f"[yukawa lattice] {prec} phi vs direct {e:.2e}")
    assert e < (1e-12 if prec == "f64" else 1e-6)
