"""Units, box placement and the force-error reference on the HIP path.

- The Newtonian device direct sum (hpm_direct_sum, the reference of every reported force error,
  Sec. 3.2's accuracy measure) against the oracle's O(N^2) sum, potential and acceleration, with
  G != 1 and softening.
- A whole solve with G = 2.5 in a box of size 2 placed at (-1, -0.5, 0.25): the far field takes
  G and the node spacing h_l = size / (2^l N_g) from the Green tables (Eq. 1), the near field
  multiplies by G in the leaf pass, and cell centres come from box_lo; the oracle gets the same
  problem. Every source-to-target route, both precisions, against the parity bars: FP64 1e-10
  relative per particle in potential, FP32 1e-5 relative RMS in potential (accelerations 1e-9 and
  1e-4 relative RMS)."""
import numpy as np
import pytest

from oracle import hpm as ohpm
from oracle.direct import direct_sum as oracle_direct_sum
from synth import plummer_sphere
from tests.hpmcase import log, rel_each_max, rel_max, rel_rms

pytestmark = pytest.mark.gpu

G = 2.5
BOX_LO = (-1.0, -0.5, 0.25)
BOX = 2.0


def _placed(prec):
    p = plummer_sphere(3000, 21, a=0.08)
    dt = np.float32 if prec == "f32" else np.float64
    x = BOX_LO[0] + BOX * p.x
    y = BOX_LO[1] + BOX * p.y
    z = BOX_LO[2] + BOX * p.z
    return [np.ascontiguousarray(a, dt) for a in (x, y, z, p.m)]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_newtonian_direct_sum_matches_oracle(prec):
    import torch
    from paper_1906_10734_amd import hpm
    x, y, z, m = _placed(prec)
    dt = torch.float32 if prec == "f32" else torch.float64
    tx, ty, tz, tm = (torch.tensor(a, dtype=dt, device="cuda") for a in (x, y, z, m))
    tg = torch.arange(0, x.size, 5, device="cuda", dtype=torch.int32)
    phi, ax, ay, az = hpm.direct_sum(tx, ty, tz, tm, tg, G, 2e-3)
    rphi, racc = oracle_direct_sum(x, y, z, m, G, 2e-3, targets=tg.cpu().numpy())
    acc = torch.stack([ax, ay, az], 1).cpu().numpy()
    e_phi, e_acc = rel_each_max(phi.cpu().numpy(), rphi), rel_each_max(acc, racc)
    log(f"[direct] {prec} per-particle phi {e_phi:.2e} acc {e_acc:.2e}")
    assert e_phi < 1e-12
    assert e_acc < 1e-11


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("m2l,ng", [("grid", 4), ("grid", 6), ("cells", 4), ("shared", 6)])
def test_gconst_and_placed_box_match_oracle(m2l, ng, prec):
    import torch
    from paper_1906_10734_amd import hpm
    x, y, z, m = _placed(prec)
    kw = dict(leaf_capacity=16, max_depth=7)
    prob = ohpm.Problem(ng=ng, softening=2e-3, gconst=G, box_lo=BOX_LO, box_size=BOX, **kw)
    ophi, oacc, h = ohpm.solve(x, y, z, m, prob)
    dt = torch.float32 if prec == "f32" else torch.float64
    tx, ty, tz, tm = (torch.tensor(a, dtype=dt, device="cuda") for a in (x, y, z, m))
    plan = hpm.Plan(hpm.Problem(ng=ng, precision=prec, softening=2e-3, gconst=G, box_lo=BOX_LO,
                                box_size=BOX, m2l=m2l, **kw), tx, ty, tz)
    phi, ax, ay, az = plan(tm)
    torch.cuda.synchronize()
    locs = h.all_locals()
    for lvl in range(2, h.tree.max_level + 1):
        assert rel_max(plan.locals(lvl), locs[lvl]) < (1e-10 if prec == "f64" else 2e-5), lvl
    phi = phi.double().cpu().numpy()
    acc = torch.stack([ax, ay, az], 1).double().cpu().numpy()
    e_phi, e_acc = rel_rms(phi, ophi), rel_rms(acc, oacc)
    log(f"[units] G={G} box {BOX} at {BOX_LO} {m2l} ng={ng} {prec}: phi {e_phi:.2e} acc {e_acc:.2e}")
    if prec == "f64":
        assert rel_each_max(phi, ophi) < 1e-10
        assert e_acc < 1e-9
    else:
        assert e_phi < 1e-5
        assert e_acc < 1e-4
    plan.close()
