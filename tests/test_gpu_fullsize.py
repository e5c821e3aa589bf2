"""Full-size parity: the 2^18-particle Plummer workload, solved exactly as the benchmark solves it
(same problem, same plan calls), checked on sampled outputs against values the FP64 oracle wrote
(tests/golden/make_plummer2p18.py): 256 particles' potentials and accelerations, and the local
gridlet potentials of 48 target cells at levels >= 2, matched by level and integer coordinates.
Every source-to-target route the benchmark times is checked: the padded grid, the cell-by-cell
route and the route with the transform shared by siblings (against the same values: the oracle's
modes agree to rounding), and the padded grid and the cell route with extended target gridlets
(against the oracle's extended values).

Tolerances as in the small-case parity tests: FP64 path 1e-10 relative per particle (potential
and acceleration), FP32 path 1e-5 relative RMS in potential (acceleration 1e-4, local gridlets
2e-5 of the level's largest value)."""
import os

import numpy as np
import pytest

from tests.hpmcase import log, rel_each_max, rel_max, rel_rms

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = {"f64": dict(local=1e-10, phi=1e-10, acc=1e-9),
       "f32": dict(local=2e-5, phi=1e-5, acc=1e-4)}


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("ng,extended", [(4, False), (6, False), (4, True), (6, True)])
def test_plummer2p18_sampled_outputs_match_oracle(ng, extended, prec):
    _check(ng, prec, "grid", extended)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("ng,extended", [(4, False), (6, False), (4, True), (6, True)])
def test_plummer2p18_cell_route_matches_oracle(ng, extended, prec):
    _check(ng, prec, "cells", extended)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("ng", [4, 6])
def test_plummer2p18_shared_route_matches_oracle(ng, prec):
    _check(ng, prec, "shared", False)


def _check(ng, prec, m2l, extended):
    import torch
    from paper_1906_10734_amd import hpm
    from synth import plummer_sphere
    tag = "_ext" if extended else ""
    gold = np.load(os.path.join(HERE, "golden", f"plummer2p18_ng{ng}{tag}_{prec}.npz"))
    log(f"[fullsize] plummer 2^18 ng={ng} {prec} {m2l}{tag}")
    p = plummer_sphere(2 ** 18, 1001).astype(np.float32 if prec == "f32" else np.float64)
    dt = torch.float32 if prec == "f32" else torch.float64
    x, y, z, m = (torch.tensor(a, dtype=dt, device="cuda") for a in (p.x, p.y, p.z, p.m))
    plan = hpm.Plan(hpm.Problem(ng=ng, precision=prec, leaf_capacity=64, max_depth=10,
                                softening=1e-3, m2l=m2l, extended=extended), x, y, z)
    out = [torch.empty(p.n, dtype=dt, device="cuda") for _ in range(4)]
    for _ in range(2):  # the benchmark's step: rebuild, then execute
        plan.rebuild(x, y, z)
        plan.execute(m, *out)
    torch.cuda.synchronize()
    info = plan.info()
    cpl = list(info["cells_per_level"][:info["n_levels"]])
    assert cpl == list(gold["cells_per_level"]), "tree differs from the oracle's"
    assert info["n_targets"] == int(gold["n_targets"])

    s = torch.tensor(gold["sample"], device="cuda")
    phi = out[0][s].double().cpu().numpy()
    acc = torch.stack([o[s].double() for o in out[1:]], 1).cpu().numpy()
    tol = TOL[prec]
    e_phi, e_acc = rel_rms(phi, gold["phi"]), rel_rms(acc, gold["acc"])
    log(f"   sampled phi rel rms {e_phi:.2e}  acc rel rms {e_acc:.2e}")
    assert e_phi < tol["phi"]
    assert e_acc < tol["acc"]
    if prec == "f64":
        assert rel_max(phi, gold["phi"]) < 1e-10
        assert rel_each_max(phi, gold["phi"]) < 1e-10
        assert rel_each_max(acc, gold["acc"]) < 1e-10

    worst = 0.0
    for lvl in np.unique(gold["cell_level"]):
        cells = plan.cells(int(lvl))
        index = {tuple(c): i for i, c in enumerate(cells["coords"].tolist())}
        loc = plan.locals(int(lvl))
        for k in np.nonzero(gold["cell_level"] == lvl)[0]:
            i = index[tuple(gold["cell_coord"][k].tolist())]
            ref = gold["cell_local"][k]
            worst = max(worst, float(np.max(np.abs(loc[i] - ref)) / np.max(np.abs(ref))))
    log(f"   sampled locals rel max {worst:.2e}")
    assert worst < tol["local"]
    plan.close()
