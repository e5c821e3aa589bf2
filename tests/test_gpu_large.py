"""The largest workload, 2^24 particles (32 Plummer spheres on a 10% uniform background, at most
32 per leaf, depth at most 10, N_g = 4), checked through properties that hold at any size, since
the oracle cannot solve it in test time:

- the FP32 path matches the FP64 path to 1e-5 relative RMS in potential on sampled particles
  (the precision bar, FP64 standing in for the oracle it matches to 1e-10 on smaller trees);
- both paths' accelerations agree with the FP64 direct sum on sampled particles to the method's
  accuracy at N_g = 4 (a few 1e-3 RMS);
- the tree is complete: every particle lies in exactly one leaf (leaf ranges tile [0, n)), and
  the number of targets is what the level counts say;
- the cell-by-cell source-to-target route gives the padded grid's results: FP64 to 1e-11
  relative RMS in potential on the sampled particles, FP32 to 1e-5."""
import numpy as np
import pytest

from tests.hpmcase import log

pytestmark = pytest.mark.gpu


def test_clustered_2p24():
    import torch
    from paper_1906_10734_amd import hpm
    from synth import clustered_spheres, random_subset
    n = 2 ** 24
    parts = clustered_spheres(n, 1002)
    sample = torch.tensor(random_subset(n, 2048, 4004), device="cuda")
    out = {}
    for prec in ("f32", "f64"):
        p = parts.astype(np.float32 if prec == "f32" else np.float64)
        dt = torch.float32 if prec == "f32" else torch.float64
        x, y, z, m = (torch.tensor(a, dtype=dt, device="cuda") for a in (p.x, p.y, p.z, p.m))
        plan = hpm.Plan(hpm.Problem(ng=4, precision=prec, leaf_capacity=32, max_depth=10,
                                    softening=1e-3), x, y, z)
        phi, ax, ay, az = plan(m)
        torch.cuda.synchronize()
        info = plan.info()
        log(f"[large] {prec}: levels {info['cells_per_level']} targets {info['n_targets']}")
        assert info["n_targets"] == sum(info["cells_per_level"][2:])
        assert torch.isfinite(phi).all() and torch.isfinite(ax).all()
        # leaves tile the sorted particle range
        cover = np.zeros(n + 1, np.int64)
        for lvl in range(info["n_levels"]):
            c = plan.cells(lvl)
            leaf = ~c["split"]
            np.add.at(cover, c["pb"][leaf], 1)
            np.add.at(cover, c["pe"][leaf], -1)
        assert np.all(np.cumsum(cover)[:n] == 1)
        acc = torch.stack([ax, ay, az], 1)
        out[prec] = (phi[sample].double(), acc[sample].double(), (x, y, z, m))
        plan.close()
    e_phi = float((out["f32"][0] - out["f64"][0]).norm() / out["f64"][0].norm())
    log(f"[large] phi f32 vs f64 rel rms {e_phi:.2e}")
    assert e_phi < 1e-5
    x, y, z, m = out["f64"][2]
    _, rax, ray, raz = hpm.direct_sum(x, y, z, m, sample[:512], 1.0, 1e-3)
    ref = torch.stack([rax, ray, raz], 1)
    for prec in ("f32", "f64"):
        e = (out[prec][1][:512] - ref).norm(dim=1) / ref.norm(dim=1)
        rms = float(e.pow(2).mean().sqrt())
        log(f"[large] {prec} force error vs direct sum rms {rms:.2e}")
        assert rms < 2e-2
    # the cell-by-cell route on the same tree
    for prec, tol in (("f64", 1e-11), ("f32", 1e-5)):
        p = parts.astype(np.float32 if prec == "f32" else np.float64)
        dt = torch.float32 if prec == "f32" else torch.float64
        x, y, z, m = (torch.tensor(a, dtype=dt, device="cuda") for a in (p.x, p.y, p.z, p.m))
        phi, ax, ay, az = hpm.solve(hpm.Problem(ng=4, precision=prec, leaf_capacity=32,
                                                max_depth=10, softening=1e-3, m2l="cells"),
                                    x, y, z, m)
        torch.cuda.synchronize()
        e_c = float((phi[sample].double() - out["f64"][0]).norm() / out["f64"][0].norm())
        log(f"[large] cell route {prec}: phi vs padded grid (f64) rel rms {e_c:.2e}")
        assert e_c < tol
        del x, y, z, m, phi, ax, ay, az


def test_clustered_2p24_sampled_outputs_match_oracle():
    # Parity at the largest workload (FP32, its own precision): the oracle's values for 128
    # sampled particles and 24 sampled target cells (tests/golden/make_clustered2p24.py, oracle
    # only), same tree; bars as in the small-case parity tests (1e-5 relative RMS in potential,
    # 1e-4 in acceleration, local gridlets 2e-5 of their largest value).
    import os
    import torch
    from paper_1906_10734_amd import hpm
    from synth import clustered_spheres
    from tests.hpmcase import rel_max, rel_rms
    gold = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                "clustered2p24_ng4_f32.npz"))
    p = clustered_spheres(2 ** 24, 1002).astype(np.float32)
    x, y, z, m = (torch.tensor(a, dtype=torch.float32, device="cuda") for a in (p.x, p.y, p.z, p.m))
    plan = hpm.Plan(hpm.Problem(ng=4, precision="f32", leaf_capacity=32, max_depth=10,
                                softening=1e-3), x, y, z)
    phi, ax, ay, az = plan(m)
    torch.cuda.synchronize()
    info = plan.info()
    assert list(info["cells_per_level"][:info["n_levels"]]) == list(gold["cells_per_level"])
    assert info["n_targets"] == int(gold["n_targets"])
    s = torch.tensor(gold["sample"], device="cuda")
    e_phi = rel_rms(phi[s].double().cpu().numpy(), gold["phi"])
    acc = torch.stack([ax[s], ay[s], az[s]], 1).double().cpu().numpy()
    e_acc = rel_rms(acc, gold["acc"])
    worst = 0.0
    for lvl in np.unique(gold["cell_level"]):
        cells = plan.cells(int(lvl))
        index = {tuple(c): i for i, c in enumerate(cells["coords"].tolist())}
        loc = plan.locals(int(lvl))
        for k in np.nonzero(gold["cell_level"] == lvl)[0]:
            i = index[tuple(gold["cell_coord"][k].tolist())]
            worst = max(worst, rel_max(loc[i], gold["cell_local"][k]))
    log(f"[large] 2^24 vs oracle: phi rel rms {e_phi:.2e} acc rel rms {e_acc:.2e} "
        f"locals rel max {worst:.2e}")
    assert e_phi < 1e-5
    assert e_acc < 1e-4
    assert worst < 2e-5
    plan.close()
