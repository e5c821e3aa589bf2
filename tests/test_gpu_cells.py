"""The cell-by-cell source-to-target route (the alternative weighed in Sec. 2.5) on the HIP path.

It computes the same interaction-zone sums as the padded (8 N_g)^3 grid (Sec. 2.1, Eq. 1), so it
is held to the same bar: against the oracle's own cell-by-cell mode (which its CPU tests pin to
the pairwise definition), FP64 to 1e-10 relative in every target gridlet and in the potential,
FP32 to 2e-5 in the gridlets and 1e-5 relative RMS in the potential; and against the padded-grid
route of this library on the same tree, FP64 to 1e-12."""
import numpy as np
import pytest

from tests.hpmcase import device, gpu_problem, log, oracle, particles, rel_max, rel_rms

pytestmark = pytest.mark.gpu

TOL = {"f64": dict(local=1e-10, phi=1e-10, acc=1e-9), "f32": dict(local=2e-5, phi=1e-5, acc=1e-4)}


def _run(name, ng, prec, m2l, **kern):
    import torch
    from paper_1906_10734_amd import hpm
    p, kw = particles(name, prec)
    x, y, z, m = device(p, torch)
    plan = hpm.Plan(gpu_problem(ng, prec, kw, m2l=m2l, **kern), x, y, z)
    phi, ax, ay, az = plan(m)
    torch.cuda.synchronize()
    info = plan.info()
    locs = {lvl: plan.locals(lvl) for lvl in range(2, info["n_levels"])}
    plan.close()
    acc = torch.stack([ax, ay, az], 1).double().cpu().numpy()
    return phi.double().cpu().numpy(), acc, locs


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name,ng,kern", [
    ("plummer3000_cap16", 4, {}),
    ("clustered5000_cap8", 2, {}),
    ("uniform4096_d3", 3, {}),
    ("plummer3000_cap64", 6, {}),
    ("plummer1000_cap1", 4, {}),
    ("plummer3000_cap16", 4, dict(kernel="yukawa", screening=0.05)),
])
def test_cells_route_matches_oracle(name, ng, kern, prec):
    log(f"[cells] {name} ng={ng} {prec} {kern}")
    h, ophi, oacc = oracle(name, prec, ng, mode="cells", **kern)
    phi, acc, locs = _run(name, ng, prec, "cells", **kern)
    tol = TOL[prec]
    olocs = h.all_locals()
    for lvl in range(2, h.tree.max_level + 1):
        e = rel_max(locs[lvl], olocs[lvl])
        assert e < tol["local"], ("locals", lvl, e)
    e_phi, e_acc = rel_rms(phi, ophi), rel_rms(acc, oacc)
    log(f"   phi rel rms {e_phi:.2e}  acc rel rms {e_acc:.2e}")
    assert e_phi < tol["phi"]
    assert e_acc < tol["acc"]


@pytest.mark.parametrize("name,ng", [("plummer3000_cap16", 4), ("plummer3000_cap64", 6)])
def test_cells_route_equals_grid_route(name, ng):
    phi_c, acc_c, loc_c = _run(name, ng, "f64", "cells")
    phi_g, acc_g, loc_g = _run(name, ng, "f64", "grid")
    for lvl in loc_c:
        assert rel_max(loc_c[lvl], loc_g[lvl]) < 1e-12, lvl
    assert rel_rms(phi_c, phi_g) < 1e-12
    assert rel_rms(acc_c, acc_g) < 1e-11


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_cells_route_two_far_particles(prec):
    # two particles in separate level-2 cells meet only through the source-to-target step
    import torch
    from paper_1906_10734_amd import hpm
    from oracle import hpm as ohpm
    pos = np.array([[0.1, 0.1, 0.1], [0.9, 0.6, 0.35]])
    m = np.array([2.0, 3.0])
    dt = torch.float32 if prec == "f32" else torch.float64
    npdt = np.float32 if prec == "f32" else np.float64
    x, y, z, mm = (torch.tensor(a.astype(npdt), dtype=dt, device="cuda")
                   for a in (pos[:, 0], pos[:, 1], pos[:, 2], m))
    phi, ax, ay, az = hpm.solve(gpu_problem(4, prec, dict(uniform_depth=3), m2l="cells"), x, y, z, mm)
    p64 = pos.astype(npdt).astype(np.float64)
    ophi, oacc, _ = ohpm.solve(p64[:, 0], p64[:, 1], p64[:, 2], m,
                               ohpm.Problem(ng=4, softening=1e-3, uniform_depth=3), mode="cells")
    acc = torch.stack([ax, ay, az], 1).double().cpu().numpy()
    assert rel_rms(phi.double().cpu().numpy(), ophi) < TOL[prec]["phi"]
    assert rel_rms(acc, oacc) < TOL[prec]["acc"]


def test_cells_route_small_trees():
    # fewer than three levels: no source-to-target step at all (root leaf)
    import torch
    from paper_1906_10734_amd import hpm
    rng = np.random.default_rng(4)
    pos = rng.random((40, 3))
    x, y, z, m = (torch.tensor(a, device="cuda") for a in (pos[:, 0], pos[:, 1], pos[:, 2], np.ones(40)))
    phi_c = hpm.solve(gpu_problem(4, "f64", dict(leaf_capacity=64), m2l="cells"), x, y, z, m)[0]
    phi_g = hpm.solve(gpu_problem(4, "f64", dict(leaf_capacity=64)), x, y, z, m)[0]
    assert torch.equal(phi_c, phi_g)


# ---- extended target gridlets (Sec. 2.5), built on the cell-by-cell route ---------------------

@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name,ng,kern", [
    ("plummer3000_cap16", 4, {}),
    ("clustered5000_cap8", 2, {}),
    ("uniform4096_d3", 3, {}),
    ("plummer3000_cap64", 6, {}),
    ("plummer3000_cap16", 4, dict(kernel="yukawa", screening=0.05)),
])
def test_extended_gridlet_matches_oracle(name, ng, kern, prec):
    # N_g + 2 target nodes per axis: the gridlets, the potentials and the accelerations against
    # the oracle's extended cell-by-cell mode, at the same bar as the other routes
    log(f"[cells ext] {name} ng={ng} {prec} {kern}")
    h, ophi, oacc = oracle(name, prec, ng, mode="cells", extended=True, **kern)
    phi, acc, locs = _run(name, ng, prec, "cells", extended=True, **kern)
    tol = TOL[prec]
    olocs = h.all_locals()
    for lvl in range(2, h.tree.max_level + 1):
        assert locs[lvl].shape == olocs[lvl].shape == (len(olocs[lvl]), (ng + 2) ** 3)
        e = rel_max(locs[lvl], olocs[lvl])
        assert e < tol["local"], ("locals", lvl, e)
    e_phi, e_acc = rel_rms(phi, ophi), rel_rms(acc, oacc)
    log(f"   phi rel rms {e_phi:.2e}  acc rel rms {e_acc:.2e}")
    assert e_phi < tol["phi"]
    assert e_acc < tol["acc"]


def test_extended_gridlet_routes_and_orders():
    # extended gridlets: cell route at every order, padded grid at N_g = 4 and 6, shared route
    # never
    import torch
    from paper_1906_10734_amd import hpm
    p, kw = particles("plummer3000_cap16", "f64")
    x, y, z, m = device(p, torch)
    for ng, m2l in ((2, "grid"), (3, "grid"), (4, "shared")):
        with pytest.raises(RuntimeError, match="HPM_ERR_UNSUPPORTED"):
            hpm.Plan(gpu_problem(ng, "f64", kw, m2l=m2l, extended=True), x, y, z)


# ---- extended target gridlets on the padded (8 N_g)^3 grid: window [(2+c) N_g - 1, (3+c) N_g + 1)

@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name,ng,kern", [
    ("plummer3000_cap16", 4, {}),
    ("clustered5000_cap8", 4, {}),
    ("uniform4096_d3", 4, {}),
    ("plummer3000_cap64", 6, {}),
    ("plummer1000_cap1", 4, {}),
    ("plummer3000_cap16", 4, dict(kernel="yukawa", screening=0.05)),
])
def test_extended_gridlet_on_grid_route_matches_oracle(name, ng, kern, prec):
    # against the oracle's extended padded-grid mode (pinned to its direct sum), the same bar
    log(f"[grid ext] {name} ng={ng} {prec} {kern}")
    h, ophi, oacc = oracle(name, prec, ng, mode="fft", extended=True, **kern)
    phi, acc, locs = _run(name, ng, prec, "grid", extended=True, **kern)
    tol = TOL[prec]
    olocs = h.all_locals()
    for lvl in range(2, h.tree.max_level + 1):
        assert locs[lvl].shape == olocs[lvl].shape == (len(olocs[lvl]), (ng + 2) ** 3)
        assert rel_max(locs[lvl], olocs[lvl]) < tol["local"], ("locals", lvl)
    e_phi, e_acc = rel_rms(phi, ophi), rel_rms(acc, oacc)
    log(f"   phi rel rms {e_phi:.2e}  acc rel rms {e_acc:.2e}")
    assert e_phi < tol["phi"]
    assert e_acc < tol["acc"]


@pytest.mark.parametrize("ng", [4, 6])
def test_extended_grid_route_equals_extended_cell_route(ng):
    phi_c, acc_c, loc_c = _run("plummer3000_cap16", ng, "f64", "cells", extended=True)
    phi_g, acc_g, loc_g = _run("plummer3000_cap16", ng, "f64", "grid", extended=True)
    for lvl in loc_c:
        assert rel_max(loc_c[lvl], loc_g[lvl]) < 1e-12, lvl
    assert rel_rms(phi_c, phi_g) < 1e-12
    assert rel_rms(acc_c, acc_g) < 1e-11
