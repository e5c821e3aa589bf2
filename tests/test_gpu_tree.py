"""Tree build on the device vs the oracle's tree rule: integer results, compared exactly."""
import numpy as np
import pytest

from oracle.tree import Tree
from tests.hpmcase import CASES, device, gpu_problem, log, particles

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name", list(CASES))
def test_tree_matches_oracle(name, prec):
    import torch
    from paper_1906_10734_amd import hpm
    log(f"[tree] {name} {prec}")
    p, kw = particles(name, prec)
    x, y, z, m = device(p, torch)
    plan = hpm.Plan(gpu_problem(4, prec, kw), x, y, z)
    t = Tree(p.as_f64().positions(), uniform_depth=kw.get("uniform_depth", 0),
             leaf_capacity=kw.get("leaf_capacity", 64), max_depth=kw.get("max_depth", 10))
    assert np.array_equal(plan.perm(), t.perm)
    info = plan.info()
    assert info["cells_per_level"] == [len(l) for l in t.levels]
    for l, lev in enumerate(t.levels):
        c = plan.cells(l)
        assert np.array_equal(c["coords"], lev.coords), l
        assert np.array_equal(c["pb"], lev.pb), l
        assert np.array_equal(c["pe"], lev.pe), l
        assert np.array_equal(c["split"], lev.split), l
        assert np.array_equal(c["parent"], lev.parent), l
    assert info["n_leaves"] == sum(int((~lev.split).sum()) for lev in t.levels)
    plan.close()


def test_tiny_hand_tree():
    import torch
    from paper_1906_10734_amd import hpm
    pos = np.array([[0.10, 0.10, 0.10], [0.90, 0.90, 0.90], [0.30, 0.30, 0.30],
                    [0.20, 0.05, 0.15], [0.60, 0.70, 0.80]])
    x, y, z = (torch.tensor(pos[:, k], dtype=torch.float64, device="cuda") for k in range(3))
    plan = hpm.Plan(hpm.Problem(ng=2, precision="f64", leaf_capacity=2, max_depth=3), x, y, z)
    assert plan.perm().tolist() == [0, 3, 2, 4, 1]
    assert plan.info()["cells_per_level"] == [1, 2, 2]
    assert plan.cells(1)["split"].tolist() == [True, False]


def test_out_of_box_and_nan_are_reported():
    import torch
    from paper_1906_10734_amd import hpm
    x = torch.tensor([0.1, 0.5, 1.5], dtype=torch.float64, device="cuda")
    y = torch.full((3,), 0.5, dtype=torch.float64, device="cuda")
    with pytest.raises(hpm.HpmError, match="OUT_OF_BOX"):
        hpm.Plan(hpm.Problem(precision="f64"), x, y, y)
    x[2] = float("nan")
    with pytest.raises(hpm.HpmError, match="NONFINITE"):
        hpm.Plan(hpm.Problem(precision="f64"), x, y, y)
    x[2] = 1.0  # the upper face belongs to the last cell
    plan = hpm.Plan(hpm.Problem(precision="f64"), x, y, y)
    assert plan.info()["n_particles"] == 3


def test_rebuild_outgrowing_the_cell_arrays():
    # 300 tight clumps of 65 particles (leaf capacity 64): each clump is a chain of one cell per
    # level down to the maximum depth, about 2400 cells for 19500 particles, more than the plan's
    # first estimate (6 n / capacity). The level loop stops where the cells outgrow the arrays,
    # the host grows them and the build resumes there; the tree must equal the oracle's exactly,
    # for a fresh plan and for a rebuild of a plan made for a small set.
    import torch
    from paper_1906_10734_amd import hpm
    from synth import uniform_cube
    rng = np.random.default_rng(5)
    centers = rng.random((300, 3)) * 0.98 + 0.01
    pos = (centers[:, None, :] + rng.random((300, 65, 3)) * 1e-5).reshape(-1, 3)
    t = Tree(pos, leaf_capacity=64, max_depth=10)
    assert sum(len(l) for l in t.levels) > 6 * len(pos) // 64 + 64
    x, y, z = (torch.tensor(pos[:, k], dtype=torch.float64, device="cuda") for k in range(3))
    small = uniform_cube(64, 31).astype(np.float64)
    xs, ys, zs, _ = device(small, torch)
    kw = dict(leaf_capacity=64, max_depth=10)
    fresh = hpm.Plan(gpu_problem(4, "f64", kw), x, y, z)
    grown = hpm.Plan(gpu_problem(4, "f64", kw), xs, ys, zs)
    grown.rebuild(x, y, z)
    for plan in (fresh, grown):
        info = plan.info()
        log(f"[tree regrow] levels {info['cells_per_level']}")
        assert info["cells_per_level"] == [len(l) for l in t.levels]
        assert np.array_equal(plan.perm(), t.perm)
        for l, lev in enumerate(t.levels):
            c = plan.cells(l)
            assert np.array_equal(c["coords"], lev.coords), l
            assert np.array_equal(c["pb"], lev.pb), l
            assert np.array_equal(c["pe"], lev.pe), l
            assert np.array_equal(c["split"], lev.split), l
            assert np.array_equal(c["parent"], lev.parent), l
        plan.close()


@pytest.mark.parametrize("n", [2 ** 21 + 12345, 2 ** 22 + 7])
def test_large_sets_sort_and_levels_match_oracle(n):
    # sets past 2^20 and 2^22 keys, where the sort passes use larger tiles (4096 and 16384 keys):
    # the permutation (stable key order) and every level's cells equal the oracle's tree
    import torch
    from paper_1906_10734_amd import hpm
    from synth import plummer_sphere
    log(f"[tree] plummer n={n}")
    p = plummer_sphere(n, 77).astype(np.float32)
    x, y, z, _ = device(p, torch)
    kw = dict(leaf_capacity=64, max_depth=10)
    plan = hpm.Plan(gpu_problem(4, "f32", kw), x, y, z)
    t = Tree(p.as_f64().positions(), leaf_capacity=64, max_depth=10)
    assert np.array_equal(plan.perm(), t.perm)
    info = plan.info()
    assert info["cells_per_level"] == [len(l) for l in t.levels]
    for l, lev in enumerate(t.levels):
        c = plan.cells(l)
        assert np.array_equal(c["pb"], lev.pb), l
        assert np.array_equal(c["pe"], lev.pe), l
        assert np.array_equal(c["split"], lev.split), l
        assert np.array_equal(c["parent"], lev.parent), l
    plan.close()
