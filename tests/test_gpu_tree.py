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
