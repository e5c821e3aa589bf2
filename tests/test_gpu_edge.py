"""Degenerate and edge inputs on the HIP path, against the FP64 oracle (or a closed form).

- one particle: nothing acts on it;
- two particles in separate level-2 cells of a uniform tree: the pair interacts only through
  the source-to-target step (they are in each other's interaction zone);
- fewer particles than the leaf capacity: the root is the only leaf, no source-to-target step;
- coincident particles: the tree stops at the maximum depth with an over-full leaf, and each
  particle feels -G (n-1) m / eps;
- particles on the upper faces of the box (clamped into the last cell)."""
import numpy as np
import pytest

from oracle import hpm as ohpm
from tests.hpmcase import gpu_problem, log, rel_rms

pytestmark = pytest.mark.gpu

TOL = {"f64": dict(phi=1e-10, acc=1e-9), "f32": dict(phi=1e-5, acc=1e-4)}


def _solve(pos, m, prec, ng, kw, eps=1e-3):
    import torch
    from paper_1906_10734_amd import hpm
    dt = torch.float32 if prec == "f32" else torch.float64
    npdt = np.float32 if prec == "f32" else np.float64
    pos = np.asarray(pos, npdt)
    m = np.asarray(m, npdt)
    x, y, z, mm = (torch.tensor(a, dtype=dt, device="cuda") for a in (pos[:, 0], pos[:, 1], pos[:, 2], m))
    phi, ax, ay, az = hpm.solve(gpu_problem(ng, prec, kw, eps=eps), x, y, z, mm)
    torch.cuda.synchronize()
    acc = torch.stack([ax, ay, az], 1).double().cpu().numpy()
    return phi.double().cpu().numpy(), acc, pos.astype(np.float64), m.astype(np.float64)


def _oracle(pos, m, ng, kw, eps=1e-3):
    prob = ohpm.Problem(ng=ng, softening=eps, **kw)
    phi, acc, _ = ohpm.solve(pos[:, 0], pos[:, 1], pos[:, 2], m, prob)
    return phi, acc


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_single_particle_feels_nothing(prec):
    phi, acc, _, _ = _solve([[0.3, 0.6, 0.2]], [1.0], prec, 4, dict(leaf_capacity=8, max_depth=5))
    assert np.all(phi == 0.0) and np.all(acc == 0.0)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_two_far_particles_interact_through_source_to_target(prec):
    pos = [[0.1, 0.1, 0.1], [0.9, 0.6, 0.35]]
    m = [2.0, 3.0]
    kw = dict(uniform_depth=3)
    phi, acc, p64, m64 = _solve(pos, m, prec, 4, kw)
    ophi, oacc = _oracle(p64, m64, 4, kw)
    log(f"[edge two-body] {prec} phi {rel_rms(phi, ophi):.2e} acc {rel_rms(acc, oacc):.2e}")
    assert rel_rms(phi, ophi) < TOL[prec]["phi"]
    assert rel_rms(acc, oacc) < TOL[prec]["acc"]
    assert np.all(phi < 0)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_single_leaf_tree_is_a_direct_sum(prec):
    rng = np.random.default_rng(4)
    pos = rng.random((40, 3))
    m = rng.random(40)
    kw = dict(leaf_capacity=64, max_depth=8)
    phi, acc, p64, m64 = _solve(pos, m, prec, 4, kw)
    ophi, oacc = _oracle(p64, m64, 4, kw)
    assert rel_rms(phi, ophi) < TOL[prec]["phi"]
    assert rel_rms(acc, oacc) < TOL[prec]["acc"]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_coincident_particles(prec):
    n, eps = 100, 1e-2
    pos = np.tile([[0.61, 0.27, 0.44]], (n, 1))
    m = np.full(n, 0.5)
    phi, acc, _, _ = _solve(pos, m, prec, 4, dict(leaf_capacity=8, max_depth=6), eps=eps)
    expect = -(n - 1) * 0.5 / eps
    assert np.max(np.abs(phi - expect)) < (1e-12 if prec == "f64" else 1e-5) * abs(expect)
    assert np.max(np.abs(acc)) < 1e-9 * abs(expect)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_particles_on_upper_faces(prec):
    rng = np.random.default_rng(8)
    pos = rng.random((600, 3))
    pos[:50, 0] = 1.0
    pos[50:100, 1] = 1.0
    pos[100:120, :] = 1.0
    m = np.full(600, 1.0 / 600)
    kw = dict(leaf_capacity=8, max_depth=6)
    phi, acc, p64, m64 = _solve(pos, m, prec, 4, kw)
    ophi, oacc = _oracle(p64, m64, 4, kw)
    assert rel_rms(phi, ophi) < TOL[prec]["phi"]
    assert rel_rms(acc, oacc) < TOL[prec]["acc"]
