"""Pins of the whole oracle HPM against what the paper and the mathematics fix."""
import numpy as np
import pytest

from oracle import hpm
from oracle.direct import direct_sum, force_error, potential_error
from synth import gridlet_node_lattice, plummer_sphere, point_source_with_tracers, uniform_cube


@pytest.mark.parametrize("eps", [0.0, 1e-3])
@pytest.mark.parametrize("mode", ["fft", "direct"])
def test_particles_on_gridlet_nodes_reproduce_direct_sum(eps, mode):
    # Sec. 2 (the Liska special case): with one particle on every node of a uniform level-2
    # mesh the effective masses are the particle masses, the padded FFT is exact, level-1 local
    # potentials vanish and Eq. (7) is exact at nodes, so HPM equals the direct sum.
    p = gridlet_node_lattice(4, 2, seed=7)
    prob = hpm.Problem(ng=4, softening=eps, uniform_depth=2)
    phi, acc, _ = hpm.solve(p.x, p.y, p.z, p.m, prob, mode=mode)
    ref, _ = direct_sum(p.x, p.y, p.z, p.m, 1.0, eps)
    assert potential_error(phi, ref) < 1e-13
    assert np.max(np.abs(phi - ref) / np.abs(ref)) < 1e-12


def test_two_body_closed_form():
    x, y, z = np.array([0.1, 0.4]), np.array([0.2, 0.6]), np.array([0.3, 0.3])
    m = np.array([2.0, 3.0])
    phi, acc = direct_sum(x, y, z, m, 1.5, 0.1)
    r2 = 0.3 ** 2 + 0.4 ** 2
    assert phi[0] == pytest.approx(-1.5 * 3.0 / np.sqrt(r2 + 0.01))
    assert phi[1] == pytest.approx(-1.5 * 2.0 / np.sqrt(r2 + 0.01))
    assert acc[0] == pytest.approx(1.5 * 3.0 * np.array([0.3, 0.4, 0.0]) / (r2 + 0.01) ** 1.5)
    assert acc[1] == pytest.approx(-1.5 * 2.0 * np.array([0.3, 0.4, 0.0]) / (r2 + 0.01) ** 1.5)


def test_fft_and_direct_modes_agree_on_adaptive_tree():
    # Includes interaction-zone cubes that lie inside coarser leaves.
    p = plummer_sphere(1200, 3, a=0.08)
    prob = hpm.Problem(ng=3, softening=1e-3, leaf_capacity=12, max_depth=6)
    a_phi, a_acc, h = hpm.solve(p.x, p.y, p.z, p.m, prob, mode="fft")
    assert len(h._virtual) > 0
    b_phi, b_acc, _ = hpm.solve(p.x, p.y, p.z, p.m, prob, mode="direct")
    assert potential_error(a_phi, b_phi) < 1e-13
    assert np.max(np.abs(a_acc - b_acc)) < 1e-12 * np.abs(b_acc).max()


def test_linear_in_masses():
    # Sec. 3.2: the Poisson equation is linear; so is every HPM step.
    p = plummer_sphere(1500, 4, a=0.1)
    rng = np.random.default_rng(9)
    m1, m2 = rng.random(p.n), rng.random(p.n)
    prob = hpm.Problem(ng=4, softening=1e-3, leaf_capacity=16, max_depth=6)
    f = lambda m: hpm.solve(p.x, p.y, p.z, m, prob)[:2]  # noqa: E731
    p1, a1 = f(m1)
    p2, a2 = f(m2)
    p12, a12 = f(2.0 * m1 + m2)
    assert np.max(np.abs(p12 - (2 * p1 + p2))) < 1e-13 * np.abs(p12).max()
    assert np.max(np.abs(a12 - (2 * a1 + a2))) < 1e-12 * np.abs(a12).max()


def test_point_source_error_falls_with_gridlet_order():
    # Sec. 3.2 test: a point source, relative acceleration error against the analytic field.
    p = point_source_with_tracers(source=(0.81, 0.77, 0.86), tracers_per_axis=12, seed=2)
    eps = 1e-3
    d = p.positions()[1:] - p.positions()[0]
    r2 = np.sum(d * d, axis=1) + eps * eps
    a_ref = -d / r2[:, None] ** 1.5
    errs = []
    for ng in (2, 4, 6):
        prob = hpm.Problem(ng=ng, softening=eps, uniform_depth=3)
        phi, acc, _ = hpm.solve(p.x, p.y, p.z, p.m, prob)
        errs.append(force_error(acc[1:], a_ref)[0])
        assert potential_error(phi[1:], -1.0 / np.sqrt(r2)) < [3e-2, 2e-3, 1e-4][len(errs) - 1]
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-3


def test_uniform_cube_force_error_vs_direct_sum():
    # Convergence on the 4096-particle uniform workload; N_g = 6 reaches 1e-4 RMS force error.
    p = uniform_cube(4096, 1000)
    ref_phi, ref_acc = direct_sum(p.x, p.y, p.z, p.m, 1.0, 1e-3)
    out = {}
    for ng in (2, 4):
        prob = hpm.Problem(ng=ng, softening=1e-3, uniform_depth=3)
        phi, acc, _ = hpm.solve(p.x, p.y, p.z, p.m, prob)
        out[ng] = (force_error(acc, ref_acc)[0], potential_error(phi, ref_phi))
    assert out[2][0] > out[4][0]
    assert out[4][0] < 5e-3 and out[4][1] < 1e-4


def test_uniform_sphere_closed_form():
    # Uniform ball of radius R and mass 1: phi = -(3R^2 - r^2)/(2R^3) inside; shot noise ~ 1/sqrt(N).
    rng = np.random.default_rng(11)
    n, R = 6000, 0.3
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    pos = 0.5 + v * (R * rng.random(n) ** (1 / 3))[:, None]
    m = np.full(n, 1.0 / n)
    prob = hpm.Problem(ng=4, softening=1e-3, leaf_capacity=32, max_depth=7)
    phi, _, _ = hpm.solve(pos[:, 0], pos[:, 1], pos[:, 2], m, prob)
    r = np.linalg.norm(pos - 0.5, axis=1)
    want = -(3 * R * R - r * r) / (2 * R ** 3)
    assert potential_error(phi, want) < 3.0 / np.sqrt(n)


@pytest.mark.parametrize("kernel,screening", [("newton", 0.0), ("yukawa", 0.2)])
def test_cell_by_cell_transforms_equal_direct_mode(kernel, screening):
    # Sec. 2.5's alternative (a padded (2 N_g)^3 transform per source cube, products summed and
    # transformed back once) computes the same source-to-target sums as the definition.
    p = plummer_sphere(1500, 21, a=0.1)
    prob = hpm.Problem(ng=4, softening=1e-3, leaf_capacity=16, max_depth=7, kernel=kernel,
                       screening=screening)
    phi_c, acc_c, _ = hpm.solve(p.x, p.y, p.z, p.m, prob, mode="cells")
    phi_d, acc_d, _ = hpm.solve(p.x, p.y, p.z, p.m, prob, mode="direct")
    assert potential_error(phi_c, phi_d) < 1e-13
    assert force_error(acc_c, acc_d)[0] < 1e-11


def test_outer_and_central_cubes_partition_every_childs_zone():
    # The sets the shared-transform route splits a child's zone into: the block cubes outside the
    # central 4^3 (common to all 8 children) and the central cubes off the child's near zone.
    # Brute force over the 8 children of an interior parent: disjoint, and their union is the
    # zone (189 = 152 + 37).
    from oracle.tree import Tree
    parent = np.array([5, 6, 7])
    origin = 2 * (parent - 1)
    for c in range(8):
        child = 2 * parent + np.array([c & 1, (c >> 1) & 1, (c >> 2) & 1])
        zone = {tuple(q) for q in Tree.interaction_positions(child, 5)}
        outer = {tuple(origin + np.array(b)) for b in np.ndindex(6, 6, 6)
                 if not all(1 <= v <= 4 for v in b)}
        central = {tuple(origin + np.array(b)) for b in np.ndindex(6, 6, 6)
                   if all(1 <= v <= 4 for v in b)}
        near = {tuple(child + np.array(d) - 1) for d in np.ndindex(3, 3, 3)}
        assert len(zone) == 189 and len(outer) == 152
        assert outer <= zone and (central - near) <= zone
        assert outer | (central - near) == zone and not (outer & (central - near))
        assert len(central - near) == 37


@pytest.mark.parametrize("kernel,screening", [("newton", 0.0), ("yukawa", 0.2)])
def test_shared_transform_equals_direct_mode(kernel, screening):
    # The transform shared by siblings (one padded grid of the outer cubes per parent, the central
    # cubes cell by cell) computes the same sums as the definition, on an adaptive tree with
    # cubes inside coarser leaves and zones cut by the box faces.
    p = plummer_sphere(1500, 21, a=0.1)
    prob = hpm.Problem(ng=4, softening=1e-3, leaf_capacity=16, max_depth=7, kernel=kernel,
                       screening=screening)
    phi_s, acc_s, h = hpm.solve(p.x, p.y, p.z, p.m, prob, mode="shared")
    assert len(h._shared) > 0 and len(h._virtual) > 0
    phi_d, acc_d, _ = hpm.solve(p.x, p.y, p.z, p.m, prob, mode="direct")
    assert potential_error(phi_s, phi_d) < 1e-13
    assert force_error(acc_s, acc_d)[0] < 1e-11


def test_shared_transform_on_the_node_lattice_equals_direct_sum():
    p = gridlet_node_lattice(3, 2, seed=7)
    prob = hpm.Problem(ng=3, softening=1e-3, uniform_depth=2)
    phi, _, _ = hpm.solve(p.x, p.y, p.z, p.m, prob, mode="shared")
    ref, _ = direct_sum(p.x, p.y, p.z, p.m, 1.0, 1e-3)
    assert potential_error(phi, ref) < 1e-13
