"""Pins of the oracle's second interaction kernel (screened, Yukawa) against what the mathematics
fixes. The method is kernel independent (Abstract; Sec. 4): only the lattice Green function of
the source-to-target step and the near-zone pair sum change."""
import numpy as np
import pytest

from oracle import green, hpm
from oracle.direct import direct_sum, force_error, potential_error
from synth import gridlet_node_lattice, plummer_sphere, point_source_with_tracers

LAM = 0.05


def test_force_is_minus_gradient_of_potential():
    # a = -grad phi, checked by central differences of the oracle's own potential (the two are
    # coded separately: potential() and force_coefficient()).
    rng = np.random.default_rng(3)
    src = rng.random((5, 3))
    m = rng.random(5)
    x0 = np.array([0.43, 0.51, 0.47])
    for eps in (0.0, 1e-2):
        def phi(x):
            d = x[None, :] - src
            return float(np.sum(m * green.potential(np.sum(d * d, 1), 1.3, eps, "yukawa", LAM)))
        d = x0[None, :] - src
        c = green.force_coefficient(np.sum(d * d, 1), 1.3, eps, "yukawa", LAM)
        acc = -np.sum((m * c)[:, None] * d, axis=0)
        h = 1e-6
        grad = np.array([(phi(x0 + h * e) - phi(x0 - h * e)) / (2 * h) for e in np.eye(3)])
        assert np.allclose(acc, -grad, rtol=1e-6, atol=0)


def test_screened_kernel_solves_the_modified_helmholtz_equation():
    # Away from the origin, g = -exp(-r/lam)/r satisfies lap g = g / lam^2 (eps = 0).
    r0 = np.array([0.031, -0.017, 0.022])
    h = 1e-4

    def g(v):
        return green.potential(np.array([v @ v]), 1.0, 0.0, "yukawa", LAM)[0]
    lap = sum(g(r0 + h * e) + g(r0 - h * e) - 2 * g(r0) for e in np.eye(3)) / (h * h)
    assert lap == pytest.approx(g(r0) / LAM ** 2, rel=2e-4)  # O(h^2) difference error


def test_long_screening_length_reduces_to_newton():
    p = plummer_sphere(300, 5)
    phi_n, acc_n = direct_sum(p.x, p.y, p.z, p.m, 1.0, 1e-3)
    phi_y, acc_y = direct_sum(p.x, p.y, p.z, p.m, 1.0, 1e-3, kernel="yukawa", screening=1e7)
    assert potential_error(phi_y, phi_n) < 1e-6
    assert force_error(acc_y, acc_n)[0] < 1e-6


@pytest.mark.parametrize("mode", ["fft", "direct"])
def test_gridlet_node_lattice_equals_direct_sum(mode):
    # The exactness argument of the gridlet-node case does not depend on the kernel.
    p = gridlet_node_lattice(4, 2, seed=7)
    prob = hpm.Problem(ng=4, softening=1e-3, uniform_depth=2, kernel="yukawa", screening=LAM)
    phi, _, _ = hpm.solve(p.x, p.y, p.z, p.m, prob, mode=mode)
    ref, _ = direct_sum(p.x, p.y, p.z, p.m, 1.0, 1e-3, kernel="yukawa", screening=LAM)
    assert potential_error(phi, ref) < 1e-13


def test_fft_and_direct_modes_agree():
    p = plummer_sphere(1500, 21, a=0.1)
    prob = hpm.Problem(ng=4, softening=1e-3, leaf_capacity=16, max_depth=7, kernel="yukawa",
                       screening=0.2)
    phi_f, acc_f, _ = hpm.solve(p.x, p.y, p.z, p.m, prob, mode="fft")
    phi_d, acc_d, _ = hpm.solve(p.x, p.y, p.z, p.m, prob, mode="direct")
    assert potential_error(phi_f, phi_d) < 1e-13
    assert force_error(acc_f, acc_d)[0] < 1e-11


def test_point_source_field_converges_with_gridlet_order():
    # Massless tracers around one source feel exactly the kernel of that source.
    p = point_source_with_tracers(source=(0.81, 0.77, 0.86), tracers_per_axis=12, seed=2)
    lam, eps = 0.3, 1e-3
    d = p.positions()[1:] - p.positions()[0]
    r2 = np.sum(d * d, axis=1)
    s = np.sqrt(r2 + eps * eps)
    phi_ref = -np.exp(-s / lam) / s
    a_ref = -(np.exp(-s / lam) * (1 / (lam * s * s) + 1 / s ** 3))[:, None] * d
    errs = []
    for ng in (2, 4, 6):
        prob = hpm.Problem(ng=ng, softening=eps, uniform_depth=3, kernel="yukawa", screening=lam)
        phi, acc, _ = hpm.solve(p.x, p.y, p.z, p.m, prob)
        errs.append((force_error(acc[1:], a_ref)[0], potential_error(phi[1:], phi_ref)))
    assert errs[0][0] > errs[1][0] > errs[2][0]
    assert errs[2][0] < 1e-3 and errs[2][1] < 1e-4


def test_unknown_kernel_rejected():
    with pytest.raises(ValueError):
        hpm.HPM(np.array([0.5]), np.array([0.5]), np.array([0.5]), np.array([1.0]),
                hpm.Problem(kernel="spline"))
    with pytest.raises(ValueError):
        direct_sum([0.5], [0.5], [0.5], [1.0], kernel="yukawa", screening=0.0)
