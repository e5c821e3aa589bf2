"""Pins of the oracle's extended target gridlet (Sec. 2.5): the gridlet widened by one node on
every side, N_g + 2 nodes per axis at the same spacing, used for the source-to-target output and
for parent-to-child and leaf interpolation (Eq. 6-7 on that node set); sources keep N_g^3
effective masses. The paper states that the (8 N_g)^3 padded transform stays exact for the
widened window, because an n-point transform samples every wavenumber up to n/2 correctly."""
import numpy as np
import pytest
import scipy.fft as sfft

from oracle import hpm, tables
from oracle.direct import direct_sum, force_error, potential_error
from synth import gridlet_node_lattice, plummer_sphere
from tests.test_oracle_operators import _poly

RNG = np.random.default_rng(77)


@pytest.mark.parametrize("ng", [2, 3, 4, 6])
def test_extended_nodes(ng):
    # N_g + 2 nodes at spacing 1/N_g: the gridlet's own nodes, plus one just outside each face
    x = tables.nodes(ng, 1)
    assert len(x) == ng + 2
    assert np.allclose(np.diff(x), 1.0 / ng, rtol=0, atol=1e-15)
    assert np.array_equal(x[1:-1], tables.nodes(ng))
    assert x[0] == pytest.approx(-0.5 - 0.5 / ng) and x[-1] == pytest.approx(0.5 + 0.5 / ng)


@pytest.mark.parametrize("ng", [2, 3, 4, 6])
def test_extended_interpolant_reproduces_polynomials(ng):
    # Eq. (6)-(7) on N_g + 2 nodes are exact for per-axis degree <= N_g + 1, at particles inside
    # the cell (with the gradient) and at a child's widened nodes (parent-to-child).
    npt = ng + 2
    f, grad = _poly(npt, 100 + ng)
    xp = tables.node_positions(ng, 1)
    phi = f(xp)
    L = 0.125
    x = RNG.random((40, 3)) - 0.5
    pot, acc = hpm.l2p(phi, x * L, ng, L, ext=1)
    scale = np.abs(phi).max()
    tol = 1e-11 * scale * 10 ** (npt / 2)
    assert np.max(np.abs(pot - f(x))) < tol
    assert np.max(np.abs(acc + grad(x) / L)) < 10 * tol / L
    for c in (0, 5, 7):
        a = np.array(tables.child_offset(c))
        child = hpm.l2l(phi, c, ng, ext=1)
        assert child.shape == (npt ** 3,)
        assert np.max(np.abs(child - f((a + xp) / 2.0))) < tol


def test_extended_window_of_the_padded_transform_is_exact():
    # The widened target window reaches offsets of up to 4 N_g nodes from a source: the
    # (8 N_g)^3 transform still gives the pairwise sums (Sec. 2.5), and so does the cell-by-cell
    # route with its (2 N_g + 2)^3 cyclic arrays.
    p = plummer_sphere(1500, 21, a=0.1)
    prob = hpm.Problem(ng=4, softening=1e-3, leaf_capacity=16, max_depth=7, extended=True)
    phi_f, acc_f, h = hpm.solve(p.x, p.y, p.z, p.m, prob, mode="fft")
    phi_d, acc_d, _ = hpm.solve(p.x, p.y, p.z, p.m, prob, mode="direct")
    phi_c, acc_c, _ = hpm.solve(p.x, p.y, p.z, p.m, prob, mode="cells")
    assert potential_error(phi_f, phi_d) < 1e-13
    assert potential_error(phi_c, phi_d) < 1e-13
    assert force_error(acc_f, acc_d)[0] < 1e-11
    assert force_error(acc_c, acc_d)[0] < 1e-11
    assert all(v.shape[1] == 6 ** 3 for v in h.all_locals().values())


def test_extended_window_fails_with_less_padding():
    # The same window on a (6 N_g)^3 grid wraps around: the padding is what makes it exact.
    p = plummer_sphere(600, 5, a=0.1)
    prob = hpm.Problem(ng=3, softening=1e-3, uniform_depth=3, extended=True)
    h = hpm.HPM(p.x, p.y, p.z, p.m, prob, mode="fft")
    lev = h.tree.levels[3]
    coord = lev.coords[len(lev) // 2]
    src = [(np.asarray(q), h._cube_gridlet(3, q)) for q in h.tree.interaction_positions(coord, 3)
           if h._cube_gridlet(3, q) is not None]
    good = h._m2l_fft(3, coord, src)
    h.mode = "direct"
    ref = h._m2l_direct(3, coord, src)
    assert np.max(np.abs(good - ref)) < 1e-12 * np.abs(ref).max()
    ng, n = 3, 18                     # a 6 N_g grid instead of 8 N_g
    origin = 2 * ((np.asarray(coord) >> 1) - 1)
    grid = np.zeros((n, n, n))
    for q, g in src:
        b = q - origin
        grid[b[2] * ng:(b[2] + 1) * ng, b[1] * ng:(b[1] + 1) * ng,
             b[0] * ng:(b[0] + 1) * ng] = g.reshape(ng, ng, ng)
    d = tables.periodic_distance(n).astype(float)
    dz, dy, dx = np.meshgrid(d, d, d, indexing="ij")
    hl = h.tree.cube_size(3) / ng
    g6 = tables.green_physical((dx * dx + dy * dy + dz * dz) * hl * hl, 1.0, 1e-3)
    pot = sfft.irfftn(sfft.rfftn(grid) * sfft.rfftn(g6), s=grid.shape)
    tb = np.asarray(coord) - origin
    sl = [slice(tb[a] * ng - 1, (tb[a] + 1) * ng + 1) for a in (2, 1, 0)]
    bad = pot[sl[0], sl[1], sl[2]].ravel()
    assert np.max(np.abs(bad - ref)) > 1e-4 * np.abs(ref).max()


def test_extended_lattice_equals_direct_sum():
    # Particles on the gridlet nodes of a depth-2 tree: the widened gridlet contains the
    # original nodes, so interpolation there returns the exact far field.
    p = gridlet_node_lattice(4, 2, seed=7)
    prob = hpm.Problem(ng=4, softening=1e-3, uniform_depth=2, extended=True)
    phi, _, _ = hpm.solve(p.x, p.y, p.z, p.m, prob)
    ref, _ = direct_sum(p.x, p.y, p.z, p.m, 1.0, 1e-3)
    assert potential_error(phi, ref) < 1e-13


def test_extended_gridlet_is_at_least_as_accurate():
    # Sec. 2.5 reports an accuracy gain from the widened gridlet; on this tree the force error
    # drops by more than a factor of 5 at N_g = 3 and 4.
    p = plummer_sphere(1500, 21, a=0.1)
    ref, aref = direct_sum(p.x, p.y, p.z, p.m, 1.0, 1e-3)
    for ng in (3, 4):
        e = []
        for ext in (False, True):
            prob = hpm.Problem(ng=ng, softening=1e-3, leaf_capacity=16, max_depth=7, extended=ext)
            _, acc, _ = hpm.solve(p.x, p.y, p.z, p.m, prob, mode="cells")
            e.append(force_error(acc, aref)[0])
        assert e[1] < e[0] / 5
