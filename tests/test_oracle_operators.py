"""Pins of the oracle's single-cell operators: moment matching (Eq. 4), child-to-parent
(Sec. 2.3), interpolation (Eq. 6-7), and the padded-FFT source-to-target step (Sec. 2.1)."""
import numpy as np
import pytest

from oracle import hpm, tables
from oracle.tree import Tree

RNG = np.random.default_rng(12345)


def moments_about_centre(rel, m, ng, L):
    """sum_j m_j (r_j/L)^n for every tensor multi-index n (right side of Eq. 4, times 1/1)."""
    nidx = tables.multi_index(ng)
    x = rel / L
    return np.array([np.sum(m * np.prod(x ** nidx[k], axis=1)) for k in range(ng ** 3)])


@pytest.mark.parametrize("ng", [2, 3, 4, 6, 8])
def test_effective_masses_reproduce_cell_moments(ng):
    # Eq. (4): sum_p M_p x_p^n = (n!/L^n) Q_n for every n in the tensor set.
    L = 0.37
    rel = (RNG.random((50, 3)) - 0.5) * L
    m = RNG.random(50)
    mp = hpm.p2m(rel, m, ng, L)
    xp = tables.node_positions(ng)
    nidx = tables.multi_index(ng)
    lhs = np.array([np.sum(mp * np.prod(xp ** nidx[k], axis=1)) for k in range(ng ** 3)])
    rhs = moments_about_centre(rel, m, ng, L)
    assert np.max(np.abs(lhs - rhs)) / np.sum(np.abs(m)) < 1e-12


@pytest.mark.parametrize("ng", [2, 4, 6])
def test_particle_on_node_gives_its_mass_on_that_node(ng):
    L = 2.0
    xp = tables.node_positions(ng)
    q = 3 % ng ** 3
    mp = hpm.p2m(xp[q:q + 1] * L, np.array([0.7]), ng, L)
    want = np.zeros(ng ** 3)
    want[q] = 0.7
    assert np.max(np.abs(mp - want)) < 1e-12


@pytest.mark.parametrize("ng", [2, 3, 4, 6])
def test_child_to_parent_equals_direct_fit_of_parent(ng):
    # The parent's gridlet from its children (Sec. 2.3) equals the fit of all its particles.
    L = 1.0
    rel = (RNG.random((200, 3)) - 0.5) * L
    m = RNG.random(200)
    parent = hpm.p2m(rel, m, ng, L)
    kids = {}
    for c in range(8):
        a = np.array(tables.child_offset(c))
        inside = np.all((rel >= 0) == (a > 0), axis=1)
        kids[c] = hpm.p2m(rel[inside] - a * L / 2.0, m[inside], ng, L / 2.0)
    merged = hpm.m2m(kids, ng)
    assert np.max(np.abs(merged - parent)) / np.abs(parent).max() < 1e-11


def _poly(ng, seed):
    """Random polynomial of per-axis degree <= ng-1 and its gradient (callables on (k,3))."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((ng, ng, ng))

    def f(x):
        px = x[:, 0:1] ** np.arange(ng)
        py = x[:, 1:2] ** np.arange(ng)
        pz = x[:, 2:3] ** np.arange(ng)
        return np.einsum("abc,ka,kb,kc->k", c, px, py, pz)

    def grad(x):
        e = np.arange(ng)
        dpow = lambda v: e * v ** np.maximum(e - 1, 0)  # noqa: E731
        px, py, pz = (x[:, i:i + 1] ** e for i in range(3))
        dx, dy, dz = (dpow(x[:, i:i + 1]) for i in range(3))
        return np.stack([np.einsum("abc,ka,kb,kc->k", c, dx, py, pz),
                         np.einsum("abc,ka,kb,kc->k", c, px, dy, pz),
                         np.einsum("abc,ka,kb,kc->k", c, px, py, dz)], axis=1)
    return f, grad


@pytest.mark.parametrize("ng", [2, 3, 4, 6, 8])
def test_interpolant_reproduces_polynomials_and_gradients(ng):
    # Eq. (6)-(7) are exact for per-axis degree <= N_g - 1; so is the child evaluation of L2L.
    f, grad = _poly(ng, ng)
    xp = tables.node_positions(ng)
    phi = f(xp)
    L = 0.25
    x = RNG.random((40, 3)) - 0.5
    pot, acc = hpm.l2p(phi, x * L, ng, L)
    scale = np.abs(phi).max()
    assert np.max(np.abs(pot - f(x))) < 1e-11 * scale * 10 ** (ng / 2)
    assert np.max(np.abs(acc + grad(x) / L)) < 1e-10 * scale / L * 10 ** (ng / 2)
    for c in (0, 3, 7):
        a = np.array(tables.child_offset(c))
        child = hpm.l2l(phi, c, ng)
        assert np.max(np.abs(child - f((a + xp) / 2.0))) < 1e-11 * scale * 10 ** (ng / 2)


def _random_target_setup(ng, level, seed):
    rng = np.random.default_rng(seed)
    n = 4 * 8 ** level
    pos = rng.random((n, 3))
    pos[:, 0] = 0.3 + 0.4 * pos[:, 0]
    h = hpm.HPM(pos[:, 0], pos[:, 1], pos[:, 2], rng.random(n),
                hpm.Problem(ng=ng, softening=0.0, uniform_depth=level), mode="fft")
    return h


@pytest.mark.parametrize("ng", [2, 3, 4, 6, 8])
def test_fft_source_to_target_equals_direct_gridlet_sum(ng):
    # Sec. 2.1: one (8 N_g)^3 zero-padded FFT with the exact lattice Green function gives the
    # same target potentials as the 189 cube-by-cube sums, to rounding.
    h = _random_target_setup(ng, 3, 1)
    lev = h.tree.levels[3]
    for i in (0, len(lev) // 2, len(lev) - 1):
        a = h._m2l_fft(3, lev.coords[i], [(np.asarray(q), h._cube_gridlet(3, q))
                                           for q in h.tree.interaction_positions(lev.coords[i], 3)
                                           if h._cube_gridlet(3, q) is not None])
        h.mode = "direct"
        b = h.m2l(3, lev.coords[i])
        h.mode = "fft"
        assert np.max(np.abs(a - b)) < 1e-13 * np.abs(b).max()


def test_direct_source_to_target_is_pairwise_sum_over_nodes():
    # The direct route equals an independent node-as-particle pair sum.
    ng = 3
    h = _random_target_setup(ng, 3, 2)
    lev = h.tree.levels[3]
    i = len(lev) // 3
    coord = lev.coords[i]
    h.mode = "direct"
    got = h.m2l(3, coord)
    L = h.tree.cube_size(3)
    xp = tables.node_positions(ng)
    spos, sm = [], []
    for q in h.tree.interaction_positions(coord, 3):
        g = h._cube_gridlet(3, q)
        if g is not None:
            spos.append(h.tree.cube_centre(3, q) + L * xp)
            sm.append(g)
    spos, sm = np.concatenate(spos), np.concatenate(sm)
    tpos = h.tree.cube_centre(3, coord) + L * xp
    want = np.array([-np.sum(sm / np.linalg.norm(t - spos, axis=1)) for t in tpos])
    assert np.max(np.abs(got - want)) < 1e-13 * np.abs(want).max()


@pytest.mark.parametrize("ng", [2, 4])
def test_padding_to_8ng_is_needed_and_enough(ng):
    # Sec. 2.1: n = 8 N_g is exact for the target gridlet (largest axis offset under 4 N_g);
    # a 6 N_g grid wraps sources onto the target and is not.
    import scipy.fft as sfft
    rng = np.random.default_rng(3)
    n6 = 6 * ng
    src = rng.random((n6, n6, n6))
    t0 = 3 * ng  # target cube 3 of the 6-cube block (octant c = 1 along each axis)
    src[t0 - ng:t0 + 2 * ng, t0 - ng:t0 + 2 * ng, t0 - ng:t0 + 2 * ng] = 0.0
    h = 0.1
    idx = np.arange(n6)
    zz, yy, xx = np.meshgrid(idx, idx, idx, indexing="ij")
    want = np.zeros((ng, ng, ng))
    for k in range(ng):
        for j in range(ng):
            for i in range(ng):
                r = h * np.sqrt((xx - t0 - i) ** 2 + (yy - t0 - j) ** 2 + (zz - t0 - k) ** 2)
                r[src == 0] = 1.0
                want[k, j, i] = -np.sum(np.where(src > 0, src / r, 0.0))
    for n, exact in ((8 * ng, True), (6 * ng, False)):
        d = tables.periodic_distance(n)
        dz, dy, dx = np.meshgrid(d, d, d, indexing="ij")
        r2 = (dx * dx + dy * dy + dz * dz) * h * h
        r2[0, 0, 0] = h * h
        grid = np.zeros((n, n, n))
        grid[:n6, :n6, :n6] = src
        pot = sfft.irfftn(sfft.rfftn(grid) * sfft.rfftn(-1.0 / np.sqrt(r2)), s=grid.shape)
        got = pot[t0:t0 + ng, t0:t0 + ng, t0:t0 + ng]
        err = np.max(np.abs(got - want)) / np.abs(want).max()
        assert (err < 1e-12) == exact, (n, err)
