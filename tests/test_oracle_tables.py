"""Pins of the oracle's constant tables against what Sec. 2.2, Sec. 2.3 and Eq. (1) fix."""
import itertools

import numpy as np
import pytest

from oracle import tables

NGS = [2, 3, 4, 5, 6, 7, 8]


def lagrange_1d(ng, u):
    """Independent closed form: l_p(u) = prod_{m != p} (u - x_m) / (x_p - x_m)."""
    xs = [(k + 0.5) / ng - 0.5 for k in range(ng)]
    out = np.ones((ng,) + np.shape(u))
    for p in range(ng):
        for m in range(ng):
            if m != p:
                out[p] *= (np.asarray(u) - xs[m]) / (xs[p] - xs[m])
    return out


@pytest.mark.parametrize("ng", NGS)
def test_nodes_are_cell_centred(ng):
    # Sec. 2.2: x_p = (i + 1/2)/N_g - 1/2, symmetric about 0, spacing 1/N_g.
    x = tables.nodes(ng)
    assert np.allclose(x, -x[::-1], atol=0)
    assert np.allclose(np.diff(x), 1.0 / ng, rtol=0, atol=1e-15)
    assert x[0] == pytest.approx(0.5 / ng - 0.5)


@pytest.mark.parametrize("ng", NGS)
def test_inverse_1d_is_inverse(ng):
    a1, b1 = tables.vandermonde_1d(ng), tables.inverse_1d(ng)
    assert np.max(np.abs(b1 @ a1 - np.eye(ng))) < 1e-12 * max(1, np.abs(b1).max())
    assert np.max(np.abs(a1 @ b1 - np.eye(ng))) < 1e-12 * max(1, np.abs(b1).max())


@pytest.mark.parametrize("ng", [2, 3, 4])
def test_inverse_3d_is_inverse_of_vandermonde_3d(ng):
    # A_{np} = x_p^n over multi-indices, built here element by element (not via Kronecker).
    xp = tables.node_positions(ng)
    nidx = tables.multi_index(ng)
    a = np.array([[np.prod(xp[p] ** nidx[n]) for p in range(ng ** 3)] for n in range(ng ** 3)])
    assert np.allclose(a, tables.vandermonde_3d(ng), rtol=0, atol=1e-15)
    assert np.max(np.abs(tables.inverse_3d(ng) @ a - np.eye(ng ** 3))) < 1e-10


@pytest.mark.parametrize("ng", NGS)
def test_inverse_rows_are_lagrange_coefficients(ng):
    # sum_n B_pn u^n is the polynomial that is 1 at node p and 0 at the others.
    u = np.linspace(-0.5, 0.5, 11)
    poly = tables.inverse_1d(ng) @ (u[None, :] ** np.arange(ng)[:, None])
    assert np.max(np.abs(poly - lagrange_1d(ng, u))) < 1e-10


@pytest.mark.parametrize("ng", NGS)
@pytest.mark.parametrize("a", [-0.5, 0.5])
def test_child_to_parent_1d_equals_lagrange_at_shifted_nodes(ng, a):
    # Sec. 2.3 formula vs the closed form T1[p, q] = l_p((a + x_q)/2).
    t1 = tables.child_to_parent_1d(ng, a)
    u = (a + tables.nodes(ng)) / 2.0
    assert np.max(np.abs(t1 - lagrange_1d(ng, u))) < 1e-10


@pytest.mark.parametrize("ng", [2, 3, 4])
def test_child_to_parent_3d_matches_formula_elementwise(ng):
    # Full multi-index double sum of Sec. 2.3 for one child, against the factorised matrix.
    from math import comb
    c = 5
    a = np.array(tables.child_offset(c))
    b = tables.inverse_3d(ng)
    av = tables.vandermonde_3d(ng)
    nidx = tables.multi_index(ng)
    M = ng ** 3
    t = np.zeros((M, M))
    for n in range(M):
        for m in range(M):
            if np.any(nidx[m] > nidx[n]):
                continue
            k = nidx[n] - nidx[m]
            coef = np.prod([comb(int(nidx[n][i]), int(nidx[m][i])) for i in range(3)])
            coef *= np.prod(a ** k) / 2.0 ** nidx[n].sum()
            t += coef * np.outer(b[:, n], av[m, :])
    assert np.max(np.abs(t - tables.child_to_parent(ng, c))) < 1e-10


def test_child_offsets_follow_paper_numbering():
    # Sec. 2.3: child 1 is (-1/2,-1/2,-1/2), child 2 is (+1/2,-1/2,-1/2).
    assert tables.child_offset(0) == (-0.5, -0.5, -0.5)
    assert tables.child_offset(1) == (0.5, -0.5, -0.5)
    assert tables.child_offset(6) == (-0.5, 0.5, 0.5)
    assert sorted(tables.child_offset(c) for c in range(8)) == sorted(
        itertools.product((-0.5, 0.5), repeat=3))


def test_periodic_distance():
    # Sec. 2.1: |i|_p = i for i <= n/2, n - i above.
    assert list(tables.periodic_distance(8)) == [0, 1, 2, 3, 4, 3, 2, 1]
    assert list(tables.periodic_distance(5)) == [0, 1, 2, 2, 1]


def test_green_lattice_values():
    ng, h, eps = 2, 0.25, 0.0
    g = tables.green_lattice(ng, h, 1.0, eps)
    n = 8 * ng
    assert g.shape == (n, n, n)
    assert g[0, 0, 1] == pytest.approx(-1.0 / h)
    assert g[0, 0, n - 1] == pytest.approx(-1.0 / h)          # periodic image
    assert g[3, 4, 0] == pytest.approx(-1.0 / (5 * h))
    assert g[0, 0, 0] == g[0, 0, 1]                            # unsoftened origin convention
    assert np.allclose(g, g[::-1, :, :][np.r_[n - 1, 0:n - 1]])  # even in z
    gs = tables.green_lattice(ng, h, 2.0, 0.1)
    assert gs[0, 0, 0] == pytest.approx(-2.0 / 0.1)
    assert gs[0, 1, 1] == pytest.approx(-2.0 / np.sqrt(2 * h * h + 0.01))
