"""Constant HPM tables, in FP64 (test infrastructure only; never imported by the product).

Sec. 2.2: a gridlet of N_g points per axis has nodes x_p = ((i+1/2)/N_g - 1/2, ...) in units of the
cell size, centred on the cell. The moment-matching system is the Vandermonde matrix
A_{np} = x_p^n and its inverse B = A^{-1}. Indices n and p are raveled with x fastest:
p = i + N_g (j + N_g k).

Reading of "order up to and including N_g - 1" (Sec. 2.2): the multi-index n runs over the tensor
set {0..N_g-1}^3, which is what makes A square. A is then the Kronecker product A1 x A1 x A1 of
the 1-D Vandermonde matrix, and its inverse is B1 x B1 x B1. B1 is computed exactly in rational
arithmetic (the nodes are rationals) and rounded once to float64.

Sec. 2.3: the child-to-parent matrix T^C for child offset a^C (components +-1/2 in units where
the parent spans [-1, 1]). Its defining double sum over n and m factorises over the three axes
because every term is a product of per-axis factors.

Eq. (1): the exact lattice Green function with periodic distance |i|_p.

Sec. 2.5 (extended gridlet): a target gridlet widened by one node on every side, N_g + 2 nodes
per axis at the same spacing, i.e. nodes (i + 1/2)/N_g - 1/2 for i = -1 .. N_g. The functions
below take ``ext`` = 1 for that node set (0: the gridlet of Sec. 2.2); sources always use ext = 0.
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache
from math import comb, factorial

import numpy as np

from . import green


def node_fractions(ng: int, ext: int = 0) -> list:
    """Gridlet node coordinates (i + 1/2)/N_g - 1/2, i = -ext .. N_g - 1 + ext, as exact
    rationals (Sec. 2.2; ext = 1 is the extended gridlet of Sec. 2.5)."""
    return [Fraction(2 * i + 1 - ng, 2 * ng) for i in range(-ext, ng + ext)]


def nodes(ng: int, ext: int = 0) -> np.ndarray:
    return np.array([float(f) for f in node_fractions(ng, ext)], dtype=np.float64)


def _vandermonde_exact(ng: int, ext: int = 0) -> list:
    """A1[n][p] = x_p^n with rational entries (n, p < N_g + 2 ext)."""
    xs = node_fractions(ng, ext)
    k = len(xs)
    return [[xs[p] ** n for p in range(k)] for n in range(k)]


def _invert_exact(a: list) -> list:
    """Gauss-Jordan inverse of a small non-singular rational matrix."""
    n = len(a)
    aug = [list(row) + [Fraction(int(i == j)) for j in range(n)] for i, row in enumerate(a)]
    for col in range(n):
        piv = next(r for r in range(col, n) if aug[r][col] != 0)
        aug[col], aug[piv] = aug[piv], aug[col]
        pv = aug[col][col]
        aug[col] = [v / pv for v in aug[col]]
        for r in range(n):
            if r != col and aug[r][col] != 0:
                f = aug[r][col]
                aug[r] = [vr - f * vc for vr, vc in zip(aug[r], aug[col])]
    return [row[n:] for row in aug]


# Extended precision (x86 80-bit) for the dynamic arithmetic of Eq. (2), (5), (6) and (7): the
# monomial basis is ill-conditioned at high N_g (cond(A1) = 7.3e4 at N_g = 8), so doing these
# steps literally in float64 would leave the oracle with ~1e-10 relative roundoff of its own.
LD = np.longdouble


def _to(rows, dtype):
    return np.array([[dtype(v.numerator) / dtype(v.denominator) for v in row] for row in rows],
                    dtype=dtype)


@lru_cache(maxsize=None)
def vandermonde_1d(ng: int, dtype=np.float64) -> np.ndarray:
    """A1[n, p] = x_p^n (1-D factor of A, Sec. 2.2), exact, rounded once to ``dtype``."""
    return _to(_vandermonde_exact(ng), dtype)


@lru_cache(maxsize=None)
def _inverse_1d_exact(ng: int, ext: int = 0) -> list:
    return _invert_exact(_vandermonde_exact(ng, ext))


@lru_cache(maxsize=None)
def inverse_1d(ng: int, dtype=np.float64, ext: int = 0) -> np.ndarray:
    """B1[p, n] = (A1^{-1})[p, n], exact rational inverse rounded once (Sec. 2.2)."""
    return _to(_inverse_1d_exact(ng, ext), dtype)


def kron3(ax: np.ndarray, ay: np.ndarray, az: np.ndarray) -> np.ndarray:
    """3-D matrix from per-axis factors with raveled index x + N_g (y + N_g z)."""
    return np.kron(az, np.kron(ay, ax))


@lru_cache(maxsize=None)
def vandermonde_3d(ng: int, dtype=np.float64) -> np.ndarray:
    """A[n, p] = x_p^n over multi-indices (Sec. 2.2)."""
    a1 = vandermonde_1d(ng, dtype)
    return kron3(a1, a1, a1)


@lru_cache(maxsize=None)
def inverse_3d(ng: int, dtype=np.float64, ext: int = 0) -> np.ndarray:
    """B[p, n] = A^{-1} (Sec. 2.2, the matrix of Eq. 5; of Eq. 6 for a target gridlet)."""
    b1 = inverse_1d(ng, dtype, ext)
    return kron3(b1, b1, b1)


@lru_cache(maxsize=None)
def multi_index(ng: int) -> np.ndarray:
    """(M, 3) array of (n_x, n_y, n_z) for raveled n = n_x + N_g (n_y + N_g n_z)."""
    r = np.arange(ng)
    nz, ny, nx = np.meshgrid(r, r, r, indexing="ij")
    return np.stack([nx.ravel(), ny.ravel(), nz.ravel()], axis=1)


@lru_cache(maxsize=None)
def node_positions(ng: int, ext: int = 0) -> np.ndarray:
    """((N_g + 2 ext)^3, 3) gridlet node coordinates x_p in cell units, raveled like p."""
    xs = nodes(ng, ext)
    idx = multi_index(ng + 2 * ext)
    return xs[idx]


@lru_cache(maxsize=None)
def factorial_vector(ng: int, dtype=np.float64) -> np.ndarray:
    """n! = n_x! n_y! n_z! for each raveled n."""
    f = np.array([factorial(k) for k in range(ng)], dtype=dtype)
    idx = multi_index(ng)
    return f[idx[:, 0]] * f[idx[:, 1]] * f[idx[:, 2]]


def child_offset(c: int) -> tuple:
    """a^C for child octant c = c_x + 2 c_y + 4 c_z: -1/2 or +1/2 per axis (Sec. 2.3).

    Child 1 in the paper's numbering is (-1/2,-1/2,-1/2), child 2 is (+1/2,-1/2,-1/2), i.e. the
    x component varies fastest; octant c here is the paper's child c + 1.
    """
    return tuple(0.5 if (c >> ax) & 1 else -0.5 for ax in range(3))


@lru_cache(maxsize=None)
def child_to_parent_1d(ng: int, a: float, dtype=np.float64) -> np.ndarray:
    """Per-axis factor of T^C (Sec. 2.3), summed exactly in rationals and rounded once:
    T1[p, q] = sum_n sum_{m<=n} B1[p,n] * n!/(m!(n-m)!) * a^(n-m) / 2^n * A1[m,q]."""
    b1 = _inverse_1d_exact(ng)
    a1 = _vandermonde_exact(ng)
    fa = Fraction(a).limit_denominator(2)
    rows = []
    for p in range(ng):
        row = []
        for q in range(ng):
            s = Fraction(0)
            for n in range(ng):
                for m in range(n + 1):
                    s += b1[p][n] * comb(n, m) * fa ** (n - m) / Fraction(2) ** n * a1[m][q]
            row.append(s)
        rows.append(row)
    return _to(rows, dtype)


@lru_cache(maxsize=None)
def child_to_parent(ng: int, c: int, dtype=np.float64) -> np.ndarray:
    """T^C (M x M) for child octant c: M^P_p = sum_C sum_q T^C_{pq} M^C_q (Sec. 2.3)."""
    ax, ay, az = child_offset(c)
    return kron3(child_to_parent_1d(ng, ax, dtype), child_to_parent_1d(ng, ay, dtype),
                 child_to_parent_1d(ng, az, dtype))


def periodic_distance(n: int) -> np.ndarray:
    """|i|_p for i = 0..n-1 (Sec. 2.1): i for i <= n/2, n - i above."""
    i = np.arange(n)
    return np.where(i <= n // 2, i, n - i).astype(np.float64)


def green_physical(r2: np.ndarray, gconst: float, softening: float, kernel: str = "newton",
                   screening: float = 0.0) -> np.ndarray:
    """Point-mass potential kernel g(r) (see green.py).

    The paper's Eq. (1) is the 1/(4 pi r) kernel in grid units; the method is kernel independent
    (Sec. 4). The default is gravity with Plummer softening eps (eps = 0 gives 1/r).
    """
    return green.potential(r2, gconst, softening, kernel, screening)


def green_lattice(ng: int, h: float, gconst: float, softening: float, kernel: str = "newton",
                  screening: float = 0.0) -> np.ndarray:
    """Exact lattice Green function on the (8 N_g)^3 FFT grid, indexed [z, y, x] (Eq. 1).

    G[k, j, i] = g(h * sqrt(|i|_p^2 + |j|_p^2 + |k|_p^2)) with node spacing h. The grid edge is
    8 N_g (Sec. 2.1: the largest target-to-source offset along an axis is under 4 N_g). At the
    origin, for eps = 0, the value at unit offset is used (the paper's choice for its 2-D example).
    """
    n = 8 * ng
    d = periodic_distance(n)
    dz, dy, dx = np.meshgrid(d, d, d, indexing="ij")
    r2 = (dx * dx + dy * dy + dz * dz) * (h * h)
    if softening == 0.0:
        r2[0, 0, 0] = h * h
    return green_physical(r2, gconst, softening, kernel, screening)
