"""Hierarchical Particle-Mesh in FP64, step by step in the paper's order.

TEST INFRASTRUCTURE ONLY (parity oracle); the product never imports this module.

Steps (Sec. 1, enumerated list, and Sec. 2):
  P2M  leaf effective masses from Cartesian multipoles: Eq. (2) then Eq. (5).
  M2M  child-to-parent translation with the matrices T^C (Sec. 2.3).
  M2L  source-to-target over the 189-cube interaction zone (Sec. 2.1). Three modes:
         "direct": the definition, sum_Q sum_q g(r_p - r_q) M_q over every IZ gridlet node;
         "fft":    the method, one zero-padded (8 N_g)^3 FFT of the IZ effective masses times the
                   transform of the exact lattice Green function (Eq. 1), target gridlet read out;
         "cells":  the cell-by-cell alternative the paper compares against (Sec. 2.5): for each
                   source cube a zero-padded (2 N_g)^3 transform times the transform of the
                   Green function at that cube's offset, the products summed and transformed
                   back once.
         "shared": the transform shared by the children of one parent. Every child's zone lies
                   in the parent's 6^3 block of cubes; the 152 cubes outside the block's central
                   4^3 are in the zone of all 8 children, so one zero-padded (8 N_g)^3 transform
                   of them per parent serves every child (its window read out per child). The
                   zone's other 37 cubes (the central 4^3 minus the child's 27 near cubes) are
                   added cell by cell. The two sets partition the zone, so nothing is
                   subtracted.
  L2L  parent-to-child: potential multipoles Eq. (6), polynomial Eq. (7) at the child nodes.
  L2P  Eq. (7) at each particle, its gradient for the acceleration.

Extended gridlet (Sec. 2.5, Problem.extended): target gridlets (the M2L output and the locals of
L2L and L2P) carry N_g + 2 nodes per axis, the gridlet widened by one node on every side at the
same spacing; Eq. (6)-(7) then use that node set (polynomials of degree N_g + 1 per axis). The
sources keep N_g^3 effective masses.
  P2P  near zone (27 cubes) by direct summation (Sec. 1, item 1).

Readings (the paper is silent): the potential kernel is g(r) = -G (r^2+eps^2)^{-1/2}; expansions
are about the cell centre in units of the cell size; M2L starts at level 2 (a non-periodic root has
no neighbours, so level-1 interaction zones are empty); the far-field acceleration is minus the
analytic gradient of the Eq. (7) interpolant; the near-zone force is the exact softened force; a
particle does not act on itself. Zones are cube-complete (see tree.py).
"""
from __future__ import annotations

from dataclasses import dataclass
from functools import lru_cache

import numpy as np
import scipy.fft as sfft

from . import green, tables
from .tree import Tree


@dataclass
class Problem:
    ng: int = 4
    softening: float = 1e-3
    gconst: float = 1.0
    box_lo: tuple = (0.0, 0.0, 0.0)
    box_size: float = 1.0
    uniform_depth: int = 0
    leaf_capacity: int = 64
    max_depth: int = 10
    kernel: str = "newton"   # point-mass kernel (green.py); "yukawa" needs a screening length
    screening: float = 0.0
    extended: bool = False   # target gridlets widened by one node per side (Sec. 2.5)


# ---------------------------------------------------------------------------------------------
# Single-cell operators
# ---------------------------------------------------------------------------------------------

LD = tables.LD


def monomials(x: np.ndarray, ng: int) -> np.ndarray:
    """(k, M) array of x^n over the raveled multi-indices n (x in any units), extended precision."""
    nidx = tables.multi_index(ng)
    x = np.asarray(x, dtype=LD)
    out = np.ones((x.shape[0], nidx.shape[0]), dtype=LD)
    for ax in range(3):
        out *= x[:, ax][:, None] ** nidx[:, ax][None, :]
    return out


def p2m(rel: np.ndarray, m: np.ndarray, ng: int, L: float) -> np.ndarray:
    """Effective masses of a cell of size L from particles at offsets ``rel`` from its centre.

    Eq. (2): Q_n = (1/n!) sum_j m_j r_j^n (Cartesian multipoles about the centre);
    Eq. (5): M_p = sum_n B_pn (n!/L^n) Q_n.
    """
    nfact = tables.factorial_vector(ng, LD)
    nsum = tables.multi_index(ng).sum(axis=1)
    q = (np.asarray(m, dtype=LD) @ monomials(rel, ng)) / nfact            # Eq. (2)
    mp = tables.inverse_3d(ng, LD) @ (nfact / LD(L) ** nsum * q)          # Eq. (5)
    return mp.astype(np.float64)


def m2m(children: dict, ng: int) -> np.ndarray:
    """M^P = sum_C T^C M^C over the real children {octant: M^C} (Sec. 2.3)."""
    out = np.zeros(ng ** 3, dtype=LD)
    for c, mc in children.items():
        out += tables.child_to_parent(ng, c, LD) @ np.asarray(mc, dtype=LD)
    return out.astype(np.float64)


def potential_multipoles(phi: np.ndarray, ng: int, ext: int = 0) -> np.ndarray:
    """Eq. (6): V_n = sum_p B_pn Phi_p (extended precision), on the target gridlet's nodes."""
    return tables.inverse_3d(ng, LD, ext).T @ np.asarray(phi, dtype=LD)


@lru_cache(maxsize=None)
def _child_node_monomials(ng: int, octant: int, ext: int = 0) -> np.ndarray:
    """u^n at the child's nodes u = (a^C + x_p)/2 in parent units (geometry only, cached)."""
    a = np.asarray(tables.child_offset(octant), dtype=LD)
    u = (a[None, :] + tables.node_positions(ng, ext).astype(LD)) / LD(2)
    return monomials(u, ng + 2 * ext)


def l2l(phi_parent: np.ndarray, octant: int, ng: int, ext: int = 0) -> np.ndarray:
    """Parent contribution on a child gridlet: Phi^C_p = Phi^P((a^C + x_p)/2), Eq. (6)-(7)."""
    v = potential_multipoles(phi_parent, ng, ext)
    return (_child_node_monomials(ng, octant, ext) @ v).astype(np.float64)    # Eq. (7)


def l2p(phi: np.ndarray, rel: np.ndarray, ng: int, L: float, ext: int = 0):
    """Eq. (7) at particles (offsets ``rel`` from the cell centre) and minus its gradient.

    Returns (potential (k,), acceleration (k, 3)).
    """
    v = potential_multipoles(phi, ng, ext)
    x = np.asarray(rel, dtype=LD) / LD(L)
    npt = ng + 2 * ext
    pot = monomials(x, npt) @ v
    nidx = tables.multi_index(npt)
    acc = np.zeros((x.shape[0], 3), dtype=LD)
    for ax in range(3):
        dm = np.ones((x.shape[0], nidx.shape[0]), dtype=LD)
        for bx in range(3):
            e = nidx[:, bx]
            if bx == ax:
                dm *= e[None, :] * x[:, bx][:, None] ** np.maximum(e - 1, 0)[None, :]
            else:
                dm *= x[:, bx][:, None] ** e[None, :]
        acc[:, ax] = -(dm @ v) / LD(L)
    return pot.astype(np.float64), acc.astype(np.float64)


def pair_sum(tpos: np.ndarray, tids: np.ndarray, spos: np.ndarray, sm: np.ndarray,
             sids: np.ndarray, gconst: float, eps: float, kernel: str = "newton",
             screening: float = 0.0):
    """Direct sum of the kernel over sources on targets, skipping equal particle ids."""
    d = tpos[:, None, :] - spos[None, :, :]
    r2 = np.einsum("tsk,tsk->ts", d, d)
    same = tids[:, None] == sids[None, :]
    r2 = np.where(same, 1.0, r2)
    g = np.where(same, 0.0, green.potential(r2, gconst, eps, kernel, screening))
    c = np.where(same, 0.0, green.force_coefficient(r2, gconst, eps, kernel, screening))
    pot = (sm[None, :] * g).sum(axis=1)
    acc = -np.einsum("ts,tsk->tk", sm[None, :] * c, d)
    return pot, acc


# ---------------------------------------------------------------------------------------------
# Whole method
# ---------------------------------------------------------------------------------------------

class HPM:
    """One HPM evaluation. ``mode`` selects the M2L route: "fft" (the method), "direct" (the
    definition) or "cells" (cell-by-cell transforms)."""

    def __init__(self, x, y, z, m, prob: Problem, mode: str = "fft"):
        green.check(prob.kernel, prob.screening)
        self.prob = prob
        self.mode = mode
        pos = np.stack([np.asarray(x, np.float64), np.asarray(y, np.float64),
                        np.asarray(z, np.float64)], axis=1)
        self.tree = Tree(pos, prob.box_lo, prob.box_size, uniform_depth=prob.uniform_depth,
                         leaf_capacity=prob.leaf_capacity, max_depth=prob.max_depth)
        t = self.tree
        self.pos = pos[t.perm]
        self.m = np.asarray(m, np.float64)[t.perm]
        self.ng = prob.ng
        self.M = prob.ng ** 3
        self.ext = 1 if prob.extended else 0
        self.ne = prob.ng + 2 * self.ext     # target gridlet nodes per axis
        self.ML = self.ne ** 3
        self._virtual = {}
        self._ghat = {}
        self._shared = {}
        if mode == "shared" and self.ext:
            raise ValueError("the shared-transform route has no extended gridlet")
        self.gridlets = {}
        self.locals = {}
        self._upsweep()

    # ---- geometry helpers ------------------------------------------------------------------
    def _cube_gridlet(self, l: int, q) -> np.ndarray | None:
        """Effective masses of level-l cube position q: the real cell's, else P2M of the particles
        inside it (a part of a coarser leaf), else None (empty)."""
        t = self.tree
        ci = t.real_cell(l, q)
        if ci >= 0:
            return self.gridlets[l][ci]
        key = (l, tuple(q))
        if key not in self._virtual:
            b, e = t.cube_range(l, q)
            if e > b:
                self._virtual[key] = p2m(self.pos[b:e] - t.cube_centre(l, q), self.m[b:e],
                                         self.ng, t.cube_size(l))
            else:
                self._virtual[key] = None
        return self._virtual[key]

    # ---- step 1 + 2: P2M at leaves, M2M up the tree ------------------------------------------
    def _upsweep(self):
        t, ng = self.tree, self.ng
        for l in range(t.max_level, 1, -1):
            lev = t.levels[l]
            g = np.zeros((len(lev), self.M))
            for i in range(len(lev)):
                if lev.split[i]:
                    kids = {c: self.gridlets[l + 1][k] for c, k in enumerate(lev.children[i]) if k >= 0}
                    g[i] = m2m(kids, ng)
                else:
                    b, e = lev.pb[i], lev.pe[i]
                    g[i] = p2m(self.pos[b:e] - t.cube_centre(l, lev.coords[i]), self.m[b:e], ng,
                               t.cube_size(l))
            self.gridlets[l] = g

    # ---- step 3: source-to-target -------------------------------------------------------------
    def _ghat_level(self, l: int) -> np.ndarray:
        if l not in self._ghat:
            h = self.tree.cube_size(l) / self.ng
            glat = tables.green_lattice(self.ng, h, self.prob.gconst, self.prob.softening,
                                        self.prob.kernel, self.prob.screening)
            self._ghat[l] = sfft.rfftn(glat)
        return self._ghat[l]

    def m2l(self, l: int, coord) -> np.ndarray:
        t, ng = self.tree, self.ng
        coord = np.asarray(coord, dtype=np.int64)
        sources = []
        for q in t.interaction_positions(coord, l):
            g = self._cube_gridlet(l, q)
            if g is not None:
                sources.append((np.asarray(q), g))
        if not sources:
            return np.zeros(self.ML)
        if self.mode == "direct":
            return self._m2l_direct(l, coord, sources)
        if self.mode == "cells":
            return self._m2l_cells(l, coord, sources)
        if self.mode == "shared":
            return self._m2l_shared(l, coord, sources)
        return self._m2l_fft(l, coord, sources)

    def _green_offset(self, l: int, d: tuple) -> np.ndarray:
        """Transform of the C^3 cyclic Green array for source cube offset d (cube units), with
        C = 2 N_g + 2 ext: entry u holds g(h |d N_g - u_c|) with u_c = u for u < N_g + ext and
        u - C otherwise, so that every target-minus-source node offset of that cube pair,
        d N_g + (p - q) with -N_g - ext < p - q < N_g + ext, is stored once (no wrap-around)."""
        key = ("cells", l, d)
        if key not in self._ghat:
            ng, ext = self.ng, self.ext
            C = 2 * ng + 2 * ext
            h = self.tree.cube_size(l) / ng
            u = np.arange(C)
            uc = np.where(u < ng + ext, u, u - C).astype(np.float64)
            oz, oy, ox = np.meshgrid(d[2] * ng - uc, d[1] * ng - uc, d[0] * ng - uc, indexing="ij")
            r2 = (ox * ox + oy * oy + oz * oz) * h * h
            g = tables.green_physical(r2, self.prob.gconst, self.prob.softening, self.prob.kernel,
                                      self.prob.screening)
            self._ghat[key] = sfft.rfftn(g)
        return self._ghat[key]

    def _m2l_cells(self, l, coord, sources):
        """Cell-by-cell: sum over sources of rfft(source padded to C^3) * Ghat_d, one inverse
        transform, the target gridlet read out (target node p = -ext .. N_g - 1 + ext sits at
        cyclic index p mod C: the convolution pairs it with source node q through entry
        (p - q) mod C, whose stored offset is d N_g - (p - q))."""
        ng, ext = self.ng, self.ext
        C = 2 * ng + 2 * ext
        acc = None
        for q, g in sources:
            d = tuple(int(v) for v in (np.asarray(q) - coord))
            pad = np.zeros((C, C, C))
            pad[:ng, :ng, :ng] = g.reshape(ng, ng, ng)
            term = sfft.rfftn(pad) * self._green_offset(l, d)
            acc = term if acc is None else acc + term
        out = sfft.irfftn(acc, s=(C, C, C))
        idx = np.arange(-ext, ng + ext) % C
        return out[np.ix_(idx, idx, idx)].ravel().copy()

    def _m2l_direct(self, l, coord, sources):
        t, ng = self.tree, self.ng
        L = t.cube_size(l)
        xp = tables.node_positions(ng)
        tnodes = t.cube_centre(l, coord) + L * tables.node_positions(ng, self.ext)
        out = np.zeros(self.ML)
        for q, g in sources:
            snodes = t.cube_centre(l, q) + L * xp
            d = tnodes[:, None, :] - snodes[None, :, :]
            r2 = np.einsum("tsk,tsk->ts", d, d)
            out += tables.green_physical(r2, self.prob.gconst, self.prob.softening,
                                         self.prob.kernel, self.prob.screening) @ g
        return out

    def _m2l_fft(self, l, coord, sources):
        ng = self.ng
        n = 8 * ng
        origin = 2 * ((coord >> 1) - 1)            # lower corner cube of the 6^3 block
        grid = np.zeros((n, n, n))                 # [z, y, x]
        for q, g in sources:
            b = q - origin
            grid[b[2] * ng:(b[2] + 1) * ng, b[1] * ng:(b[1] + 1) * ng,
                 b[0] * ng:(b[0] + 1) * ng] = g.reshape(ng, ng, ng)
        pot = sfft.irfftn(sfft.rfftn(grid) * self._ghat_level(l), s=grid.shape)
        tb = coord - origin
        e = self.ext   # the extended gridlet reaches one node into the neighbouring cubes
        return pot[tb[2] * ng - e:(tb[2] + 1) * ng + e, tb[1] * ng - e:(tb[1] + 1) * ng + e,
                   tb[0] * ng - e:(tb[0] + 1) * ng + e].ravel().copy()

    def _m2l_shared(self, l, coord, sources):
        """Outer cubes of the parent's block (some block coordinate outside 1..4) through one
        padded transform per parent, cached and read out at this child's window; the central
        cubes of this child's zone cell by cell."""
        ng = self.ng
        n = 8 * ng
        origin = 2 * ((coord >> 1) - 1)
        outer, central = [], []
        for q, g in sources:
            b = np.asarray(q) - origin
            (central if np.all((b >= 1) & (b <= 4)) else outer).append((q, g))
        key = (l, tuple(int(v) for v in (coord >> 1)))
        if key not in self._shared:
            grid = np.zeros((n, n, n))
            for q, g in outer:
                b = np.asarray(q) - origin
                grid[b[2] * ng:(b[2] + 1) * ng, b[1] * ng:(b[1] + 1) * ng,
                     b[0] * ng:(b[0] + 1) * ng] = g.reshape(ng, ng, ng)
            self._shared[key] = sfft.irfftn(sfft.rfftn(grid) * self._ghat_level(l), s=grid.shape)
        pot = self._shared[key]
        tb = coord - origin
        out = pot[tb[2] * ng:(tb[2] + 1) * ng, tb[1] * ng:(tb[1] + 1) * ng,
                  tb[0] * ng:(tb[0] + 1) * ng].ravel().copy()
        if central:
            out += self._m2l_cells(l, coord, central)
        return out

    # ---- step 4: parent-to-child, level by level ------------------------------------------------
    def local(self, l: int, i: int) -> np.ndarray:
        """Gridlet potential of real cell i at level l >= 2 (from the far field only)."""
        store = self.locals.setdefault(l, {})
        if i not in store:
            lev = self.tree.levels[l]
            phi = self.m2l(l, lev.coords[i])
            if l > 2:
                par = int(lev.parent[i])
                phi = phi + l2l(self.local(l - 1, par), int(lev.keys[i] & 7), self.ng, self.ext)
            store[i] = phi
        return store[i]

    # ---- leaves: far field at particles plus near zone ---------------------------------------
    def leaf_fields(self, l: int, i: int, sel: np.ndarray):
        """Far field (Eq. 7 and its gradient, levels >= 2) and near-zone direct sum at the
        sorted slots ``sel`` of leaf i of level l. Returns (phi_far, acc_far, phi_near, acc_near)."""
        t, p = self.tree, self.prob
        lev = t.levels[l]
        if l >= 2:
            pf, af = l2p(self.local(l, i), self.pos[sel] - t.cube_centre(l, lev.coords[i]),
                         self.ng, t.cube_size(l), self.ext)
        else:
            pf, af = np.zeros(sel.size), np.zeros((sel.size, 3))
        srcs = [t.cube_range(l, q) for q in t.near_positions(lev.coords[i], l)]
        sidx = np.concatenate([np.arange(sb, se) for sb, se in srcs if se > sb])
        pn, an = pair_sum(self.pos[sel], sel, self.pos[sidx], self.m[sidx], sidx, p.gconst,
                          p.softening, p.kernel, p.screening)
        return pf, af, pn, an

    def evaluate(self, sample: np.ndarray | None = None):
        """Potential and acceleration of every particle (or of the sorted slots in ``sample``).

        Returns dict with sorted-order arrays: phi, acc, phi_far, acc_far, phi_near, acc_near,
        and ``slots`` (the sorted slots evaluated).
        """
        t = self.tree
        n = t.n
        want = np.ones(n, bool) if sample is None else np.zeros(n, bool)
        if sample is not None:
            want[np.asarray(sample)] = True
        phi_far = np.zeros(n)
        acc_far = np.zeros((n, 3))
        phi_near = np.zeros(n)
        acc_near = np.zeros((n, 3))
        for l, i in t.leaves():
            lev = t.levels[l]
            b, e = int(lev.pb[i]), int(lev.pe[i])
            sel = np.nonzero(want[b:e])[0] + b
            if sel.size == 0:
                continue
            phi_far[sel], acc_far[sel], phi_near[sel], acc_near[sel] = self.leaf_fields(l, i, sel)
        slots = np.nonzero(want)[0]
        return dict(phi=phi_far + phi_near, acc=acc_far + acc_near, phi_far=phi_far,
                    acc_far=acc_far, phi_near=phi_near, acc_near=acc_near, slots=slots)

    def all_locals(self) -> dict:
        """Gridlet potentials of every real cell at levels >= 2, as arrays per level."""
        out = {}
        for l in range(2, self.tree.max_level + 1):
            out[l] = np.stack([self.local(l, i) for i in range(len(self.tree.levels[l]))]) \
                if len(self.tree.levels[l]) else np.zeros((0, self.ML))
        return out


def solve(x, y, z, m, prob: Problem, mode: str = "fft", sample: np.ndarray | None = None):
    """Potentials and accelerations in INPUT order (all particles, or the input indices in
    ``sample``). Returns (phi, acc, hpm) where phi/acc are indexed like ``sample`` (or all)."""
    h = HPM(x, y, z, m, prob, mode)
    inv = np.empty_like(h.tree.perm)
    inv[h.tree.perm] = np.arange(h.tree.n)
    if sample is None:
        r = h.evaluate()
        return r["phi"][inv], r["acc"][inv], h
    slots = inv[np.asarray(sample)]
    r = h.evaluate(slots)
    return r["phi"][slots], r["acc"][slots], h
