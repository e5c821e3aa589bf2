"""Oct-tree rule and zone geometry (test infrastructure only; never imported by the product).

Sec. 1: the cubic root (level 0) is split into 8 children, recursively; the tree need not have
uniform depth. The near zone of a cell is the cells touching it (27 with itself); its interaction
zone (IZ) is the children of its parent's near zone that are not in its own near zone,
6^3 - 3^3 = 189 cells for an interior cell.

Readings where the paper is silent:
  * Cells are half-open, located by floor(2^D (x - lo) / size) in float64, computed as
    (x - lo) * (2^D / size); a coordinate equal to the upper face is clamped into the last cell.
  * Adaptive rule: a cell at level l is split while it holds more than ``leaf_capacity``
    particles and l < ``max_depth``; uniform rule: split while l < ``uniform_depth``. Empty
    children are not created.
  * Particles are ordered by a Morton key (bit 3b = bit b of the x index, 3b+1 of y, 3b+2 of z),
    ties broken by input index (stable sort); every cube's particles are then contiguous.
  * Cube-complete zones: near zone and IZ are sets of cube *positions* at the target's level. A
    position without a real cell but with particles (part of a coarser leaf) contributes through
    the particles inside it; an empty position contributes nothing. Summed over a leaf's chain of
    ancestors this partitions the box exactly.
"""
from __future__ import annotations

import numpy as np


class OutOfBox(ValueError):
    pass


def morton_key(ix: np.ndarray, iy: np.ndarray, iz: np.ndarray, bits: int) -> np.ndarray:
    """Interleave the low ``bits`` bits of the three integer coordinates (x lowest)."""
    ix = np.asarray(ix, dtype=np.int64)
    iy = np.asarray(iy, dtype=np.int64)
    iz = np.asarray(iz, dtype=np.int64)
    key = np.zeros(np.broadcast(ix, iy, iz).shape, dtype=np.int64)
    for b in range(bits):
        key |= ((ix >> b) & 1) << (3 * b)
        key |= ((iy >> b) & 1) << (3 * b + 1)
        key |= ((iz >> b) & 1) << (3 * b + 2)
    return key


def cell_index(pos: np.ndarray, box_lo, box_size: float, depth: int) -> np.ndarray:
    """Integer cube coordinates at level ``depth`` for (N, 3) float64 positions."""
    lo = np.asarray(box_lo, dtype=np.float64)
    if not np.all(np.isfinite(pos)):
        raise OutOfBox("non-finite position")
    if np.any(pos < lo) or np.any(pos > lo + box_size):
        raise OutOfBox("position outside the box")
    scale = float(2 ** depth) / float(box_size)
    t = np.floor((pos - lo) * scale).astype(np.int64)
    return np.clip(t, 0, 2 ** depth - 1)


class Level:
    """Real cells of one level, in Morton order."""

    def __init__(self, level, coords, keys, pb, pe):
        self.level = level
        self.coords = coords          # (n, 3) int64 cube coordinates at this level
        self.keys = keys              # (n,) int64 Morton keys at this level
        self.pb = pb                  # first particle (sorted order)
        self.pe = pe                  # one past the last particle
        self.split = np.zeros(len(keys), dtype=bool)
        self.parent = np.full(len(keys), -1, dtype=np.int64)
        self.children = np.full((len(keys), 8), -1, dtype=np.int64)

    def __len__(self):
        return len(self.keys)

    def find(self, keys: np.ndarray) -> np.ndarray:
        """Cell index of each Morton key at this level, -1 where no real cell exists."""
        keys = np.asarray(keys, dtype=np.int64)
        i = np.searchsorted(self.keys, keys)
        i = np.minimum(i, len(self.keys) - 1)
        ok = self.keys[i] == keys if len(self.keys) else np.zeros(keys.shape, bool)
        return np.where(ok, i, -1)


class Tree:
    def __init__(self, pos: np.ndarray, box_lo=(0.0, 0.0, 0.0), box_size: float = 1.0, *,
                 uniform_depth: int = 0, leaf_capacity: int = 64, max_depth: int = 10):
        pos = np.ascontiguousarray(pos, dtype=np.float64)
        self.n = pos.shape[0]
        self.box_lo = np.asarray(box_lo, dtype=np.float64)
        self.box_size = float(box_size)
        self.uniform = uniform_depth > 0
        self.depth = int(uniform_depth if self.uniform else max_depth)
        self.leaf_capacity = int(leaf_capacity)
        D = self.depth
        ijk = cell_index(pos, self.box_lo, self.box_size, D)
        key = morton_key(ijk[:, 0], ijk[:, 1], ijk[:, 2], D)
        self.perm = np.argsort(key, kind="stable")       # sorted slot -> input index
        self.keys = key[self.perm]                        # depth-D keys, sorted
        self.ijk = ijk[self.perm]                         # depth-D coordinates, sorted
        self.levels: list[Level] = []
        active = np.ones(self.n, dtype=bool)
        prev_cell = None
        for l in range(D + 1):
            shift = D - l
            idx = np.nonzero(active)[0]
            if idx.size == 0:
                break
            pref = self.keys[idx] >> (3 * shift)
            head = np.ones(idx.size, dtype=bool)
            head[1:] = pref[1:] != pref[:-1]
            hpos = np.nonzero(head)[0]
            pb = idx[hpos]
            last = np.append(hpos[1:] - 1, idx.size - 1)
            pe = idx[last] + 1
            coords = self.ijk[pb] >> shift
            lev = Level(l, coords, pref[hpos], pb, pe)
            count = pe - pb
            if self.uniform:
                lev.split[:] = l < D
            else:
                lev.split[:] = (count > self.leaf_capacity) & (l < D)
            cell_of = np.repeat(np.arange(len(pb)), count)   # per active particle
            if prev_cell is not None:
                up = self.levels[l - 1]
                par = prev_cell[pb]
                lev.parent[:] = par
                up.children[par, lev.keys & 7] = np.arange(len(pb))
            full_cell = np.full(self.n, -1, dtype=np.int64)
            full_cell[idx] = cell_of
            prev_cell = full_cell
            self.levels.append(lev)
            active = np.zeros(self.n, dtype=bool)
            keep = lev.split[cell_of]
            active[idx[keep]] = True
        self._prefix = {}

    # ---- cube geometry -------------------------------------------------------------------
    @property
    def max_level(self) -> int:
        return len(self.levels) - 1

    def cube_size(self, l: int) -> float:
        return self.box_size / (2 ** l)

    def cube_centre(self, l: int, coord) -> np.ndarray:
        return self.box_lo + (np.asarray(coord, dtype=np.float64) + 0.5) * self.cube_size(l)

    def prefix(self, l: int) -> np.ndarray:
        if l not in self._prefix:
            self._prefix[l] = self.keys >> (3 * (self.depth - l))
        return self._prefix[l]

    @staticmethod
    def _key(coord, l: int) -> int:
        """Morton key of a level-l cube (plain Python ints; same bit order as morton_key)."""
        x, y, z = (int(v) for v in coord)
        k = 0
        for b in range(l):
            k |= ((x >> b) & 1) << (3 * b) | ((y >> b) & 1) << (3 * b + 1) | ((z >> b) & 1) << (3 * b + 2)
        return k

    def cube_range(self, l: int, coord) -> tuple:
        """[b, e) in sorted order of all particles inside level-l cube ``coord`` (any position)."""
        x, y, z = (int(v) for v in coord)
        side = 1 << l
        if not (0 <= x < side and 0 <= y < side and 0 <= z < side):
            return (0, 0)
        k = self._key((x, y, z), l)
        p = self.prefix(l)
        return (int(np.searchsorted(p, k, "left")), int(np.searchsorted(p, k, "right")))

    def real_cell(self, l: int, coord) -> int:
        """Index of the real cell at level-l position ``coord``, or -1."""
        if l > self.max_level:
            return -1
        if not hasattr(self, "_lookup"):
            self._lookup = [dict(zip(map(tuple, lev.coords.tolist()), range(len(lev))))
                            for lev in self.levels]
        return self._lookup[l].get(tuple(int(v) for v in coord), -1)

    @staticmethod
    def near_positions(coord, l: int) -> list:
        """The up to 27 level-l cube positions within one cube of ``coord`` (itself included)."""
        x, y, z = (int(v) for v in coord)
        side = 1 << l
        return [(x + dx, y + dy, z + dz)
                for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                if 0 <= x + dx < side and 0 <= y + dy < side and 0 <= z + dz < side]

    @staticmethod
    def interaction_positions(coord, l: int) -> list:
        """IZ positions of a level-l target: children of the parent's near zone, minus the
        target's own near zone, inside the box (Sec. 1; 189 for an interior target)."""
        x, y, z = (int(v) for v in coord)
        side = 1 << l
        out = []
        for qz in range(2 * ((z >> 1) - 1), 2 * ((z >> 1) + 1) + 2):
            for qy in range(2 * ((y >> 1) - 1), 2 * ((y >> 1) + 1) + 2):
                for qx in range(2 * ((x >> 1) - 1), 2 * ((x >> 1) + 1) + 2):
                    if not (0 <= qx < side and 0 <= qy < side and 0 <= qz < side):
                        continue
                    if abs(qx - x) <= 1 and abs(qy - y) <= 1 and abs(qz - z) <= 1:
                        continue
                    out.append((qx, qy, qz))
        return out

    def leaves(self):
        """(level, cell index) of every leaf."""
        for l, lev in enumerate(self.levels):
            for i in np.nonzero(~lev.split)[0]:
                yield l, int(i)
