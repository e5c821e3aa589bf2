#!/usr/bin/env python3
"""Writes the expected values for the sampled parity test of the large clustered workload, from
the FP64 oracle only.

Workload: 2^24 equal-mass particles, 32 Plummer spheres on a 10% uniform background (seed 1002,
synth.clustered_spheres), positions and masses rounded once to float32 (the workload's precision)
and then evaluated in FP64; adaptive tree with at most 32 particles per leaf and depth at most 10,
N_g = 4, Plummer softening 1e-3, G = 1, the padded-grid source-to-target route (Sec. 2.1). The
oracle computes:
  - potential and acceleration of 128 sampled particles (input indices, seed 3005);
  - the local gridlet potential (Eq. 6-7 chain plus source-to-target) of 24 sampled target cells
    of levels >= 2 (seed 3006), identified by level and integer coordinates;
  - the number of cells per level (the tree both sides must build).

  python tests/golden/make_clustered2p24.py   # writes tests/golden/clustered2p24_ng4_f32.npz
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import hpm as ohpm  # noqa: E402
from synth import clustered_spheres, random_subset  # noqa: E402

N = 2 ** 24
N_SAMPLE = 128
N_CELLS = 24


def make():
    t0 = time.perf_counter()
    p = clustered_spheres(N, 1002).astype(np.float32)
    sample = random_subset(N, N_SAMPLE, 3005)
    print(f"particles drawn: {time.perf_counter() - t0:.1f} s", flush=True)
    phi, acc, h = ohpm.solve(p.x, p.y, p.z, p.m,
                             ohpm.Problem(ng=4, softening=1e-3, leaf_capacity=32, max_depth=10),
                             mode="fft", sample=sample)
    print(f"sampled solve: {time.perf_counter() - t0:.1f} s", flush=True)
    t = h.tree
    counts = [len(t.levels[l]) for l in range(2, t.max_level + 1)]
    rng = np.random.default_rng(3006)
    pick = []
    for k in np.sort(rng.choice(sum(counts), size=N_CELLS, replace=False)):
        l = 2
        while k >= counts[l - 2]:
            k -= counts[l - 2]
            l += 1
        pick.append((l, int(k)))
    cell_level = np.array([l for l, _ in pick], np.int32)
    cell_coord = np.array([t.levels[l].coords[i] for l, i in pick], np.int32).reshape(-1, 3)
    cell_local = np.stack([h.local(l, i) for l, i in pick])
    out = os.path.join(HERE, "clustered2p24_ng4_f32.npz")
    np.savez(out, sample=sample, phi=phi, acc=acc, cell_level=cell_level, cell_coord=cell_coord,
             cell_local=cell_local, n_targets=np.int64(sum(counts)),
             cells_per_level=np.array([len(lv) for lv in t.levels], np.int64))
    print(f"{out}: {time.perf_counter() - t0:.1f} s, {sum(counts)} targets", flush=True)


if __name__ == "__main__":
    make()
