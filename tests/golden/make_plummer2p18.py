#!/usr/bin/env python3
"""Writes the expected values for the full-size Plummer parity tests, from the FP64 oracle only.

Workload: 2^18 equal-mass particles from a Plummer sphere (scale radius 0.05, truncated at 0.5,
centred in the unit box, seed 1001), adaptive tree with at most 64 particles per leaf and depth
at most 10, Plummer softening 1e-3, G = 1. For each gridlet order and input precision (the
positions and masses rounded once to float32 or kept in float64, then evaluated in FP64), the
oracle computes:
  - potential and acceleration of 256 sampled particles (input indices, seed 3003);
  - the local gridlet potential (far field, Eq. 6-7 chain plus source-to-target) of 48 sampled
    target cells of levels >= 2 (seed 3004), identified by level and integer coordinates.
The same with extended target gridlets (N_g + 2 nodes per axis, Sec. 2.5) goes to the "_ext"
files.

  python tests/golden/make_plummer2p18.py   # writes tests/golden/plummer2p18_ng{4,6}[_ext]_{f32,f64}.npz
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
from synth import plummer_sphere, random_subset  # noqa: E402

N = 2 ** 18
N_SAMPLE = 256
N_CELLS = 48
KW = dict(leaf_capacity=64, max_depth=10)
EPS = 1e-3


def make(ng: int, prec: str, extended: bool = False):
    p = plummer_sphere(N, 1001).astype(np.float32 if prec == "f32" else np.float64)
    sample = random_subset(N, N_SAMPLE, 3003)
    t0 = time.perf_counter()
    phi, acc, h = ohpm.solve(p.x, p.y, p.z, p.m,
                             ohpm.Problem(ng=ng, softening=EPS, extended=extended, **KW),
                             mode="fft", sample=sample)
    t = h.tree
    cand = [(l, i) for l in range(2, t.max_level + 1) for i in range(len(t.levels[l]))]
    rng = np.random.default_rng(3004)
    pick = [cand[k] for k in np.sort(rng.choice(len(cand), size=min(N_CELLS, len(cand)),
                                                replace=False))]
    cell_level = np.array([l for l, _ in pick], np.int32)
    cell_coord = np.array([t.levels[l].coords[i] for l, i in pick], np.int32).reshape(-1, 3)
    cell_local = np.stack([h.local(l, i) for l, i in pick])
    out = os.path.join(HERE, f"plummer2p18_ng{ng}{'_ext' if extended else ''}_{prec}.npz")
    np.savez(out, sample=sample, phi=phi, acc=acc, cell_level=cell_level, cell_coord=cell_coord,
             cell_local=cell_local, n_targets=np.int64(len(cand)),
             cells_per_level=np.array([len(lv) for lv in t.levels], np.int64))
    print(f"{out}: {time.perf_counter() - t0:.1f} s, {len(cand)} targets", flush=True)


if __name__ == "__main__":
    for extended in (False, True):
        for ng in (4, 6):
            for prec in ("f32", "f64"):
                make(ng, prec, extended)
