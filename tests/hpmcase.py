"""Shared helpers of the GPU parity tests: seeded cases, device upload, oracle runs (cached)."""
from __future__ import annotations

import functools
import sys

import numpy as np

from oracle import hpm as ohpm
from synth import (gridlet_node_lattice, plummer_sphere, point_source_with_tracers,
                   uniform_cube, clustered_spheres)


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


CASES = {
    # name: (generator, tree/problem keywords)
    "uniform4096_d3": (lambda: uniform_cube(4096, 1000), dict(uniform_depth=3)),
    "lattice_d2": (lambda: gridlet_node_lattice(4, 2, seed=7), dict(uniform_depth=2)),
    "plummer3000_cap16": (lambda: plummer_sphere(3000, 11, a=0.08), dict(leaf_capacity=16, max_depth=7)),
    "plummer3000_cap64": (lambda: plummer_sphere(3000, 14, a=0.08), dict(leaf_capacity=64, max_depth=10)),
    "plummer1000_cap1": (lambda: plummer_sphere(1000, 12, a=0.2), dict(leaf_capacity=1, max_depth=10)),
    "clustered5000_cap8": (lambda: clustered_spheres(5000, 13, n_spheres=6), dict(leaf_capacity=8, max_depth=8)),
    "point_source": (lambda: point_source_with_tracers(tracers_per_axis=10, seed=3), dict(uniform_depth=3)),
}


@functools.lru_cache(maxsize=None)
def particles(name: str, prec: str):
    gen, kw = CASES[name]
    p = gen().astype(np.float32 if prec == "f32" else np.float64)
    return p, kw


@functools.lru_cache(maxsize=None)
def oracle(name: str, prec: str, ng: int, eps: float = 1e-3, kernel: str = "newton",
           screening: float = 0.0, mode: str = "fft", extended: bool = False):
    """Oracle HPM on the same (rounded) inputs: (hpm object, phi, acc) in input order. ``mode``
    is the oracle's source-to-target route ("fft": the padded grid, "cells": cell by cell)."""
    p, kw = particles(name, prec)
    prob = ohpm.Problem(ng=ng, softening=eps, kernel=kernel, screening=screening,
                        extended=extended, **kw)
    phi, acc, h = ohpm.solve(p.x, p.y, p.z, p.m, prob, mode=mode)
    return h, phi, acc


def device(p, torch):
    dt = torch.float32 if p.x.dtype == np.float32 else torch.float64
    return [torch.tensor(a, dtype=dt, device="cuda") for a in (p.x, p.y, p.z, p.m)]


def gpu_problem(ng: int, prec: str, kw: dict, eps: float = 1e-3, kernel: str = "newton",
                screening: float = 0.0, m2l: str = "grid", extended: bool = False):
    from paper_1906_10734_amd import hpm
    return hpm.Problem(ng=ng, precision=prec, softening=eps, kernel=kernel, screening=screening,
                       m2l=m2l, extended=extended,
                       uniform_depth=kw.get("uniform_depth", 0),
                       leaf_capacity=kw.get("leaf_capacity", 64),
                       max_depth=kw.get("max_depth", 10))


def rel_rms(a, b) -> float:
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.sqrt(np.sum((a - b) ** 2) / max(np.sum(b * b), 1e-300)))


def rel_max(a, b) -> float:
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def rel_each_max(a, b, floor: float = 1e-3) -> float:
    """Largest per-particle relative error max_i |a_i - b_i| / max(|b_i|, floor * rms|b|) (rows
    of a 2-D array are vectors); the floor keeps particles where the field nearly cancels from
    dividing by a value far below the field's scale."""
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    if a.ndim == 1:
        a, b = a[:, None], b[:, None]
    d = np.linalg.norm(a - b, axis=1)
    r = np.linalg.norm(b, axis=1)
    scale = np.sqrt(np.mean(r * r))
    return float(np.max(d / np.maximum(r, floor * max(scale, 1e-300))))
