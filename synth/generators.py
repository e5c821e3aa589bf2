"""Seeded particle generators (positions in a cubic box, masses).

All draws use numpy's PCG64 bit generator with an explicit integer seed and are made in float64.
A caller that runs a single-precision path rounds the positions once (``Particles.astype``) and
hands the rounded values to every consumer, so that the oracle and the GPU see the same input.

Distributions follow the workloads the method is meant for: a uniform cube, a truncated Plummer
sphere, and a superposition of Plummer spheres on a uniform background. Two structured sets serve
as exact checks: particles placed on gridlet nodes (the case in which the effective masses equal
the particle masses) and a single point mass surrounded by massless tracers (the accuracy test of
the paper's Sec. 3.2).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Particles:
    """Structure-of-arrays particle set. ``x, y, z, m`` are 1-D arrays of one dtype."""

    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    m: np.ndarray
    box_lo: tuple = (0.0, 0.0, 0.0)
    box_size: float = 1.0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def astype(self, dtype) -> "Particles":
        """Round once to ``dtype`` (float32 or float64); the result is what every consumer uses."""
        cast = lambda a: np.ascontiguousarray(a, dtype=dtype)  # noqa: E731
        return Particles(cast(self.x), cast(self.y), cast(self.z), cast(self.m),
                         self.box_lo, self.box_size, dict(self.meta))

    def as_f64(self) -> "Particles":
        return self.astype(np.float64)

    def positions(self) -> np.ndarray:
        return np.stack([self.x, self.y, self.z], axis=1)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _pack(pos: np.ndarray, m: np.ndarray, **meta) -> Particles:
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    return Particles(pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(),
                     np.ascontiguousarray(m, dtype=np.float64), meta=meta)


def uniform_cube(n: int, seed: int) -> Particles:
    """``n`` particles uniform in [0,1)^3 with equal masses 1/n."""
    rng = _rng(seed)
    pos = rng.random((n, 3))
    return _pack(pos, np.full(n, 1.0 / n), kind="uniform", seed=seed)


def _plummer_offsets(rng: np.random.Generator, n: int, a: float, r_t: float) -> np.ndarray:
    """Offsets from the centre of a Plummer sphere of scale radius ``a`` truncated at ``r_t``.

    The enclosed-mass fraction of a Plummer sphere is u = (r^2/(r^2+a^2))^{3/2}; drawing u uniform
    in (0, u(r_t)) and inverting, r = a (u^{-2/3} - 1)^{-1/2}, samples the truncated profile.
    Directions are isotropic.
    """
    u_t = (r_t * r_t / (r_t * r_t + a * a)) ** 1.5
    u = rng.random(n) * u_t
    u = np.maximum(u, 1e-300)
    r = a / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
    mu = rng.random(n) * 2.0 - 1.0
    ph = rng.random(n) * (2.0 * np.pi)
    s = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    return np.stack([r * s * np.cos(ph), r * s * np.sin(ph), r * mu], axis=1)


def plummer_sphere(n: int, seed: int, a: float = 0.05, r_t: float = 0.5,
                   centre=(0.5, 0.5, 0.5)) -> Particles:
    """``n`` equal-mass particles from a Plummer sphere (scale ``a``, truncated at ``r_t``)."""
    rng = _rng(seed)
    pos = _plummer_offsets(rng, n, a, r_t) + np.asarray(centre, dtype=np.float64)
    pos = np.clip(pos, 0.0, np.nextafter(1.0, 0.0))
    return _pack(pos, np.full(n, 1.0 / n), kind="plummer", seed=seed, a=a, r_t=r_t)


def clustered_spheres(n: int, seed: int, n_spheres: int = 32, a_range=(0.005, 0.05),
                      weight_range=(1.0, 10.0), background: float = 0.10,
                      r_t: float = 0.5) -> Particles:
    """Superposition of Plummer spheres on a uniform background, equal particle masses 1/n.

    Scale radii are log-uniform in ``a_range``, centres uniform in the unit cube, and the sphere
    weights are log-uniform over ``weight_range``. A fraction ``background`` of the particles is
    uniform; the rest is split among the spheres in proportion to their weights. Samples that fall
    outside the box are drawn again.
    """
    rng = _rng(seed)
    a_k = np.exp(rng.uniform(np.log(a_range[0]), np.log(a_range[1]), n_spheres))
    c_k = rng.random((n_spheres, 3))
    w_k = np.exp(rng.uniform(np.log(weight_range[0]), np.log(weight_range[1]), n_spheres))
    n_bg = int(round(background * n))
    counts = rng.multinomial(n - n_bg, w_k / w_k.sum())
    parts = [rng.random((n_bg, 3))]
    for k in range(n_spheres):
        need = int(counts[k])
        got = []
        while need > 0:
            p = _plummer_offsets(rng, need, a_k[k], r_t) + c_k[k]
            ok = np.all((p >= 0.0) & (p < 1.0), axis=1)
            got.append(p[ok])
            need -= int(ok.sum())
        if got:
            parts.append(np.concatenate(got))
    pos = np.concatenate(parts)
    pos = pos[rng.permutation(pos.shape[0])]
    return _pack(pos, np.full(n, 1.0 / n), kind="clustered", seed=seed)


def gridlet_node_lattice(ng: int, level: int, seed: int, mass_scale: float = 1.0) -> Particles:
    """One particle on every gridlet node of every cell of a uniform level ``level`` mesh.

    Node k of a cell of size L sits at (k + 1/2) L / ng from the cell's lower corner (Sec. 2.2).
    Masses are drawn uniform in [0.5, 1.5) times ``mass_scale`` / count so that an index mix-up
    shows in the result. There are (2^level * ng)^3 particles, in x-fastest lattice order.
    """
    rng = _rng(seed)
    k = 2 ** level * ng
    idx = np.arange(k, dtype=np.float64)
    pos1 = (idx + 0.5) / k  # (cell*ng + node + 1/2) / (2^level ng)
    zz, yy, xx = np.meshgrid(pos1, pos1, pos1, indexing="ij")
    pos = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    m = rng.uniform(0.5, 1.5, pos.shape[0]) * (mass_scale / pos.shape[0])
    return _pack(pos, m, kind="gridlet_nodes", seed=seed, ng=ng, level=level)


def point_source_with_tracers(source=(0.8, 0.8, 0.8), mass: float = 1.0, tracers_per_axis: int = 16,
                              seed: int = 0, jitter: float = 0.5) -> Particles:
    """A unit point mass plus massless tracers on a jittered lattice filling the box.

    The first particle is the source; the tracers (mass 0) feel only its field, whose exact value
    is -G m / sqrt(r^2 + eps^2).
    """
    rng = _rng(seed)
    k = tracers_per_axis
    idx = np.arange(k, dtype=np.float64)
    zz, yy, xx = np.meshgrid(idx, idx, idx, indexing="ij")
    lat = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    pos = (lat + 0.5 + jitter * (rng.random(lat.shape) - 0.5)) / k
    pos = np.concatenate([np.asarray(source, dtype=np.float64)[None, :], pos])
    m = np.zeros(pos.shape[0])
    m[0] = mass
    return _pack(pos, m, kind="point_source", seed=seed)


def random_subset(n: int, k: int, seed: int) -> np.ndarray:
    """Sorted indices of ``k`` distinct particles out of ``n`` (seeded)."""
    rng = _rng(seed)
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False))


# Workloads of the method's evaluation, each with its particle set, tree rule and gridlet order.
# The seeds are 1000 + the workload's index.
WORKLOADS = {
    "uniform4096_depth3": dict(n=4096, gen="uniform", seed=1000, uniform_depth=3, ng=4,
                               softening=1e-3, precision="f64"),
    "plummer2p18_cap64": dict(n=2 ** 18, gen="plummer", seed=1001, leaf_capacity=64,
                              max_depth=10, ng=4, softening=1e-3, precision="f32",
                              error_subset=4096, error_seed=2002),
    "clustered2p24_cap32": dict(n=2 ** 24, gen="clustered", seed=1002, leaf_capacity=32,
                                max_depth=10, ng=4, softening=1e-3, precision="f32"),
}


def workload(name: str, n: int | None = None) -> Particles:
    """Particle set of a named workload (optionally with a different count ``n``)."""
    w = WORKLOADS[name]
    count = w["n"] if n is None else int(n)
    gen = {"uniform": uniform_cube, "plummer": plummer_sphere, "clustered": clustered_spheres}[w["gen"]]
    return gen(count, w["seed"])


# Mixes of independent solves. Each request is described by its particle count, distribution and
# seed; request_particles draws its set.
def batch_requests(count: int = 512, seed: int = 1003) -> list[dict]:
    """The batched workload: ``count`` solves with N log-uniform in [2^10, 2^18] (rounded), even
    indices a uniform cube and odd ones a Plummer sphere (as the 2^18 workload), gridlet order 4
    or 6 by a seeded coin."""
    rng = _rng(seed)
    n = np.rint(2.0 ** rng.uniform(10.0, 18.0, count)).astype(np.int64)
    ng = np.where(rng.random(count) < 0.5, 4, 6)
    return [dict(n=int(n[i]), kind="uniform" if i % 2 == 0 else "plummer", ng=int(ng[i]),
                 seed=seed * 1000 + i) for i in range(count)]


def serve_requests(count: int, seed: int = 1004) -> list[dict]:
    """The served workload's request pool: N log-uniform in [2^12, 2^20] (rounded); uniform cube,
    Plummer sphere or clustered set (8 spheres on a 10% background) with equal odds; a relative
    force tolerance of 1e-4 for every request."""
    rng = _rng(seed)
    n = np.rint(2.0 ** rng.uniform(12.0, 20.0, count)).astype(np.int64)
    kind = rng.integers(0, 3, count)
    names = ("uniform", "plummer", "clustered")
    return [dict(n=int(n[i]), kind=names[int(kind[i])], tolerance=1e-4, seed=seed * 1000 + i)
            for i in range(count)]


def request_particles(req: dict) -> Particles:
    """Particle set of one request of batch_requests or serve_requests."""
    if req["kind"] == "uniform":
        return uniform_cube(req["n"], req["seed"])
    if req["kind"] == "plummer":
        return plummer_sphere(req["n"], req["seed"])
    return clustered_spheres(req["n"], req["seed"], n_spheres=8)
