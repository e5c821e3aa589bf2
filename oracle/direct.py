"""O(N^2) direct sum, the force-error reference (test infrastructure only).

phi_i = sum_{j != i} m_j g(r_ij) and a_i = -sum_{j != i} m_j c(r_ij) (r_i - r_j) with the kernel's
potential g and force coefficient c (green.py); for the default kernel
phi_i = -G sum_{j != i} m_j (r_ij^2 + eps^2)^{-1/2},
a_i   = -G sum_{j != i} m_j (r_i - r_j) (r_ij^2 + eps^2)^{-3/2}.
"""
from __future__ import annotations

import numpy as np

from . import green


def direct_sum(x, y, z, m, gconst: float = 1.0, softening: float = 0.0,
               targets: np.ndarray | None = None, chunk_pairs: int = 1 << 22,
               kernel: str = "newton", screening: float = 0.0):
    """Potential and acceleration at ``targets`` (input indices; all particles if None)."""
    pos = np.stack([np.asarray(x, np.float64), np.asarray(y, np.float64),
                    np.asarray(z, np.float64)], axis=1)
    m = np.asarray(m, np.float64)
    n = pos.shape[0]
    tgt = np.arange(n) if targets is None else np.asarray(targets)
    phi = np.zeros(tgt.size)
    acc = np.zeros((tgt.size, 3))
    step = max(1, chunk_pairs // max(n, 1))
    green.check(kernel, screening)
    for s in range(0, tgt.size, step):
        t = tgt[s:s + step]
        d = pos[t][:, None, :] - pos[None, :, :]
        r2 = np.einsum("tsk,tsk->ts", d, d)
        self_mask = t[:, None] == np.arange(n)[None, :]
        r2 = np.where(self_mask, 1.0, r2)
        g = np.where(self_mask, 0.0, green.potential(r2, gconst, softening, kernel, screening))
        c = np.where(self_mask, 0.0, green.force_coefficient(r2, gconst, softening, kernel, screening))
        phi[s:s + step] = (m[None, :] * g).sum(axis=1)
        acc[s:s + step] = -np.einsum("ts,tsk->tk", m[None, :] * c, d)
    return phi, acc


def force_error(acc: np.ndarray, acc_ref: np.ndarray):
    """Relative acceleration error e_i = |a_i - a_i^ref| / |a_i^ref|; returns (rms, max)."""
    num = np.linalg.norm(acc - acc_ref, axis=1)
    den = np.linalg.norm(acc_ref, axis=1)
    e = num / np.where(den > 0, den, 1.0)
    return float(np.sqrt(np.mean(e * e))), float(np.max(e))


def potential_error(phi: np.ndarray, phi_ref: np.ndarray) -> float:
    """Relative RMS potential difference sqrt(sum (phi - ref)^2 / sum ref^2)."""
    return float(np.sqrt(np.sum((phi - phi_ref) ** 2) / np.sum(phi_ref ** 2)))
