"""Point-mass interaction kernels of the oracle (test infrastructure only).

The method is kernel independent (Abstract; Sec. 4): the FFT in the source-to-target step only
computes a convolution, so any Green function can stand in for Eq. (1). Each kernel here is a
potential g(r) of a unit point mass, written with the softened distance s = (r^2 + eps^2)^{1/2}:

  "newton":  g = -G / s                       (eps = 0: the bare 1/r kernel of Eq. 1)
  "yukawa":  g = -G exp(-s / lam) / s         (screened; lam > 0 is the screening length)

and the pair acceleration of target i by source j is -m_j c(r) (r_i - r_j) with
c = -(1/r) dg/dr, i.e.

  "newton":  c = G / s^3
  "yukawa":  c = G exp(-s / lam) (1 / (lam s^2) + 1 / s^3)
"""
from __future__ import annotations

import numpy as np

KERNELS = ("newton", "yukawa")


def check(kernel: str, screening: float) -> None:
    if kernel not in KERNELS:
        raise ValueError(f"unknown kernel {kernel!r}")
    if kernel == "yukawa" and not screening > 0.0:
        raise ValueError("the yukawa kernel needs a screening length > 0")


def potential(r2: np.ndarray, gconst: float, softening: float, kernel: str = "newton",
              screening: float = 0.0) -> np.ndarray:
    """g at squared distance r2 (array), for a unit mass."""
    s = np.sqrt(r2 + softening * softening)
    if kernel == "newton":
        return -gconst / s
    if kernel == "yukawa":
        return -gconst * np.exp(-s / screening) / s
    raise ValueError(f"unknown kernel {kernel!r}")


def force_coefficient(r2: np.ndarray, gconst: float, softening: float, kernel: str = "newton",
                      screening: float = 0.0) -> np.ndarray:
    """c with a_i = -sum_j m_j c (r_i - r_j), for squared distance r2."""
    s2 = r2 + softening * softening
    s = np.sqrt(s2)
    if kernel == "newton":
        return gconst / (s2 * s)
    if kernel == "yukawa":
        return gconst * np.exp(-s / screening) * (1.0 / (screening * s2) + 1.0 / (s2 * s))
    raise ValueError(f"unknown kernel {kernel!r}")
