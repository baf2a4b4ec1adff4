"""qGGMRF prior value and gradient (FP64 numpy) — test infrastructure only.

Sec. 3, eqs. "reg2" and "reg3": for every voxel ``m`` of the 3D grid and
every neighbour ``n`` with ``||m - n||_inf <= 1`` (the 26-neighbourhood),

    g_m    = sum_n w_mn h_mn
    h_mn   = (|f_m - f_n|/sigma)^2 / (c + (|f_m - f_n|/sigma)^(2-p))

and the prior is ``H(f) = lambda * sum_m g_m``.  Readings used here:

* the exponent ``q`` of the generalised Gaussian is the literal 2 of the
  numerator;
* ``w_mn`` is inversely proportional to the distance ``||m - n||_2`` and the
  26 weights sum to one (face, edge and corner values below); the
  "Gaussian" alternative is one argument away;
* neighbours outside the volume are dropped and the weights are not
  renormalised at the faces;
* ``lambda`` scales the whole prior (the paper gives no weight between the
  two terms of eq. "objfn").

Writing ``rho(u) = u^2 / (c + |u|^(2-p))``, ``H`` sums ``rho`` over ordered
pairs, so each unordered pair appears twice and, ``rho'`` being odd,

    dH/df_m = (2 lambda / sigma) * sum_n w_mn rho'((f_m - f_n)/sigma)
    rho'(u) = u (2c + p|u|^(2-p)) / (c + |u|^(2-p))^2 .
"""

from __future__ import annotations

import itertools

import numpy as np

OFFSETS = [d for d in itertools.product((-1, 0, 1), repeat=3) if d != (0, 0, 0)]


def inverse_distance_weights() -> dict[int, float]:
    """Weights by squared distance (1 face, 2 edge, 3 corner), proportional to 1/d, summing to 1."""
    total = 6 / 1.0 + 12 / np.sqrt(2.0) + 8 / np.sqrt(3.0)
    return {1: 1.0 / total, 2: (1.0 / np.sqrt(2.0)) / total, 3: (1.0 / np.sqrt(3.0)) / total}


def gaussian_weights() -> dict[int, float]:
    """Alternative reading: ``exp(-d^2/2)`` normalised over the 26 neighbours."""
    e = {k: np.exp(-k / 2.0) for k in (1, 2, 3)}
    total = 6 * e[1] + 12 * e[2] + 8 * e[3]
    return {k: v / total for k, v in e.items()}


def rho(u: np.ndarray, p: float, c: float) -> np.ndarray:
    a = np.abs(u)
    return a * a / (c + a ** (2.0 - p))


def rho_prime(u: np.ndarray, p: float, c: float) -> np.ndarray:
    a = np.abs(u) ** (2.0 - p)
    return u * (2.0 * c + p * a) / (c + a) ** 2


def _pairs(shape, off):
    """Index slices (m, n) over all voxels m whose neighbour n = m + off lies inside the volume."""
    src, dst = [], []
    for d, size in zip(off, shape):
        if d == -1:
            src.append(slice(1, size)); dst.append(slice(0, size - 1))
        elif d == 1:
            src.append(slice(0, size - 1)); dst.append(slice(1, size))
        else:
            src.append(slice(0, size)); dst.append(slice(0, size))
    return tuple(src), tuple(dst)


def value(f: np.ndarray, p: float = 1.2, sigma: float = 1.0 / 0.7, c: float = 1e-4,
          lam: float = 1.0, weights: dict[int, float] | None = None) -> float:
    """``H(f) = lambda * sum_m sum_{n in N26(m)} w_mn rho((f_m - f_n)/sigma)`` (ordered pairs)."""
    w = inverse_distance_weights() if weights is None else weights
    f = np.asarray(f, dtype=np.float64)
    total = 0.0
    for off in OFFSETS:
        sm, sn = _pairs(f.shape, off)
        total += w[sum(abs(o) for o in off)] * rho((f[sm] - f[sn]) / sigma, p, c).sum()
    return lam * total


def gradient(f: np.ndarray, p: float = 1.2, sigma: float = 1.0 / 0.7, c: float = 1e-4,
             lam: float = 1.0, weights: dict[int, float] | None = None) -> np.ndarray:
    """``dH/df_m = (2 lambda/sigma) sum_n w_mn rho'((f_m - f_n)/sigma)``."""
    w = inverse_distance_weights() if weights is None else weights
    f = np.asarray(f, dtype=np.float64)
    g = np.zeros_like(f)
    for off in OFFSETS:
        sm, sn = _pairs(f.shape, off)
        g[sm] += w[sum(abs(o) for o in off)] * rho_prime((f[sm] - f[sn]) / sigma, p, c)
    return (2.0 * lam / sigma) * g
