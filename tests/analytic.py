"""Closed-form projections used as pins (textbook formulas, independent of both paths)."""

from __future__ import annotations

import numpy as np


def ellipse_projection(ellipses, angles: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Line integrals of a sum of uniform ellipses, ``[angle, t]``.

    For an ellipse of density ``rho``, centre ``c``, semi-axes ``a`` (along
    ``psi``) and ``b``: with ``s^2 = a^2 cos^2(th - psi) + b^2 sin^2(th - psi)``
    and ``tau = t - <c, n>``, the chord integral is ``2 rho a b sqrt(s^2 - tau^2)/s^2``
    for ``|tau| <= s`` and zero otherwise.
    """
    out = np.zeros((len(angles), len(t)))
    for e in ellipses:
        for i, th in enumerate(angles):
            s2 = (e.a * np.cos(th - e.psi)) ** 2 + (e.b * np.sin(th - e.psi)) ** 2
            tau = t - (e.cx * np.cos(th) + e.cy * np.sin(th))
            out[i] += np.where(tau * tau < s2,
                               2.0 * e.rho * e.a * e.b * np.sqrt(np.maximum(s2 - tau * tau, 0.0)) / s2,
                               0.0)
    return out


def blob_projection(centre, s: float, amp: float, angles: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Line integrals of ``amp*exp(-|x-c|^2/(2 s^2))``: ``amp*sqrt(2 pi) s exp(-(t-<c,n>)^2/(2 s^2))``."""
    proj = centre[0] * np.cos(angles) + centre[1] * np.sin(angles)
    return amp * np.sqrt(2 * np.pi) * s * np.exp(-(t[None, :] - proj[:, None]) ** 2 / (2 * s * s))
