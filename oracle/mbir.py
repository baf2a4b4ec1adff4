"""MBIR objective, gradient and accelerated-gradient loop (FP64) — test infrastructure only.

Sec. 3, eq. "objfn": ``f = argmin G(f) + H(f)`` with the data term
``G = ||R f - b||^2`` and the qGGMRF prior ``H``.  Eq. "gradient" states
``grad G = R*(R f - b)``; that is literally true for ``G = 1/2 ||R f - b||^2``,
which is the reading used here, with ``R*`` the exact transpose.

Sec. 3 (last paragraph) names its optimiser only as an accelerated
gradient method with restart whose objective does not increase, citing
Giselsson and Boyd.  The loop below is the Nesterov/FISTA form with a fixed
``1/L`` step, the gradient restart test (``restart``) and, when
``monotone``, a rejection test that keeps ``x`` (and restarts the momentum)
whenever a step would raise the objective; its agreement with tomoCAM's own
optimiser is parity unpinned (no code or iterates are published).
``L = L_R + L_H`` where ``L_R`` is the largest eigenvalue of ``R^T R``
(power iteration) and ``L_H = 8 lambda/(c sigma^2)`` bounds the prior
Hessian (``max rho'' = 2/c`` at zero, weights summing to one, Gershgorin).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable

import numpy as np

from . import qggmrf
from . import radon


@dataclass
class Prior:
    p: float = 1.2
    sigma: float = 1.0 / 0.7
    c: float = 1e-4
    lam: float = 1.0
    weights: dict = field(default_factory=qggmrf.inverse_distance_weights)

    def value(self, x):
        return qggmrf.value(x, self.p, self.sigma, self.c, self.lam, self.weights)

    def grad(self, x):
        return qggmrf.gradient(x, self.p, self.sigma, self.c, self.lam, self.weights)

    def lipschitz(self) -> float:
        return 8.0 * self.lam / (self.c * self.sigma ** 2)


def radon_ops(angles: np.ndarray, n: int, n_det: int):
    """Volume operators ``(A, At)`` applying the oracle projector slice by slice."""
    A = lambda v: radon.radon_fwd_volume(v, angles, n_det)       # noqa: E731
    At = lambda s: radon.radon_adj_volume(s, angles, n)          # noqa: E731
    return A, At


def objective(x, b, A: Callable, prior: Prior | None) -> float:
    r = A(x) - b
    val = 0.5 * float(np.sum(r * r))
    if prior is not None:
        val += prior.value(x)
    return val


def gradient(x, b, A: Callable, At: Callable, prior: Prior | None) -> np.ndarray:
    """``grad Phi = R^T (R x - b) + grad H(x)``."""
    g = At(A(x) - b)
    if prior is not None:
        g = g + prior.grad(x)
    return g


def power_lipschitz(A: Callable, At: Callable, shape, iters: int = 30, seed: int = 0,
                    safety: float = 1.01) -> float:
    """Largest eigenvalue of ``A^T A`` by power iteration, times ``safety``."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(shape)
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = At(A(v))
        lam = float(np.linalg.norm(w))
        v = w / lam
    return safety * lam


@dataclass
class State:
    x: np.ndarray
    y: np.ndarray
    t: float = 1.0
    k: int = 0
    restarts: int = 0
    phi: float | None = None     # objective at x, once a monotone step has evaluated it
    rejected: int = 0            # steps the monotone test rejected


def step(state: State, b, A, At, prior: Prior | None, L: float, nonneg: bool = False,
         restart: bool = True, monotone: bool = False) -> State:
    """One accelerated-gradient iteration.

    ``g = grad Phi(y_k)``; the candidate ``z = y_k - g/L`` (projected onto
    ``x >= 0`` when ``nonneg``).  With ``restart``, ``<g, z - x_k> > 0``
    resets the momentum (``t_k = 1``).  With ``monotone``, ``z`` is rejected
    when ``Phi(z) > Phi(x_k)``: ``x_{k+1} = x_k``, ``t_k = 1`` and
    ``y_{k+1} = x_{k+1}``; the first step, before any ``Phi(x)`` is known, is
    accepted.  Otherwise ``x_{k+1} = z``.  Then ``t_{k+1} = (1 + sqrt(1 + 4
    t_k^2))/2`` and ``y_{k+1} = x_{k+1} + ((t_k - 1)/t_{k+1}) (x_{k+1} - x_k)``.
    """
    g = gradient(state.y, b, A, At, prior)
    z = state.y - g / L
    if nonneg:
        z = np.maximum(z, 0.0)
    t = state.t
    restarts, rejected, phi = state.restarts, state.rejected, state.phi
    if restart and float(np.sum(g * (z - state.x))) > 0.0:
        t = 1.0
        restarts += 1
    accept = True
    if monotone:
        phi_z = objective(z, b, A, prior)
        if phi is not None and not phi_z <= phi:
            accept = False
            t = 1.0
            rejected += 1
        else:
            phi = phi_z
    t_new = 0.5 * (1.0 + math.sqrt(1.0 + 4.0 * t * t))
    if accept:
        x_new = z
        y_new = x_new + ((t - 1.0) / t_new) * (x_new - state.x)
    else:
        x_new = state.x
        y_new = state.x.copy()
    return State(x_new, y_new, t_new, state.k + 1, restarts, phi, rejected)


def run(b, A, At, shape, prior: Prior | None, L: float, iters: int,
        x0: np.ndarray | None = None, nonneg: bool = False,
        callback: Callable | None = None, restart: bool = True, monotone: bool = False) -> State:
    """``iters`` iterations from ``x_0`` (zero by default), ``y_0 = x_0``, ``t_0 = 1``."""
    x0 = np.zeros(shape) if x0 is None else np.asarray(x0, dtype=np.float64)
    st = State(x0.copy(), x0.copy())
    for _ in range(iters):
        st = step(st, b, A, At, prior, L, nonneg, restart, monotone)
        if callback is not None:
            callback(st)
    return st
