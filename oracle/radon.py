"""Fourier-slice Radon transform as a direct non-uniform DFT (FP64 numpy).

Test infrastructure only (see the package docstring).

Discrete reading of the paper's continuous operators (Sec. 2.1 and 2.2):

* slice ``f[iy][ix]`` with pixel centres ``x = ix - N/2``, ``y = iy - N/2``;
* angle ``theta`` with unit normal ``n = (cos theta, sin theta)``
  (Sec. 2.1, the parametrisation ``n(theta)`` under eq. "inverse_radon");
* detector bins ``t_m = m - N_t/2`` and radial frequencies
  ``k_l = (l - N_t/2)/N_t`` in cycles per pixel, ``l = 0..N_t-1``.

The central-slice theorem (eq. "fourier_radon") says that the 1D Fourier
transform of a projection equals the 2D Fourier transform of the slice on
the line through the origin along ``n``.  Discretised:

    Fhat[a, l] = sum_{iy,ix} f[iy,ix] * exp(-2 pi i k_l (x cos th_a + y sin th_a))
    s[a, m]    = Re( (1/N_t) * sum_l Fhat[a, l] * exp(+2 pi i k_l t_m) )

The first line is the non-uniform sum of eq. "fourier_sum" (with the
forward sign of eq. "fourier_radon"), evaluated exactly; the second is the
inverse 1D DFT along the radial line (eq. "nufft" read in reverse).  The
result is real-valued; taking the real part is the reading for the single
Nyquist frequency ``k = -1/2`` that has no ``+1/2`` partner.

The adjoint (eq. "transpose") is taken as the exact matrix transpose of
this discrete map for real Euclidean inner products, without the
continuous measures ``dk dtheta``.

Rotation-axis offset (Sec. 4.1: the Fourier shift property moves the axis of
rotation to the centre).  When the axis projects to bin ``N_t/2 + c``
instead of ``N_t/2``, each projection is the centred one shifted by ``c``
bins, which in the radial spectrum is the phase ``exp(-2 pi i k_l c)``:

    s[a, m]    = Re( (1/N_t) * sum_l Fhat[a, l] * exp(+2 pi i k_l (t_m - c)) )

Every function below takes ``center = c`` (default 0, any real value).

Filtered back-projection (Sec. 2.1, eq. "inverse_radon" and the paragraph
after it): the inversion integral over ``theta`` in [0, pi) and ``k``,
with the sinogram's 1D transform weighted by ``|k|`` (optionally times a
low-pass window), discretised with ``dtheta = pi/N_theta`` and
``dk = 1/N_t``:

    Yhat[a, l] = sum_m y[a, m] exp(-2 pi i k_l (t_m - c))
    g[iy, ix]  = (pi/N_theta) Re sum_a (1/N_t) sum_l w(k_l) Yhat[a, l]
                 exp(+2 pi i k_l (x cos th_a + y sin th_a))

Substituting the first line into the second gives the equivalent closed
form ``s[a,m] = sum_n f_n D(t_m - <x_n, n_a>)`` with the band-limited
(Dirichlet) interpolator ``D(u) = (1/N_t) sum_l cos(2 pi k_l u)``; that form
is used for brute-force matrices and for sampling single outputs.
"""

from __future__ import annotations

import numpy as np


def pixel_coords(n: int) -> np.ndarray:
    """Pixel-centre coordinates ``i - n/2`` (pitch 1), float64."""
    return np.arange(n, dtype=np.float64) - n // 2


def radial_freqs(n_det: int) -> np.ndarray:
    """Radial frequencies ``k_l = (l - N_t/2)/N_t`` in cycles per pixel."""
    return (np.arange(n_det, dtype=np.float64) - n_det // 2) / n_det


def polar_spectrum(f: np.ndarray, angles: np.ndarray, n_det: int) -> np.ndarray:
    """``Fhat[a, l]``: the 2D DFT of the slice sampled on the polar lines.

    Eq. "fourier_sum" evaluated directly (cost O(N_t N^2) per angle).  The
    double sum is factorised exactly as
    ``sum_iy Ey[l,iy] * (sum_ix Ex[l,ix] f[iy,ix])`` with
    ``Ex = exp(-2 pi i k x cos)`` and ``Ey = exp(-2 pi i k y sin)``.
    """
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[0]
    assert f.shape == (n, n)
    x = pixel_coords(n)
    y = pixel_coords(n)
    k = radial_freqs(n_det)
    out = np.empty((len(angles), n_det), dtype=np.complex128)
    for a, th in enumerate(np.asarray(angles, dtype=np.float64)):
        px = -2.0 * np.pi * np.outer(k, x) * np.cos(th)      # phase of Ex [l, ix]
        py = -2.0 * np.pi * np.outer(k, y) * np.sin(th)      # phase of Ey [l, iy]
        # inner sum over ix, as two real products: Ex f^T
        inner = np.cos(px) @ f.T + 1j * (np.sin(px) @ f.T)   # [l, iy]
        out[a] = np.sum((np.cos(py) + 1j * np.sin(py)) * inner, axis=1)
    return out


def radon_fwd(f: np.ndarray, angles: np.ndarray, n_det: int, center: float = 0.0) -> np.ndarray:
    """Forward projection ``s = R f``, float64 [n_angles, n_det].

    Spectrum on the polar lines (``polar_spectrum``), then the inverse 1D
    DFT along each line with ``1/N_t`` and the real part (eq.
    "fourier_radon" inverted), evaluated at ``t_m - center``.  A direct
    DFT, not an FFT.
    """
    k = radial_freqs(n_det)
    t = pixel_coords(n_det) - center
    F = polar_spectrum(f, angles, n_det)
    E = np.exp(2j * np.pi * np.outer(k, t))                  # [l, m]
    return np.real(F @ E) / n_det


def radon_adj(y: np.ndarray, angles: np.ndarray, n: int, center: float = 0.0) -> np.ndarray:
    """Adjoint ``g = R^T y``, float64 [n, n] (exact transpose of ``radon_fwd``).

    Per angle: ``Yhat[l] = (1/N_t) sum_m y[m] exp(-2 pi i k_l (t_m - c))``, then
    ``g[iy,ix] += Re sum_l Yhat[l] conj(Ey[l,iy] Ex[l,ix])`` — the
    transpose of each factor of the forward map (eq. "transpose" without the
    continuous measure).
    """
    y = np.asarray(y, dtype=np.float64)
    n_angles, n_det = y.shape
    assert n_angles == len(angles)
    k = radial_freqs(n_det)
    t = pixel_coords(n_det) - center
    Em = np.exp(-2j * np.pi * np.outer(t, k))               # [m, l]
    return _backproject((y @ Em) / n_det, angles, n)


def _backproject(Yhat: np.ndarray, angles: np.ndarray, n: int) -> np.ndarray:
    """``g[iy,ix] = Re sum_a sum_l Yhat[a,l] conj(Ey[l,iy] Ex[l,ix])`` for
    radial spectra ``Yhat[a, l]`` on ``k_l = (l - N_t/2)/N_t``."""
    n_det = Yhat.shape[1]
    k = radial_freqs(n_det)
    x = pixel_coords(n)
    yc = pixel_coords(n)
    g = np.zeros((n, n), dtype=np.float64)
    for a, th in enumerate(np.asarray(angles, dtype=np.float64)):
        px = 2.0 * np.pi * np.outer(k, x) * np.cos(th)       # phase of conj(Ex)
        py = 2.0 * np.pi * np.outer(k, yc) * np.sin(th)      # phase of conj(Ey)
        B = Yhat[a][:, None] * (np.cos(py) + 1j * np.sin(py))  # [l, iy]
        # Re(B^T conj(Ex)) with conj(Ex) = cos(px) + i sin(px); contiguous
        # copies of the transposed parts keep the products on BLAS
        g += np.ascontiguousarray(B.real.T) @ np.cos(px) - np.ascontiguousarray(B.imag.T) @ np.sin(px)
    return g


def radon_fwd_volume(vol: np.ndarray, angles: np.ndarray, n_det: int, center: float = 0.0) -> np.ndarray:
    """Slice-by-slice forward projection of ``vol[z][y][x]`` -> ``[z][angle][bin]``."""
    return np.stack([radon_fwd(v, angles, n_det, center) for v in np.asarray(vol)])


def radon_adj_volume(sino: np.ndarray, angles: np.ndarray, n: int, center: float = 0.0) -> np.ndarray:
    """Slice-by-slice adjoint of ``sino[z][angle][bin]`` -> ``[z][y][x]``."""
    return np.stack([radon_adj(s, angles, n, center) for s in np.asarray(sino)])


# --------------------------------------------------------------------------
# filtered back-projection
# --------------------------------------------------------------------------

def fbp_window(k: np.ndarray, filt: str = "ramp", order: int = 2, cutoff: float = 0.25) -> np.ndarray:
    """Radial weight ``w(k)`` of the back-projection filter, ``k`` in cycles per pixel.

    ``"ramp"``: ``|k|`` (the Jacobian of eq. "inverse_radon").
    ``"butterworth"``: ``|k| / (1 + (|k|/cutoff)^(2 order))``, the ramp times
    a Butterworth low-pass whose gain is 1/2 at ``cutoff`` (the paper's
    gridrec runs use order 2 and cutoff 0.25, Sec. 5; the window's exact form
    is not given there, so this reading is stated rather than pinned).
    """
    a = np.abs(np.asarray(k, dtype=np.float64))
    if filt == "ramp":
        return a
    if filt == "butterworth":
        return a / (1.0 + (a / cutoff) ** (2 * order))
    raise ValueError(f"unknown filter {filt!r}")


def fbp(y: np.ndarray, angles: np.ndarray, n: int, filt: str = "ramp", order: int = 2,
        cutoff: float = 0.25, center: float = 0.0) -> np.ndarray:
    """Filtered back-projection of one sinogram ``y[a, m]`` -> float64 [n, n].

    Eq. "inverse_radon" discretised (``dtheta = pi/N_theta``, ``dk = 1/N_t``):
    per angle the 1D DFT of the row at ``t_m - center``, weighted by
    ``w(k_l)/N_t``, then the back-projection onto the pixel grid with the
    factor ``pi/N_theta``.
    """
    y = np.asarray(y, dtype=np.float64)
    n_angles, n_det = y.shape
    assert n_angles == len(angles)
    k = radial_freqs(n_det)
    t = pixel_coords(n_det) - center
    Em = np.exp(-2j * np.pi * np.outer(t, k))               # [m, l]
    Yhat = (y @ Em) * (fbp_window(k, filt, order, cutoff) / n_det)
    return (np.pi / n_angles) * _backproject(Yhat, angles, n)


# --------------------------------------------------------------------------
# closed form: band-limited pixel-to-bin interpolator
# --------------------------------------------------------------------------

def dirichlet(u: np.ndarray, n_det: int) -> np.ndarray:
    """``D(u) = (1/N_t) sum_l cos(2 pi k_l u)`` in closed form.

    Summing the geometric series over ``k_l = (l - N_t/2)/N_t`` gives
    ``cos(pi u/N_t) sin(pi u) / (N_t sin(pi u/N_t))``.  Where the
    denominator vanishes (``u`` a multiple of ``N_t``) and near it, the
    defining sum is evaluated instead.
    """
    u = np.asarray(u, dtype=np.float64)
    den = n_det * np.sin(np.pi * u / n_det)
    out = np.empty_like(u)
    near = np.abs(den) < 1e-6
    far = ~near
    out[far] = np.cos(np.pi * u[far] / n_det) * np.sin(np.pi * u[far]) / den[far]
    if np.any(near):
        k = radial_freqs(n_det)
        out[near] = np.cos(2.0 * np.pi * np.outer(u[near], k)).sum(axis=1) / n_det
    return out


def radon_matrix(n: int, angles: np.ndarray, n_det: int, center: float = 0.0) -> np.ndarray:
    """Explicit matrix ``A[(a,m), (iy,ix)] = D(t_m - c - x cos th_a - y sin th_a)``."""
    x = pixel_coords(n)
    X, Y = np.meshgrid(x, x, indexing="xy")                  # X[iy,ix] = x, Y[iy,ix] = y
    t = pixel_coords(n_det) - center
    rows = []
    for th in np.asarray(angles, dtype=np.float64):
        proj = (X * np.cos(th) + Y * np.sin(th)).ravel()    # <x_n, n_a>
        rows.append(dirichlet(t[:, None] - proj[None, :], n_det))
    return np.concatenate(rows, axis=0)


def radon_fwd_entries(f: np.ndarray, angles: np.ndarray, n_det: int,
                      entries: np.ndarray, center: float = 0.0) -> np.ndarray:
    """Selected outputs ``s[a, m]`` for ``entries = [(a, m), ...]`` via the closed form."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[0]
    x = pixel_coords(n)
    X, Y = np.meshgrid(x, x, indexing="xy")
    t = pixel_coords(n_det) - center
    out = np.empty(len(entries))
    for i, (a, m) in enumerate(entries):
        th = angles[a]
        out[i] = np.sum(f * dirichlet(t[m] - X * np.cos(th) - Y * np.sin(th), n_det))
    return out


def radon_adj_entries(y: np.ndarray, angles: np.ndarray, n: int,
                      pixels: np.ndarray, center: float = 0.0) -> np.ndarray:
    """Selected adjoint outputs ``g[iy, ix]`` for ``pixels = [(iy, ix), ...]`` via the closed form."""
    y = np.asarray(y, dtype=np.float64)
    n_angles, n_det = y.shape
    t = pixel_coords(n_det) - center
    c = np.cos(np.asarray(angles, dtype=np.float64))
    s = np.sin(np.asarray(angles, dtype=np.float64))
    out = np.empty(len(pixels))
    for i, (iy, ix) in enumerate(pixels):
        proj = (ix - n // 2) * c + (iy - n // 2) * s        # [a]
        out[i] = np.sum(y * dirichlet(t[None, :] - proj[:, None], n_det))
    return out
