"""Random ellipse / ellipsoid phantoms, angle sets and noise models.

Geometry convention (shared with the projector): a slice is ``f[iy][ix]``
with pixel centres at ``x = ix - N/2`` and ``y = iy - N/2`` (pitch 1); a
volume is ``f[iz][iy][ix]`` with ``z = iz - Z/2``.

Every generator takes an explicit ``numpy.random.Generator`` so that a test
and the benchmark draw identical inputs from the same seed
(``rng_for(config, z)``).  Rasterisation runs in float64 with torch so it
can use a GPU when one is present; results are identical up to FP64
rounding on either device.
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

SEED_ROOT = 230412934


def rng_for(config: int, z: int = 0) -> np.random.Generator:
    """Seeded generator for input ``z`` of workload ``config``."""
    return np.random.default_rng(np.random.SeedSequence([SEED_ROOT, int(config), int(z)]))


# --------------------------------------------------------------------------
# 2D ellipses
# --------------------------------------------------------------------------

@dataclass
class Ellipse:
    cx: float
    cy: float
    a: float      # semi-axis along direction psi
    b: float      # semi-axis perpendicular to psi
    psi: float    # orientation, radians from +x towards +y
    rho: float    # additive density


def ellipse_params(rng: np.random.Generator, n: int, count: int,
                   r_centre: float = 0.7, ax_lo: float = 0.04, ax_hi: float = 0.30,
                   r_max: float = 0.9) -> list[Ellipse]:
    """Draw ``count`` ellipses that lie inside the disc of radius ``r_max*n/2``.

    Centre at radius ``r_centre*(n/2)*sqrt(U)`` and uniform polar angle,
    semi-axes ``U[ax_lo, ax_hi]*n/2``, orientation ``U[0, pi)``, density
    ``U[0, 1]``; rejected and redrawn until ``|c| + max(a, b) <= r_max*n/2``.
    """
    half = n / 2.0
    out: list[Ellipse] = []
    while len(out) < count:
        r = r_centre * half * math.sqrt(rng.uniform())
        phi = rng.uniform(0.0, 2.0 * math.pi)
        a = rng.uniform(ax_lo, ax_hi) * half
        b = rng.uniform(ax_lo, ax_hi) * half
        psi = rng.uniform(0.0, math.pi)
        rho = rng.uniform(0.0, 1.0)
        if r + max(a, b) <= r_max * half:
            out.append(Ellipse(r * math.cos(phi), r * math.sin(phi), a, b, psi, rho))
    return out


def _subsample_offsets(ss: int) -> torch.Tensor:
    return (torch.arange(ss, dtype=torch.float64) + 0.5) / ss - 0.5


def rasterize_ellipses(params: list[Ellipse], n: int, supersample: int = 4,
                       device: str | torch.device = "cpu") -> torch.Tensor:
    """Pixel-average rasterisation (``supersample``^2 points per pixel), float64 [n, n]."""
    img = torch.zeros((n, n), dtype=torch.float64, device=device)
    off = _subsample_offsets(supersample).to(device)
    half = n // 2
    for e in params:
        c, s = math.cos(e.psi), math.sin(e.psi)
        hx = math.sqrt((e.a * c) ** 2 + (e.b * s) ** 2)
        hy = math.sqrt((e.a * s) ** 2 + (e.b * c) ** 2)
        ix0 = max(0, int(math.floor(e.cx - hx)) + half - 1)
        ix1 = min(n, int(math.ceil(e.cx + hx)) + half + 2)
        iy0 = max(0, int(math.floor(e.cy - hy)) + half - 1)
        iy1 = min(n, int(math.ceil(e.cy + hy)) + half + 2)
        if ix0 >= ix1 or iy0 >= iy1:
            continue
        xs = (torch.arange(ix0, ix1, dtype=torch.float64, device=device) - half)
        ys = (torch.arange(iy0, iy1, dtype=torch.float64, device=device) - half)
        # sub-sample coordinates [ny, ss, nx, ss]
        X = (xs[:, None] + off[None, :]).reshape(1, 1, -1)
        Y = (ys[:, None] + off[None, :]).reshape(1, -1, 1)
        dx = X - e.cx
        dy = Y - e.cy
        u = (dx * c + dy * s) / e.a
        v = (-dx * s + dy * c) / e.b
        inside = ((u * u + v * v) <= 1.0).to(torch.float64)[0]
        ny, nx = iy1 - iy0, ix1 - ix0
        frac = inside.reshape(ny, supersample, nx, supersample).mean(dim=(1, 3))
        img[iy0:iy1, ix0:ix1] += e.rho * frac
    return img


def ellipse_phantom(config: int, z: int, n: int, count: int,
                    device: str | torch.device = "cpu") -> torch.Tensor:
    """Seeded random-ellipse slice, float64 [n, n]."""
    return rasterize_ellipses(ellipse_params(rng_for(config, z), n, count), n, device=device)


# --------------------------------------------------------------------------
# 3D ellipsoids
# --------------------------------------------------------------------------

@dataclass
class Ellipsoid:
    centre: np.ndarray   # (x, y, z) in voxel units
    axes: np.ndarray     # semi-axes in isotropic units (z scaled by n/nz)
    rot: np.ndarray      # 3x3 rotation matrix (columns = principal directions)
    rho: float


def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def ellipsoid_params(rng: np.random.Generator, n: int, nz: int, count: int,
                     r_centre: float = 0.7, ax_lo: float = 0.04, ax_hi: float = 0.30,
                     r_max: float = 0.9) -> list[Ellipsoid]:
    """Draw ellipsoids inside the cylinder of radius ``r_max*n/2``.

    The z axis is scaled by ``n/nz`` so that shapes are drawn isotropically
    in a cube and then squeezed into the slab; each z cut is an ellipse.
    """
    half = n / 2.0
    out: list[Ellipsoid] = []
    while len(out) < count:
        r = r_centre * half * math.sqrt(rng.uniform())
        phi = rng.uniform(0.0, 2.0 * math.pi)
        cz = rng.uniform(-0.8, 0.8) * nz / 2.0
        axes = rng.uniform(ax_lo, ax_hi, size=3) * half
        rot = _random_rotation(rng)
        rho = rng.uniform(0.0, 1.0)
        if r + axes.max() <= r_max * half:
            out.append(Ellipsoid(np.array([r * math.cos(phi), r * math.sin(phi), cz]),
                                 axes, rot, rho))
    return out


def rasterize_ellipsoids(params: list[Ellipsoid], n: int, nz: int, supersample: int = 4,
                         device: str | torch.device = "cpu") -> torch.Tensor:
    """Rasterise into float64 [nz, n, n]: in-plane ``supersample``^2 averaging at voxel-centre z."""
    vol = torch.zeros((nz, n, n), dtype=torch.float64, device=device)
    off = _subsample_offsets(supersample).to(device)
    half = n // 2
    zscale = n / nz
    xs_all = torch.arange(n, dtype=torch.float64, device=device) - half
    for e in params:
        # quadratic form in isotropic coordinates: q(p) = (p-c)^T M (p-c)
        M = e.rot @ np.diag(1.0 / e.axes ** 2) @ e.rot.T
        Mt = torch.tensor(M, dtype=torch.float64, device=device)
        cx, cy, cz = e.centre
        ext = float(e.axes.max())
        ix0 = max(0, int(math.floor(cx - ext)) + half - 1)
        ix1 = min(n, int(math.ceil(cx + ext)) + half + 2)
        iy0 = max(0, int(math.floor(cy - ext)) + half - 1)
        iy1 = min(n, int(math.ceil(cy + ext)) + half + 2)
        X = (xs_all[ix0:ix1][:, None] + off[None, :]).reshape(1, -1) - cx
        Y = (xs_all[iy0:iy1][:, None] + off[None, :]).reshape(-1, 1) - cy
        ny, nx = iy1 - iy0, ix1 - ix0
        for iz in range(nz):
            dz = ((iz - nz // 2) - cz) * zscale
            if abs(dz) > ext:
                continue
            q = (Mt[0, 0] * X * X + Mt[1, 1] * Y * Y + Mt[2, 2] * dz * dz
                 + 2 * Mt[0, 1] * X * Y + 2 * Mt[0, 2] * X * dz + 2 * Mt[1, 2] * Y * dz)
            inside = (q <= 1.0).to(torch.float64)
            frac = inside.reshape(ny, supersample, nx, supersample).mean(dim=(1, 3))
            vol[iz, iy0:iy1, ix0:ix1] += e.rho * frac
    return vol


def ellipsoid_volume(config: int, n: int, nz: int, count: int,
                     device: str | torch.device = "cpu") -> torch.Tensor:
    return rasterize_ellipsoids(ellipsoid_params(rng_for(config, 0), n, nz, count), n, nz,
                                device=device)


def add_cracks(vol: torch.Tensor, rng: np.random.Generator, count: int,
               thickness: float = 1.5, blur_sigma: float = 1.0) -> torch.Tensor:
    """Zero thin random planes (``thickness`` voxels) inside the support, then blur them.

    Each crack is a random plane through a random interior point, clipped to
    a ball of radius ``U[0.1, 0.3]*n/2``.  The crack mask is smoothed by a
    separable Gaussian of ``blur_sigma`` voxels before it multiplies the volume.
    """
    nz, n, _ = vol.shape
    dev = vol.device
    half = n // 2
    zscale = n / nz
    zz = ((torch.arange(nz, dtype=torch.float64, device=dev) - nz // 2) * zscale)[:, None, None]
    yy = (torch.arange(n, dtype=torch.float64, device=dev) - half)[None, :, None]
    xx = (torch.arange(n, dtype=torch.float64, device=dev) - half)[None, None, :]
    keep = torch.ones_like(vol)
    for _ in range(count):
        r = 0.6 * half * math.sqrt(rng.uniform())
        phi = rng.uniform(0, 2 * math.pi)
        c = (r * math.cos(phi), r * math.sin(phi), rng.uniform(-0.6, 0.6) * nz / 2 * zscale)
        nrm = rng.normal(size=3)
        nrm /= np.linalg.norm(nrm)
        rad = rng.uniform(0.1, 0.3) * half
        d = (xx - c[0]) * nrm[0] + (yy - c[1]) * nrm[1] + (zz - c[2]) * nrm[2]
        dist2 = (xx - c[0]) ** 2 + (yy - c[1]) ** 2 + (zz - c[2]) ** 2
        keep = keep * torch.where((d.abs() <= thickness / 2) & (dist2 <= rad * rad),
                                  torch.zeros((), dtype=vol.dtype, device=dev),
                                  torch.ones((), dtype=vol.dtype, device=dev))
    if blur_sigma > 0:
        rad = int(math.ceil(3 * blur_sigma))
        t = np.arange(-rad, rad + 1, dtype=np.float64)
        k = np.exp(-0.5 * (t / blur_sigma) ** 2)
        k = k / k.sum()
        for dim in range(3):
            keep = _smooth_axis(keep, k, dim)
    return vol * keep


def _smooth_axis(m: torch.Tensor, k: np.ndarray, dim: int) -> torch.Tensor:
    """Correlate ``m`` with the odd-length taps ``k`` along ``dim``, edges replicated."""
    rad = (len(k) - 1) // 2
    size = m.shape[dim]
    lo = m.narrow(dim, 0, 1).expand(*[rad if d == dim else -1 for d in range(m.dim())])
    hi = m.narrow(dim, size - 1, 1).expand(*[rad if d == dim else -1 for d in range(m.dim())])
    padded = torch.cat([lo, m, hi], dim=dim)
    out = torch.zeros_like(m)
    for i, w in enumerate(k):
        out += float(w) * padded.narrow(dim, i, size)
    return out


def gaussian_blob(n: int, centre: tuple[float, float], s: float, amp: float = 1.0) -> np.ndarray:
    """Sampled ``amp*exp(-|x-c|^2/(2 s^2))`` on the pixel centres, float64 [n, n]."""
    x = np.arange(n) - n // 2
    X, Y = np.meshgrid(x, x, indexing="xy")
    return amp * np.exp(-((X - centre[0]) ** 2 + (Y - centre[1]) ** 2) / (2.0 * s * s))


# --------------------------------------------------------------------------
# angle sets
# --------------------------------------------------------------------------

def uniform_angles(n_angles: int, span: float = math.pi, offset: float = 0.0) -> np.ndarray:
    """``offset + a*span/n_angles`` for a = 0..n_angles-1, float64."""
    return offset + np.arange(n_angles, dtype=np.float64) * (span / n_angles)


def sparse_angles(rng: np.random.Generator, n_angles: int) -> np.ndarray:
    """Full span pi with a random offset in [0, pi/n_angles)."""
    return uniform_angles(n_angles, math.pi, rng.uniform(0.0, math.pi / n_angles))


def limited_view_angles(rng: np.random.Generator, n_angles: int) -> np.ndarray:
    """Span ``U[pi/2, pi)`` starting at ``U[0, pi - span)``."""
    span = rng.uniform(math.pi / 2, math.pi)
    off = rng.uniform(0.0, math.pi - span)
    return uniform_angles(n_angles, span, off)


def uneven_stack(rng: np.random.Generator, count: int, sizes=(512, 1024, 2048),
                 angle_range=(128, 1500)) -> list[tuple[int, np.ndarray]]:
    """``count`` slices of an uneven stack: (N, angles) with N drawn from
    ``sizes``, the angle count uniform in ``angle_range`` (inclusive), even
    slices sparse (span pi, random offset) and odd ones limited-view."""
    out = []
    for i in range(count):
        n = int(rng.choice(list(sizes)))
        na = int(rng.integers(angle_range[0], angle_range[1] + 1))
        ang = sparse_angles(rng, na) if i % 2 == 0 else limited_view_angles(rng, na)
        out.append((n, ang))
    return out


# --------------------------------------------------------------------------
# measurement noise (takes the clean data as input)
# --------------------------------------------------------------------------

def poisson_log_data(b_true: np.ndarray | torch.Tensor, rng: np.random.Generator,
                     i0: float = 1.0e4) -> np.ndarray:
    """Beer-Lambert counts ``I ~ Poisson(i0*exp(-b_true))`` returned as ``-log(max(I,1)/i0)``."""
    b = b_true.detach().cpu().numpy() if isinstance(b_true, torch.Tensor) else np.asarray(b_true)
    counts = rng.poisson(i0 * np.exp(-b.astype(np.float64)))
    return -np.log(np.maximum(counts, 1) / i0)


def gaussian_noise(b_true: np.ndarray | torch.Tensor, rng: np.random.Generator,
                   rel_sigma: float = 0.01) -> np.ndarray:
    """``b_true + N(0, (rel_sigma*max|b_true|)^2)``."""
    b = b_true.detach().cpu().numpy() if isinstance(b_true, torch.Tensor) else np.asarray(b_true)
    b = b.astype(np.float64)
    return b + rng.normal(scale=rel_sigma * np.abs(b).max(), size=b.shape)
