"""Pins of the FP64 oracle projector against closed forms, invariants and brute force.

None of these compares the oracle with itself: each expected value comes
from a textbook formula, a special case that reduces to a plain sum, an
exact identity of the discrete operator, or an independently evaluated
closed form (the Dirichlet interpolator) of the same definition.
"""

import math

import numpy as np
import pytest

import synth
from oracle import radon
from tests.analytic import blob_projection, ellipse_projection


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


# P1 — sampled Gaussian blob: band-limited, so R f equals the continuous line integral
def test_blob_closed_form():
    n, s, amp, c = 96, 3.5, 1.7, (6.3, -9.7)
    f = synth.gaussian_blob(n, c, s, amp)
    ang = np.random.default_rng(1).uniform(0, np.pi, 9)
    got = radon.radon_fwd(f, ang, n)
    ref = blob_projection(c, s, amp, ang, radon.pixel_coords(n))
    assert rel(got, ref) < 1e-10


def test_blob_closed_form_other_detector_count():
    # N_t > N: the detector grid is wider than the slice, bins stay unit-pitch
    n, nd, s, c = 64, 80, 3.0, (-4.2, 2.5)
    f = synth.gaussian_blob(n, c, s, 1.0)
    ang = np.array([0.1, 1.3, 2.9])
    got = radon.radon_fwd(f, ang, nd)
    ref = blob_projection(c, s, 1.0, ang, radon.pixel_coords(nd))
    assert rel(got, ref) < 1e-8


# P2 — theta = 0 gives column sums, theta = pi/2 gives row sums
def test_axis_angles_are_plain_sums():
    rng = np.random.default_rng(2)
    n = 24
    f = rng.standard_normal((n, n))
    s = radon.radon_fwd(f, np.array([0.0, np.pi / 2]), n)
    scale = np.abs(f).sum()
    assert np.abs(s[0] - f.sum(axis=0)).max() / scale < 1e-13
    assert np.abs(s[1] - f.sum(axis=1)).max() / scale < 1e-13


# P3 — every projection conserves mass (sum_m D(t_m - u) = 1 exactly)
def test_mass_conservation():
    rng = np.random.default_rng(3)
    n, nd = 30, 36
    f = rng.uniform(0, 1, (n, n))
    ang = rng.uniform(0, np.pi, 11)
    s = radon.radon_fwd(f, ang, nd)
    assert np.abs(s.sum(axis=1) - f.sum()).max() / f.sum() < 1e-13


# P4 — adjointness <R x, y> = <x, R^T y>
@pytest.mark.parametrize("n,nd,na", [(20, 24, 13), (32, 32, 7), (16, 16, 90)])
def test_dot_product(n, nd, na):
    rng = np.random.default_rng(4 + n)
    ang = rng.uniform(0, 2 * np.pi, na)
    x = rng.standard_normal((n, n))
    y = rng.standard_normal((na, nd))
    lhs = np.sum(radon.radon_fwd(x, ang, nd) * y)
    rhs = np.sum(x * radon.radon_adj(y, ang, n))
    assert abs(lhs - rhs) / abs(lhs) < 1e-12


# P5 — brute force: explicit matrix from the closed-form interpolator
@pytest.mark.parametrize("nd", [16, 20])
def test_brute_force_16x16(nd):
    rng = np.random.default_rng(5)
    n, na = 16, 9
    ang = np.concatenate([[0.0, np.pi / 2], rng.uniform(0, np.pi, na - 2)])
    A = radon.radon_matrix(n, ang, nd)
    f = rng.standard_normal((n, n))
    y = rng.standard_normal((na, nd))
    assert rel(radon.radon_fwd(f, ang, nd), (A @ f.ravel()).reshape(na, nd)) < 1e-13
    assert rel(radon.radon_adj(y, ang, n), (A.T @ y.ravel()).reshape(n, n)) < 1e-13


def test_dirichlet_closed_form_matches_sum():
    nd = 12
    u = np.concatenate([np.linspace(-20, 20, 401), [0.0, 12.0, -24.0, 1e-9]])
    k = radon.radial_freqs(nd)
    ref = np.cos(2 * np.pi * np.outer(u, k)).sum(axis=1) / nd
    assert np.abs(radon.dirichlet(u, nd) - ref).max() < 1e-12


def test_sampled_entries_match_full_evaluation():
    rng = np.random.default_rng(6)
    n, nd, na = 48, 52, 6
    ang = rng.uniform(0, np.pi, na)
    f = rng.standard_normal((n, n))
    y = rng.standard_normal((na, nd))
    s = radon.radon_fwd(f, ang, nd)
    g = radon.radon_adj(y, ang, n)
    e = np.stack([rng.integers(0, na, 20), rng.integers(0, nd, 20)], axis=1)
    p = np.stack([rng.integers(0, n, 20), rng.integers(0, n, 20)], axis=1)
    assert np.abs(radon.radon_fwd_entries(f, ang, nd, e) - s[e[:, 0], e[:, 1]]).max() < 1e-11
    assert np.abs(radon.radon_adj_entries(y, ang, n, p) - g[p[:, 0], p[:, 1]]).max() < 1e-11


# P6 — random ellipses against analytic chord lengths (limited by rasterisation)
def test_ellipses_against_analytic_projection():
    errs = {}
    for n in (64, 128):
        params = synth.ellipse_params(synth.rng_for(1, 0), n, 8)
        f = synth.rasterize_ellipses(params, n).numpy()
        ang = synth.uniform_angles(30)
        got = radon.radon_fwd(f, ang, n)
        ref = ellipse_projection(params, ang, radon.pixel_coords(n))
        errs[n] = rel(got, ref)
    assert errs[128] < 3e-2
    assert errs[128] < errs[64]


def test_volume_helpers_are_slicewise():
    rng = np.random.default_rng(7)
    vol = rng.standard_normal((3, 12, 12))
    ang = rng.uniform(0, np.pi, 5)
    s = radon.radon_fwd_volume(vol, ang, 12)
    assert s.shape == (3, 5, 12)
    assert rel(s[1], radon.radon_fwd(vol[1], ang, 12)) < 1e-15
    g = radon.radon_adj_volume(s, ang, 12)
    assert rel(g[2], radon.radon_adj(s[2], ang, 12)) < 1e-15


# Planted mistakes (in a copy of the oracle's arithmetic, on the CPU): each one must trip a pin.
def _fwd_transposed(f, ang, nd):
    return radon.radon_fwd(np.asarray(f).T, ang, nd)


def _fwd_wrong_sign(f, ang, nd):
    k = radon.radial_freqs(nd)
    t = radon.pixel_coords(nd)
    F = radon.polar_spectrum(f, ang, nd)
    return np.real(F @ np.exp(-2j * np.pi * np.outer(k, t))) / nd


def _fwd_no_scale(f, ang, nd):
    return radon.radon_fwd(f, ang, nd) * nd


def test_planted_mistakes_are_caught():
    rng = np.random.default_rng(8)
    n = 24
    f = rng.standard_normal((n, n))
    axes = np.array([0.0, np.pi / 2])
    # transposed operand: theta=0 no longer gives column sums
    assert np.abs(_fwd_transposed(f, axes, n)[0] - f.sum(axis=0)).max() > 1e-3
    # wrong sign of the radial inverse DFT: off-centre blob lands on the mirrored bin
    fb = synth.gaussian_blob(64, (6.0, -3.0), 3.0)
    ang = np.array([0.4, 2.0])
    ref = blob_projection((6.0, -3.0), 3.0, 1.0, ang, radon.pixel_coords(64))
    assert rel(_fwd_wrong_sign(fb, ang, 64), ref) > 0.1
    # dropped 1/N_t: mass conservation fails
    assert abs(_fwd_no_scale(f, np.array([0.3]), n).sum() - f.sum()) > 1e-3 * abs(f).sum()
    assert math.isfinite(float(f.sum()))
