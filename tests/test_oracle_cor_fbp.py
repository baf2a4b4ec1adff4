"""Pins of the oracle's rotation-axis offset and filtered back-projection.

Rotation-axis offset (Sec. 4.1, Fourier shift property): an integer offset is
a circular shift of the detector bins; a fractional one moves the closed-form
projection of a Gaussian blob by that many bins; adjointness and the explicit
closed-form matrix still hold.

Filtered back-projection (Sec. 2.1, eq. "inverse_radon"): the closed-form
projections of a Gaussian blob come back as the blob, with an error that
falls as 1/N_t^2 (the sampled ramp's only defect, at k = 0) and does not
depend on the angle count; rows that are pure cosines back-project to a plain
sum of cosines weighted by the filter; the ramp removes constants.
"""

import numpy as np
import pytest

import synth
from oracle import radon
from tests.analytic import blob_projection


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


# ---------------------------------------------------------------- rotation axis

@pytest.mark.parametrize("shift", [3, -5])
def test_integer_offset_is_a_circular_bin_shift(shift):
    rng = np.random.default_rng(20)
    n, nd, na = 24, 28, 7
    ang = rng.uniform(0, np.pi, na)
    f = rng.standard_normal((n, n))
    y = rng.standard_normal((na, nd))
    s0 = radon.radon_fwd(f, ang, nd)
    s1 = radon.radon_fwd(f, ang, nd, center=float(shift))
    assert rel(s1, np.roll(s0, shift, axis=1)) < 1e-12
    g1 = radon.radon_adj(y, ang, n, center=float(shift))
    assert rel(g1, radon.radon_adj(np.roll(y, -shift, axis=1), ang, n)) < 1e-12


@pytest.mark.parametrize("c", [2.37, -1.6])
def test_fractional_offset_moves_the_blob_projection(c):
    n, s, amp, ctr = 80, 3.2, 1.3, (4.1, -6.6)
    f = synth.gaussian_blob(n, ctr, s, amp)
    ang = np.random.default_rng(21).uniform(0, np.pi, 7)
    got = radon.radon_fwd(f, ang, n, center=c)
    ref = blob_projection(ctr, s, amp, ang, radon.pixel_coords(n) - c)
    assert rel(got, ref) < 1e-10
    # the wrong direction of the shift lands 2c bins away
    assert rel(radon.radon_fwd(f, ang, n, center=-c), ref) > 0.1


def test_offset_dot_product_and_brute_force():
    rng = np.random.default_rng(22)
    n, nd, na, c = 16, 20, 9, 1.73
    ang = rng.uniform(0, np.pi, na)
    x = rng.standard_normal((n, n))
    y = rng.standard_normal((na, nd))
    lhs = np.sum(radon.radon_fwd(x, ang, nd, c) * y)
    rhs = np.sum(x * radon.radon_adj(y, ang, n, c))
    assert abs(lhs - rhs) / abs(lhs) < 1e-12
    A = radon.radon_matrix(n, ang, nd, center=c)
    assert rel(radon.radon_fwd(x, ang, nd, c), (A @ x.ravel()).reshape(na, nd)) < 1e-13
    assert rel(radon.radon_adj(y, ang, n, c), (A.T @ y.ravel()).reshape(n, n)) < 1e-13
    e = np.array([[0, 3], [4, 17], [8, 0]])
    s = radon.radon_fwd(x, ang, nd, c)
    assert np.abs(radon.radon_fwd_entries(x, ang, nd, e, c) - s[e[:, 0], e[:, 1]]).max() < 1e-11
    p = np.array([[0, 0], [7, 11], [15, 2]])
    g = radon.radon_adj(y, ang, n, c)
    assert np.abs(radon.radon_adj_entries(y, ang, n, p, c) - g[p[:, 0], p[:, 1]]).max() < 1e-11


# ---------------------------------------------------------- filtered back-projection

def _blob_fbp_error(n_det, n_angles, c=0.0):
    n, s, ctr = 64, 4.0, (5.3, -3.1)
    f = synth.gaussian_blob(n, ctr, s, 1.0)
    ang = synth.uniform_angles(n_angles)
    y = blob_projection(ctr, s, 1.0, ang, radon.pixel_coords(n_det) - c)
    g = radon.fbp(y, ang, n, center=c)
    x = radon.pixel_coords(n)
    X, Y = np.meshgrid(x, x, indexing="xy")
    disc = X ** 2 + Y ** 2 <= (n / 2 - 2) ** 2
    return float(np.abs(g - f)[disc].max())


def test_fbp_inverts_blob_projections():
    errs = [_blob_fbp_error(nd, 100) for nd in (128, 256, 512)]
    assert errs[0] < 4e-3 and errs[1] < 1e-3 and errs[2] < 2.5e-4
    for a, b in zip(errs, errs[1:]):
        assert 3.5 < a / b < 4.6          # second order in the radial step 1/N_t
    # angular sampling is already exact for this band-limited object
    assert abs(_blob_fbp_error(256, 200) - errs[1]) < 1e-12
    # a shifted rotation axis in data and model cancels
    assert abs(_blob_fbp_error(256, 100, c=2.37) - errs[1]) < 1e-9


@pytest.mark.parametrize("filt", ["ramp", "butterworth"])
def test_fbp_of_cosine_rows(filt):
    """y[a, m] = cos(2 pi j t_m / N_t) has spectrum N_t/2 at k = +-j/N_t only, so
    g(x) = (pi/N_theta) w(j/N_t) sum_a cos(2 pi j <x, n_a> / N_t)."""
    n, nd, na, j = 20, 32, 11, 5
    ang = np.random.default_rng(23).uniform(0, np.pi, na)
    t = radon.pixel_coords(nd)
    y = np.tile(np.cos(2 * np.pi * j * t / nd), (na, 1))
    g = radon.fbp(y, ang, n, filt=filt)
    x = radon.pixel_coords(n)
    X, Y = np.meshgrid(x, x, indexing="xy")
    ref = sum(np.cos(2 * np.pi * j * (X * np.cos(th) + Y * np.sin(th)) / nd) for th in ang)
    w = radon.fbp_window(np.array([j / nd]), filt)[0]
    assert rel(g, (np.pi / na) * w * ref) < 1e-12


def test_fbp_removes_constants():
    rng = np.random.default_rng(24)
    n, nd, na = 24, 32, 13
    ang = rng.uniform(0, np.pi, na)
    g = radon.fbp(np.full((na, nd), 3.7), ang, n)
    assert np.abs(g).max() < 1e-12


def test_butterworth_window_properties():
    k = np.linspace(0.0, 0.5, 201)[1:]
    ramp = radon.fbp_window(k, "ramp")
    assert np.array_equal(ramp, k)
    for order in (1, 2, 4):
        gain = radon.fbp_window(k, "butterworth", order, 0.25) / ramp
        assert np.all(np.diff(gain) < 0)                        # low-pass, monotone
        assert abs(gain[0] - 1.0) < 1e-3                         # unit gain near k = 0
        half = radon.fbp_window(np.array([0.25]), "butterworth", order, 0.25)[0] / 0.25
        assert abs(half - 0.5) < 1e-15                           # half gain at the cutoff
    # a cutoff far above Nyquist is the plain ramp
    rng = np.random.default_rng(25)
    y = rng.standard_normal((9, 20))
    ang = rng.uniform(0, np.pi, 9)
    assert rel(radon.fbp(y, ang, 16, "butterworth", 2, 1e6), radon.fbp(y, ang, 16)) < 1e-12
