"""Pins of the FP64 qGGMRF oracle: finite differences, invariants, special cases, brute force."""

import itertools
import json
import os

import numpy as np
import pytest

from oracle import qggmrf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _paper_hyper():
    with open(os.path.join(GOLDEN, "paper_hyperparameters.json")) as fh:
        return json.load(fh)


def test_paper_hyperparameters_fixture():
    h = _paper_hyper()
    assert h["p"] == 1.2 and h["c"] == 1e-4
    assert abs(h["sigma"] - 1 / 0.7) < 1e-15
    assert h["neighbours"] == 26
    assert len(qggmrf.OFFSETS) == h["neighbours"]


def test_weights_partition_unity_and_inverse_distance():
    w = qggmrf.inverse_distance_weights()
    assert abs(6 * w[1] + 12 * w[2] + 8 * w[3] - 1.0) < 1e-15
    assert abs(w[1] / w[2] - np.sqrt(2)) < 1e-14 and abs(w[1] / w[3] - np.sqrt(3)) < 1e-14
    assert abs(w[1] - 0.052345) < 5e-7 and abs(w[2] - 0.037013) < 5e-7 and abs(w[3] - 0.030221) < 5e-7
    g = qggmrf.gaussian_weights()
    assert abs(6 * g[1] + 12 * g[2] + 8 * g[3] - 1.0) < 1e-15


def _brute_value(f, p, sigma, c, lam, w):
    nz, ny, nx = f.shape
    tot = 0.0
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        for dz, dy, dx in qggmrf.OFFSETS:
            zz, yy, xx = z + dz, y + dy, x + dx
            if 0 <= zz < nz and 0 <= yy < ny and 0 <= xx < nx:
                d = abs(f[z, y, x] - f[zz, yy, xx]) / sigma
                tot += w[abs(dz) + abs(dy) + abs(dx)] * d * d / (c + d ** (2 - p))
    return lam * tot


def test_value_brute_force():
    rng = np.random.default_rng(10)
    f = rng.uniform(0, 1, (3, 4, 5))
    h = _paper_hyper()
    w = qggmrf.inverse_distance_weights()
    ref = _brute_value(f, h["p"], h["sigma"], h["c"], 0.7, w)
    got = qggmrf.value(f, h["p"], h["sigma"], h["c"], 0.7)
    assert abs(got - ref) / ref < 1e-13


@pytest.mark.parametrize("p,c", [(1.2, 1e-4), (1.2, 1e-2), (1.5, 0.3), (2.0, 1e-4)])
def test_gradient_finite_differences(p, c):
    rng = np.random.default_rng(11)
    f = rng.uniform(0, 1, (4, 5, 6))
    sigma, lam = 1 / 0.7, 1.3
    g = qggmrf.gradient(f, p, sigma, c, lam)
    h = 1e-6
    fd = np.zeros_like(f)
    for idx in itertools.product(*map(range, f.shape)):
        e = np.zeros_like(f)
        e[idx] = h
        fd[idx] = (qggmrf.value(f + e, p, sigma, c, lam) - qggmrf.value(f - e, p, sigma, c, lam)) / (2 * h)
    assert np.linalg.norm(g - fd) / np.linalg.norm(fd) < 1e-7


def test_constant_volume_and_shift_invariance():
    rng = np.random.default_rng(12)
    f = rng.uniform(0, 1, (3, 6, 6))
    assert np.all(qggmrf.gradient(np.full((3, 6, 6), 2.5)) == 0.0)
    assert qggmrf.value(np.full((3, 6, 6), 2.5)) == 0.0
    v0 = qggmrf.value(f)
    assert abs(qggmrf.value(f + 3.75) - v0) / v0 < 1e-12
    assert np.abs(qggmrf.gradient(f + 3.75) - qggmrf.gradient(f)).max() < 1e-9 * np.abs(qggmrf.gradient(f)).max()


def test_p2_reduces_to_weighted_laplacian():
    # p = 2: rho(u) = u^2/(c+1) so dH/df_m = 4 lam/(sigma^2 (1+c)) sum_n w_mn (f_m - f_n)
    rng = np.random.default_rng(13)
    f = rng.standard_normal((3, 5, 4))
    sigma, c, lam = 0.8, 0.25, 1.7
    w = qggmrf.inverse_distance_weights()
    nz, ny, nx = f.shape
    ref = np.zeros_like(f)
    for z, y, x in itertools.product(range(nz), range(ny), range(nx)):
        for dz, dy, dx in qggmrf.OFFSETS:
            zz, yy, xx = z + dz, y + dy, x + dx
            if 0 <= zz < nz and 0 <= yy < ny and 0 <= xx < nx:
                ref[z, y, x] += w[abs(dz) + abs(dy) + abs(dx)] * (f[z, y, x] - f[zz, yy, xx])
    ref *= 4 * lam / (sigma ** 2 * (1 + c))
    got = qggmrf.gradient(f, 2.0, sigma, c, lam)
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()


def test_rho_second_derivative_bound():
    # max rho'' = rho''(0) = 2/c: the prior Lipschitz bound 8 lam/(c sigma^2) rests on it
    c, p = 1e-4, 1.2
    u = np.concatenate([np.linspace(-1e-2, 1e-2, 20001), np.linspace(-1e-6, 1e-6, 20001)])
    u = np.unique(u)
    d2 = np.gradient(qggmrf.rho_prime(u, p, c), u)
    assert d2.max() <= 2 / c * (1 + 1e-3)
    assert d2.max() >= 2 / c * (1 - 1e-3)


def test_planted_missing_factor_two_is_caught():
    rng = np.random.default_rng(14)
    f = rng.uniform(0, 1, (3, 3, 3))
    bad = 0.5 * qggmrf.gradient(f)
    h = 1e-6
    e = np.zeros_like(f)
    e[1, 1, 1] = h
    fd = (qggmrf.value(f + e) - qggmrf.value(f - e)) / (2 * h)
    assert abs(bad[1, 1, 1] - fd) > 0.1 * abs(fd)


def test_gaussian_weights_shape():
    """The alternative weights are exp(-d^2/2) normalised over the 26 neighbours:
    each step in squared distance divides the weight by e^{1/2}."""
    w = qggmrf.gaussian_weights()
    assert abs(w[1] / w[2] - np.exp(0.5)) < 1e-14 and abs(w[2] / w[3] - np.exp(0.5)) < 1e-14
    assert abs(6 * w[1] + 12 * w[2] + 8 * w[3] - 1.0) < 1e-15
    # the same Gaussian evaluated at each neighbour's offset, normalised by brute force
    raw = {o: np.exp(-0.5 * sum(c * c for c in o)) for o in qggmrf.OFFSETS}
    total = sum(raw.values())
    for o, v in raw.items():
        assert abs(w[sum(abs(c) for c in o)] - v / total) < 1e-15
