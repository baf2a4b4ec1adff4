"""Pins of the FP64 MBIR oracle: least squares, an independent minimiser, restart, resume."""

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import mbir, radon

N, NZ, NA, ND = 8, 2, 16, 16


def _geometry():
    ang = np.arange(NA) * np.pi / NA
    return ang, *mbir.radon_ops(ang, N, ND)


def _data(seed=20):
    rng = np.random.default_rng(seed)
    x_true = rng.uniform(0, 1, (NZ, N, N))
    ang, A, At = _geometry()
    b = A(x_true) + 0.01 * rng.standard_normal((NZ, NA, ND))
    return ang, A, At, b


def test_power_iteration_matches_svd():
    ang, A, At = _geometry()
    M = radon.radon_matrix(N, ang, ND)
    top = np.linalg.svd(M, compute_uv=False)[0] ** 2
    L = mbir.power_lipschitz(A, At, (NZ, N, N), iters=200, safety=1.0)
    assert abs(L - top) / top < 1e-8


def test_unregularised_iterates_reach_least_squares():
    ang, A, At, b = _data()
    M = radon.radon_matrix(N, ang, ND)
    ref = np.stack([np.linalg.lstsq(M, b[z].ravel(), rcond=None)[0].reshape(N, N) for z in range(NZ)])
    L = mbir.power_lipschitz(A, At, (NZ, N, N), iters=100)
    st = mbir.run(b, A, At, (NZ, N, N), None, L, iters=2500)
    assert np.linalg.norm(st.x - ref) / np.linalg.norm(ref) < 1e-6
    assert st.restarts > 0


def test_regularised_minimum_matches_lbfgs():
    ang, A, At, b = _data(21)
    prior = mbir.Prior(p=1.2, sigma=1.0, c=0.05, lam=0.5)
    L = mbir.power_lipschitz(A, At, (NZ, N, N), iters=100) + prior.lipschitz()
    st = mbir.run(b, A, At, (NZ, N, N), prior, L, iters=2500)
    phi = lambda v: mbir.objective(v.reshape(NZ, N, N), b, A, prior)            # noqa: E731
    jac = lambda v: mbir.gradient(v.reshape(NZ, N, N), b, A, At, prior).ravel()  # noqa: E731
    res = minimize(phi, np.zeros(NZ * N * N), jac=jac, method="L-BFGS-B",
                   options={"maxiter": 20000, "ftol": 1e-15, "gtol": 1e-12, "maxcor": 30})
    assert abs(phi(st.x.ravel()) - res.fun) / abs(res.fun) < 1e-6
    assert np.linalg.norm(st.x.ravel() - res.x) / np.linalg.norm(res.x) < 1e-3


def test_objective_decreases_and_gradient_matches_fd():
    ang, A, At, b = _data(22)
    prior = mbir.Prior(lam=0.3)
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 1, (NZ, N, N))
    g = mbir.gradient(x, b, A, At, prior)
    h = 1e-6
    for idx in [(0, 1, 2), (1, 7, 0), (0, 4, 4)]:
        e = np.zeros_like(x)
        e[idx] = h
        fd = (mbir.objective(x + e, b, A, prior) - mbir.objective(x - e, b, A, prior)) / (2 * h)
        assert abs(g[idx] - fd) <= 1e-6 * max(1.0, abs(fd))


def test_restart_resets_momentum():
    # when <g, x_{k+1} - x_k> > 0 fires, t_k = 1 so beta = 0: y_{k+1} == x_{k+1} and t_{k+1} = golden ratio
    ang, A, At, b = _data(23)
    L = mbir.power_lipschitz(A, At, (NZ, N, N), iters=50)
    st = mbir.State(np.zeros((NZ, N, N)), np.zeros((NZ, N, N)))
    fired = 0
    for _ in range(200):
        prev = st.restarts
        st = mbir.step(st, b, A, At, None, L)
        if st.restarts > prev:
            fired += 1
            assert np.array_equal(st.y, st.x)
            assert st.t == 0.5 * (1.0 + np.sqrt(5.0))
    assert fired >= 1


def test_resume_is_bit_exact():
    ang, A, At, b = _data(24)
    prior = mbir.Prior(lam=0.2, c=0.01, sigma=1.0)
    L = mbir.power_lipschitz(A, At, (NZ, N, N), iters=30) + prior.lipschitz()
    full = mbir.run(b, A, At, (NZ, N, N), prior, L, iters=6)
    half = mbir.run(b, A, At, (NZ, N, N), prior, L, iters=3)
    saved = mbir.State(half.x.copy(), half.y.copy(), half.t, half.k, half.restarts)
    for _ in range(3):
        saved = mbir.step(saved, b, A, At, prior, L)
    assert np.array_equal(saved.x, full.x) and saved.t == full.t


@pytest.mark.parametrize("nonneg", [False, True])
def test_nonneg_projection(nonneg):
    ang, A, At, b = _data(25)
    b = -np.abs(b)
    L = mbir.power_lipschitz(A, At, (NZ, N, N), iters=30)
    st = mbir.run(b, A, At, (NZ, N, N), None, L, iters=5, nonneg=nonneg)
    assert (st.x.min() >= 0.0) == nonneg


def test_gradient_fd_on_crop_geometry():
    """P11 (oracle half): the FP64 gradient on a 32x32x4 crop with 256 angles vs central differences."""
    import synth
    rng = np.random.default_rng(50)
    n, nz, na = 32, 4, 256
    vol = synth.rasterize_ellipsoids(synth.ellipsoid_params(rng, n, nz, 5), n, nz).numpy()
    ang = synth.uniform_angles(na)
    A, At = mbir.radon_ops(ang, n, n)
    b = A(vol) + 0.01 * rng.standard_normal((nz, na, n))
    prior = mbir.Prior(lam=1.0)
    x = rng.uniform(0, 1, vol.shape)
    g = mbir.gradient(x, b, A, At, prior)
    h = 1e-5
    for idx in [(0, 5, 7), (2, 16, 16), (3, 30, 1)]:
        e = np.zeros_like(x)
        e[idx] = h
        fd = (mbir.objective(x + e, b, A, prior) - mbir.objective(x - e, b, A, prior)) / (2 * h)
        assert abs(g[idx] - fd) <= 1e-7 * max(abs(fd), np.abs(g).max() * 1e-3)


def _objectives(b, A, At, prior, L, iters, **kw):
    vals = []
    mbir.run(b, A, At, (NZ, N, N), prior, L, iters,
             callback=lambda s: vals.append(mbir.objective(s.x, b, A, prior)), **kw)
    return np.array(vals)


def test_monotone_variant_never_rises_and_reaches_the_minimum():
    """Sec. 3's optimiser keeps the objective from rising: with a valid step the
    monotone variant's objective never increases and it reaches the same
    minimum as an independent solver (L-BFGS)."""
    ang, A, At, b = _data(26)
    prior = mbir.Prior(p=1.2, sigma=1.0, c=0.05, lam=0.5)
    L = mbir.power_lipschitz(A, At, (NZ, N, N), iters=100) + prior.lipschitz()
    vals = _objectives(b, A, At, prior, L, 600, monotone=True)
    assert np.all(np.diff(vals) <= 0.0)
    st = mbir.run(b, A, At, (NZ, N, N), prior, L, iters=2500, monotone=True)
    phi = lambda v: mbir.objective(v.reshape(NZ, N, N), b, A, prior)            # noqa: E731
    jac = lambda v: mbir.gradient(v.reshape(NZ, N, N), b, A, At, prior).ravel()  # noqa: E731
    res = minimize(phi, np.zeros(NZ * N * N), jac=jac, method="L-BFGS-B",
                   options={"maxiter": 20000, "ftol": 1e-15, "gtol": 1e-12, "maxcor": 30})
    assert abs(phi(st.x.ravel()) - res.fun) / abs(res.fun) < 1e-6


def test_monotone_test_catches_rising_steps():
    """With a step longer than 1/L_R (L = 0.8 L_R) the momentum lets the
    objective rise now and then; the monotone variant rejects those steps,
    never rises, and still reaches the least-squares solution."""
    ang, A, At, b = _data(27)
    M = radon.radon_matrix(N, ang, ND)
    ref = np.stack([np.linalg.lstsq(M, b[z].ravel(), rcond=None)[0].reshape(N, N) for z in range(NZ)])
    L = 0.8 * mbir.power_lipschitz(A, At, (NZ, N, N), iters=200, safety=1.0)
    plain = _objectives(b, A, At, None, L, 1500)
    assert np.any(np.diff(plain) > 0.0)
    mono = _objectives(b, A, At, None, L, 1500, monotone=True)
    assert np.all(np.diff(mono) <= 0.0)
    st = mbir.run(b, A, At, (NZ, N, N), None, L, iters=3000, monotone=True)
    assert st.rejected > 0
    assert np.linalg.norm(st.x - ref) / np.linalg.norm(ref) < 1e-6


def test_rejected_step_keeps_x_and_restarts():
    ang, A, At, b = _data(27)
    L = 0.8 * mbir.power_lipschitz(A, At, (NZ, N, N), iters=200, safety=1.0)
    st = mbir.State(np.zeros((NZ, N, N)), np.zeros((NZ, N, N)))
    seen = 0
    for _ in range(1500):
        prev = st
        st = mbir.step(st, b, A, At, None, L, monotone=True)
        if st.rejected > prev.rejected:
            seen += 1
            assert np.array_equal(st.x, prev.x) and np.array_equal(st.y, st.x)
            assert st.t == 0.5 * (1.0 + np.sqrt(5.0)) and st.phi == prev.phi
        if seen == 2:
            break
    assert seen >= 1


def test_restart_flag_off_is_plain_momentum():
    """restart=False never resets t: t_k follows t_{k+1} = (1 + sqrt(1 + 4 t_k^2))/2 from t_0 = 1."""
    ang, A, At, b = _data(29)
    L = mbir.power_lipschitz(A, At, (NZ, N, N), iters=50)
    st = mbir.run(b, A, At, (NZ, N, N), None, L, iters=40, restart=False)
    t = 1.0
    for _ in range(40):
        t = 0.5 * (1.0 + np.sqrt(1.0 + 4.0 * t * t))
    assert st.restarts == 0 and st.t == t
