"""GPU parity of the qGGMRF prior kernel, the MBIR step and the autograd path against the FP64 oracle."""

import math
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import mbir as omb
from oracle import qggmrf as oq

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    import paper_2304_12934_amd._lib as L
    L.lib()
    return torch.device("cuda", 0)


def gpu(a, dev):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev)


@pytest.mark.parametrize("shape,p,c", [((4, 32, 32), 1.2, 1e-4), ((5, 70, 70), 1.2, 1e-2),
                                       ((1, 8, 8), 2.0, 0.3), ((3, 130, 130), 1.5, 1e-3)])
def test_qggmrf_against_oracle(dev, shape, p, c):
    from paper_2304_12934_amd import Prior, qggmrf_grad
    say(f"case: qggmrf {shape} p={p} c={c}")
    rng = np.random.default_rng(sum(shape))
    f = rng.uniform(0, 1, shape).astype(np.float32).astype(np.float64)
    pr = Prior(p=p, c=c, sigma=1 / 0.7, lam=0.8)
    g0 = rng.standard_normal(shape).astype(np.float32)
    grad, val = qggmrf_grad(gpu(f, dev), pr, scale=1.5, grad=gpu(g0, dev), value=True)
    ref_g = oq.gradient(f, p, 1 / 0.7, c, 0.8)
    ref_v = oq.value(f, p, 1 / 0.7, c, 0.8)
    got = grad.cpu().numpy().astype(np.float64) - g0
    assert rel(got, 1.5 * ref_g) < 1e-5
    assert abs(float(val.item()) - ref_v) / ref_v < 1e-5


def test_qggmrf_flat_regions_have_zero_gradient(dev):
    from paper_2304_12934_amd import Prior, qggmrf_grad
    say("case: qggmrf piecewise constant")
    f = np.zeros((4, 40, 40), dtype=np.float32)
    f[:, 10:20, 10:20] = 1.0
    grad, _ = qggmrf_grad(gpu(f, dev), Prior())
    g = grad.cpu().numpy()
    assert np.all(g[:, 25:, 25:] == 0.0)
    assert np.abs(g[:, 9:21, 9:21]).max() > 0


def _crop_problem(seed=30, n=32, nz=4, na=256):
    rng = np.random.default_rng(seed)
    vol = synth.rasterize_ellipsoids(synth.ellipsoid_params(rng, n, nz, 5), n, nz).numpy()
    ang = synth.uniform_angles(na)
    A, At = omb.radon_ops(ang, n, n)
    b = A(vol) + 0.01 * rng.standard_normal((nz, na, n))
    return vol, ang, A, At, b


def test_autograd_gradient_vs_oracle(dev):
    """P11: autograd gradient of 1/2||Rx-b||^2 + H(x) on a 32x32x4 crop vs the FP64 oracle."""
    from paper_2304_12934_amd import DataFidelityFn, Plan, Prior, QGGMRFFn, RadonFn
    say("case: autograd gradient 4x32x32, 256 angles")
    vol, ang, A, At, b = _crop_problem()
    x = np.random.default_rng(31).uniform(0, 1, vol.shape)
    plan = Plan.uniform_stack(32, 32, ang, 4, device=dev)
    prior = Prior(lam=1.0)
    bt = gpu(b, dev)
    ref = omb.gradient(x, b, A, At, omb.Prior(lam=1.0))
    # fused data term
    xt = gpu(x, dev).requires_grad_(True)
    loss = DataFidelityFn.apply(xt, plan, bt) + QGGMRFFn.apply(xt, prior)
    loss.backward()
    assert rel(xt.grad.cpu().numpy(), ref) < 1e-5
    assert abs(float(loss) - omb.objective(x, b, A, omb.Prior(lam=1.0))) / float(loss) < 1e-5
    # the same graph built from RadonFn and torch arithmetic
    xt2 = gpu(x, dev).requires_grad_(True)
    r = RadonFn.apply(xt2, plan) - bt
    loss2 = 0.5 * (r.double() ** 2).sum() + QGGMRFFn.apply(xt2, prior)
    loss2.backward()
    assert rel(xt2.grad.cpu().numpy(), ref) < 1e-5


def test_mbir_step_matches_oracle_iterates(dev):
    from paper_2304_12934_amd import MBIR, Plan, Prior
    say("case: mbir_step vs oracle, 3x32x32, 48 angles, 8 iterations")
    rng = np.random.default_rng(40)
    n, nz, na = 32, 3, 48
    vol = synth.rasterize_ellipsoids(synth.ellipsoid_params(rng, n, nz, 4), n, nz).numpy()
    ang = synth.uniform_angles(na)
    A, At = omb.radon_ops(ang, n, n)
    b = A(vol) + 0.01 * rng.standard_normal((nz, na, n))
    oprior = omb.Prior(p=1.2, sigma=1.0, c=0.01, lam=0.5)
    L = omb.power_lipschitz(A, At, vol.shape, iters=60) + oprior.lipschitz()
    ref = omb.State(np.zeros(vol.shape), np.zeros(vol.shape))
    plan = Plan.uniform_stack(n, n, ang, nz, device=dev)
    m = MBIR(plan, gpu(b, dev), Prior(p=1.2, sigma=1.0, c=0.01, lam=0.5), L)
    for k in range(8):
        ref = omb.step(ref, b, A, At, oprior, L)
        m.step()
        assert rel(m.x.cpu().numpy(), ref.x) < 1e-5, k
        assert abs(float(m.state[0].item()) - ref.t) < 1e-12
    assert m.restarts == ref.restarts
    assert not m.nonfinite


def test_plain_and_autograd_paths_agree(dev):
    from paper_2304_12934_amd import MBIR, Plan, Prior, power_lipschitz
    say("case: plain vs autograd MBIR, 6x64x64, 90 angles, 15 iterations")
    rng = np.random.default_rng(41)
    n, nz, na = 64, 6, 90
    vol = synth.rasterize_ellipsoids(synth.ellipsoid_params(rng, n, nz, 6), n, nz).numpy()
    plan = Plan.uniform_stack(n, n, synth.uniform_angles(na), nz, device=dev)
    b = plan.fwd(gpu(vol, dev))
    prior = Prior(lam=0.05, c=0.01, sigma=1.0)
    L = power_lipschitz(plan, 40) + prior.lipschitz()
    m1 = MBIR(plan, b, prior, L)
    m2 = MBIR(plan, b, prior, L)
    for _ in range(15):
        m1.step()
        m2.step_autograd()
    x1, x2 = m1.x.cpu().numpy(), m2.x.cpu().numpy()
    assert rel(x2, x1) < 1e-5
    e1 = rel(x1, vol)
    assert e1 < 0.9 and math.isfinite(e1)


def test_nonfinite_data_sets_the_flag(dev):
    from paper_2304_12934_amd import MBIR, Plan, Prior
    say("case: NaN in the data")
    plan = Plan.uniform_stack(32, 32, synth.uniform_angles(16), 2, device=dev)
    b = torch.zeros(plan.sino_shape(), dtype=torch.float32, device=dev)
    b[1, 3, 7] = float("nan")
    m = MBIR(plan, b, Prior(lam=0.0), 100.0)
    m.step()
    assert m.nonfinite


@pytest.mark.parametrize("restart,monotone,frac", [(True, True, 1.0), (False, False, 1.0), (True, True, 0.8)])
def test_mbir_step_flags_match_oracle_iterates(dev, restart, monotone, frac):
    """mbir_step with the restart test on or off and the monotone rejection
    test, against the oracle's iterates; frac < 1 takes a step longer than
    1/L so that the monotone test rejects some steps."""
    from paper_2304_12934_amd import MBIR, Plan, Prior
    say(f"case: mbir_step restart={restart} monotone={monotone} L x {frac}")
    rng = np.random.default_rng(42)
    n, nz, na = 32, 3, 48
    vol = synth.rasterize_ellipsoids(synth.ellipsoid_params(rng, n, nz, 4), n, nz).numpy()
    ang = synth.uniform_angles(na)
    A, At = omb.radon_ops(ang, n, n)
    b = A(vol) + 0.01 * rng.standard_normal((nz, na, n))
    oprior = omb.Prior(p=1.2, sigma=1.0, c=0.01, lam=0.5)
    L = frac * (omb.power_lipschitz(A, At, vol.shape, iters=60) + oprior.lipschitz())
    ref = omb.State(np.zeros(vol.shape), np.zeros(vol.shape))
    plan = Plan.uniform_stack(n, n, ang, nz, device=dev)
    m = MBIR(plan, gpu(b, dev), Prior(p=1.2, sigma=1.0, c=0.01, lam=0.5), L, restart=restart, monotone=monotone)
    for k in range(12):
        ref = omb.step(ref, b, A, At, oprior, L, restart=restart, monotone=monotone)
        m.step()
        assert rel(m.x.cpu().numpy(), ref.x) < 1e-5, k
        assert abs(float(m.state[0].item()) - ref.t) < 1e-12, k
        if monotone:
            assert abs(m.objective - ref.phi) / ref.phi < 1e-5, k
    assert m.restarts == ref.restarts and m.rejected == ref.rejected
    say(f"restarts {m.restarts}, rejected {m.rejected}")


def test_power_iteration_and_step_size_in_the_library(dev):
    """nr_power_lipschitz against the largest singular value of the explicit
    matrix (squared), and the step size of nr_mbir_params."""
    from oracle import radon as ora
    from paper_2304_12934_amd import MBIR, Plan, Prior, power_lipschitz
    say("case: power iteration 2 x 16^2, 24 angles")
    n, na = 16, 24
    ang = synth.uniform_angles(na, offset=0.1)
    top = np.linalg.svd(ora.radon_matrix(n, ang, n), compute_uv=False)[0] ** 2
    plan = Plan.uniform_stack(n, n, ang, 2, device=dev)
    lr = power_lipschitz(plan, iters=300, safety=1.0)
    assert abs(lr - top) / top < 1e-5
    assert abs(power_lipschitz(plan, iters=300, safety=1.25) / lr - 1.25) < 1e-6
    prior = Prior(lam=0.3)
    m = MBIR(plan, torch.zeros(plan.sino_shape(), device=dev), prior, L_data=lr)
    assert abs(m.params.inv_L - 1.0 / (lr + omb.Prior(lam=0.3).lipschitz())) < 1e-6 * m.params.inv_L
