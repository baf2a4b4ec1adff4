"""Full sparse-view MBIR at size: 128 slices of 2560 x 2560, 361 angles in
[0, pi), 2560 bins; random ellipsoids with thin blurred cracks; Gaussian noise
of 1 % of the largest datum; 100 iterations over the whole resident stack,
the prior coupling adjacent slices.

The data are the projector's own forward of the rasterised volume plus noise
(an inverse crime, stated).  The FP64 oracle checks sampled (slice, angle)
rows of that forward; one iteration at full size is checked against the same
step composed from the separately verified entry points (forward, adjoint,
prior gradient) in FP64 on the device; the 100 iterations are checked for a
finite, decreasing objective, a data misfit at the noise level and a
reconstruction error that falls.  lambda = 300: with lambda = 1 the prior is
weak against data of this scale and the iterates fit the noise (error 0.35
after 10 iterations, 0.49 after 100); at 300 the error falls through the
whole run (0.83, 0.29, 0.16 after 10, 50, 100 iterations in a sweep of
lambda in {1, 30, 300, 3000} on this stack).
"""

import math
import sys
import time

import numpy as np
import pytest
import torch

import synth
from oracle import radon as ora

pytestmark = pytest.mark.gpu
N, NZ, NA, ITERS = 2560, 128, 361, 100
LAMBDA = 300.0
SLICES = (37, 90)
ANGLES = np.array([0, 200])


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def problem():
    from paper_2304_12934_amd import Plan, Prior, power_lipschitz
    say(f"case: sparse-view MBIR {NZ} x {N}^2, {NA} angles, 30 ellipsoids + 12 cracks")
    dev = torch.device("cuda", 0)
    t0 = time.perf_counter()
    vol64 = synth.ellipsoid_volume(5, N, NZ, 30, device=dev)
    vol = synth.add_cracks(vol64, synth.rng_for(5, 1), 12).to(torch.float32).contiguous()
    del vol64
    torch.cuda.empty_cache()
    ang = synth.uniform_angles(NA)
    plan = Plan.uniform_stack(N, N, ang, NZ, device=dev)
    b_true = plan.fwd(vol)
    b = torch.as_tensor(synth.gaussian_noise(b_true, synth.rng_for(5, 2), 0.01), dtype=torch.float32,
                        device=dev).contiguous()
    prior = Prior(lam=LAMBDA)
    L = power_lipschitz(plan, 30) + prior.lipschitz()
    torch.cuda.synchronize()
    say(f"set-up {time.perf_counter() - t0:.1f} s, L = {L:.4g}")
    return dev, ang, vol, b_true, b, plan, prior, L


def test_forward_sampled_rows(problem):
    dev, ang, vol, b_true, b, plan, prior, L = problem
    for z in SLICES:
        f = vol[z].double().cpu().numpy()
        got = b_true[z, ANGLES].double().cpu().numpy()
        e = rel(got, ora.radon_fwd(f, ang[ANGLES], N))
        say(f"slice {z}: fwd rel L2 on angles {list(ANGLES)}: {e:.3e}")
        assert e < 1e-5


def test_one_step_equals_its_composition(problem):
    """x_1 = y_0 - (R^T (R y_0 - b) + grad H(y_0)) / L from a non-zero start
    (no restart on the first step, so y_1 = x_1)."""
    from paper_2304_12934_amd import MBIR, qggmrf_grad
    dev, ang, vol, b_true, b, plan, prior, L = problem
    say("case: one mbir_step at full size vs forward + adjoint + prior composed")
    x0 = (0.9 * vol).contiguous()
    r = plan.fwd(x0) - b
    g = plan.adj(r.contiguous()).double()
    gp, _ = qggmrf_grad(x0, prior, scale=1.0, grad=torch.zeros_like(x0), value=False)
    g += gp.double()
    del r, gp
    m = MBIR(plan, b, prior, L, x0=x0)
    m.step()
    e = float(torch.linalg.vector_norm(m.grad.double() - g) / torch.linalg.vector_norm(g))
    say(f"gradient rel L2 vs composition: {e:.3e}")
    assert e < 1e-5
    # the update itself: x_1 = fl32(y_0 - grad / L), read back from the stored gradient
    want = (x0.double() - m.grad.double() / L).float()
    assert float((m.x - want).abs().max()) <= 2.0 ** -22 * float(want.abs().max())
    assert m.restarts == 0 and not m.nonfinite
    t1 = (1 + math.sqrt(5)) / 2
    assert abs(float(m.state[0].item()) - t1) < 1e-12


def test_hundred_iterations(problem):
    from paper_2304_12934_amd import MBIR, qggmrf_grad
    dev, ang, vol, b_true, b, plan, prior, L = problem
    x_ = torch.arange(N, device=dev, dtype=torch.float32) - N // 2
    mask = ((x_[None, :] ** 2 + x_[:, None] ** 2) <= (N / 2) ** 2).to(torch.float32)

    def err(x):
        return float(torch.linalg.vector_norm((x - vol) * mask) / torch.linalg.vector_norm(vol * mask))

    def misfit(x):
        r = (plan.fwd(x) - b).double()
        return 0.5 * float((r * r).sum())

    def objective(x):
        _, h = qggmrf_grad(x, prior, scale=1.0, grad=torch.zeros_like(x), value=True)
        return misfit(x) + float(h.item())

    noise = 0.5 * float(((b - b_true).double() ** 2).sum())
    m = MBIR(plan, b, prior, L)
    phi0 = objective(m.x)
    m.run(10)
    torch.cuda.synchronize()
    e10, phi10 = err(m.x), objective(m.x)
    t0 = time.perf_counter()
    m.run(40)
    torch.cuda.synchronize()
    e50 = err(m.x)
    t1 = time.perf_counter()
    m.run(ITERS - 50)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t1) + (t1 - t0)
    e100, phi100, r100 = err(m.x), objective(m.x), misfit(m.x)
    say(f"{ITERS} iterations: rel err {e10:.4f} (10) -> {e50:.4f} (50) -> {e100:.4f} ({ITERS}); objective "
        f"{phi0:.4g} -> {phi10:.4g} -> {phi100:.4g}; misfit / noise energy {r100 / noise:.3f}; "
        f"{(ITERS - 10) / dt:.2f} it/s; restarts {m.restarts}")
    assert not m.nonfinite
    assert all(math.isfinite(v) for v in (e10, e50, e100, phi10, phi100))
    assert phi100 < phi10 < phi0
    assert r100 < 2.0 * noise
    # the error falls through the run and ends well below the start's
    assert e100 <= e50 <= e10
    assert e100 < 0.25
