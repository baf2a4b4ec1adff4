"""GPU parity of radon_fwd / radon_adj (HIP, through the C ABI) against the FP64 oracle.

Tolerance: float32 relative L2 <= 1e-5 against the FP64 direct non-uniform
DFT, with the Kaiser-Bessel kernel of width 7 on a 2x oversampled grid.
"""

import sys

import numpy as np
import pytest
import torch

import synth
from oracle import radon as ora

pytestmark = pytest.mark.gpu
TOL = 1e-5


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
    L.lib()  # fails loudly when the library is missing
    return torch.device("cuda", 0)


def gpu(a, dev):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev)


def test_config1_forward_and_adjoint(dev):
    from paper_2304_12934_amd import Plan
    say("case: 128x128, 90 angles, 8 ellipses (fwd+adj)")
    n, nd = 128, 128
    ang = synth.uniform_angles(90)
    f = synth.ellipse_phantom(1, 0, n, 8).numpy()
    plan = Plan.uniform_stack(n, nd, ang, 1)
    s = plan.fwd(gpu(f[None], dev)).cpu().numpy()[0]
    ref = ora.radon_fwd(f, ang, nd)
    assert rel(s, ref) < TOL, rel(s, ref)
    y = np.random.default_rng(1).standard_normal((90, nd))
    g = plan.adj(gpu(y[None], dev)).cpu().numpy()[0]
    gref = ora.radon_adj(y, ang, n)
    assert rel(g, gref) < TOL, rel(g, gref)


def test_dot_product_gpu(dev):
    from paper_2304_12934_amd import Plan
    say("case: dot test 256x256, 97 angles")
    rng = np.random.default_rng(2)
    n, nd, na = 256, 256, 97
    ang = rng.uniform(0, np.pi, na)
    plan = Plan.uniform_stack(n, nd, ang, 1)
    x = rng.standard_normal((1, n, n)).astype(np.float32)
    y = rng.standard_normal((1, na, nd)).astype(np.float32)
    Rx = plan.fwd(gpu(x, dev)).cpu().numpy().astype(np.float64)
    Rty = plan.adj(gpu(y, dev)).cpu().numpy().astype(np.float64)
    lhs = np.sum(Rx * y.astype(np.float64))
    rhs = np.sum(x.astype(np.float64) * Rty)
    assert abs(lhs - rhs) / abs(lhs) < 1e-6, (lhs, rhs)


GEOMS = [
    # (n, n_det, n_angles, angle set)
    (16, 16, 7, "uniform"),
    (8, 16, 3, "random2pi"),
    (64, 80, 33, "random2pi"),
    (80, 64, 17, "limited"),
    (160, 160, 45, "sparse"),
    (32, 128, 1, "random2pi"),
    (256, 320, 64, "uniform"),
]


def _angles(kind, na, rng):
    if kind == "uniform":
        return synth.uniform_angles(na)
    if kind == "random2pi":
        return rng.uniform(0, 2 * np.pi, na)
    if kind == "limited":
        return synth.limited_view_angles(rng, na)
    return synth.sparse_angles(rng, na)


@pytest.mark.parametrize("n,nd,na,kind", GEOMS)
def test_geometries_against_oracle(dev, n, nd, na, kind):
    from paper_2304_12934_amd import Plan
    say(f"case: n={n} n_det={nd} angles={na} ({kind})")
    rng = np.random.default_rng(n * 1000 + nd + na)
    ang = _angles(kind, na, rng)
    plan = Plan.uniform_stack(n, nd, ang, 2)
    f = rng.standard_normal((2, n, n))
    y = rng.standard_normal((2, na, nd))
    s = plan.fwd(gpu(f, dev)).cpu().numpy()
    g = plan.adj(gpu(y, dev)).cpu().numpy()
    for z in range(2):
        assert rel(s[z], ora.radon_fwd(f[z], ang, nd)) < TOL
        assert rel(g[z], ora.radon_adj(y[z], ang, n)) < TOL


def test_uneven_stack_in_one_plan(dev):
    from paper_2304_12934_amd import Plan, SliceGeometry
    say("case: uneven stack (3 geometries)")
    rng = np.random.default_rng(3)
    geoms = [SliceGeometry(64, 64, synth.uniform_angles(21)),
             SliceGeometry(128, 160, rng.uniform(0, np.pi, 40)),
             SliceGeometry(32, 32, synth.limited_view_angles(rng, 9))]
    plan = Plan(geoms)
    fs = [rng.standard_normal((g.n, g.n)) for g in geoms]
    ys = [rng.standard_normal((len(g.angles), g.n_det)) for g in geoms]
    s = plan.fwd(gpu(np.concatenate([f.ravel() for f in fs]), dev)).cpu().numpy()
    g_all = plan.adj(gpu(np.concatenate([y.ravel() for y in ys]), dev)).cpu().numpy()
    for i, g in enumerate(geoms):
        so, vo = plan.sino_offsets[i], plan.vol_offsets[i]
        si = s[so:so + len(g.angles) * g.n_det].reshape(len(g.angles), g.n_det)
        gi = g_all[vo:vo + g.n * g.n].reshape(g.n, g.n)
        assert rel(si, ora.radon_fwd(fs[i], g.angles, g.n_det)) < TOL
        assert rel(gi, ora.radon_adj(ys[i], g.angles, g.n)) < TOL


def test_tiled_spread_matches_atomic_spread(dev):
    from paper_2304_12934_amd import Plan
    say("case: spread tiles vs atomics, 512x512, 300 angles")
    rng = np.random.default_rng(4)
    n, na = 512, 300
    ang = rng.uniform(0, np.pi, na)
    plan = Plan.uniform_stack(n, n, ang, 1)
    y = gpu(rng.standard_normal((1, na, n)), dev)
    a = plan.adj(y).cpu().numpy()
    plan.tune("spread_mode", 1)
    b = plan.adj(y).cpu().numpy()
    plan.tune("spread_mode", 0)
    assert rel(a, b) < 1e-6


def test_repeat_calls_are_stable(dev):
    from paper_2304_12934_amd import Plan
    say("case: repeated calls")
    rng = np.random.default_rng(5)
    plan = Plan.uniform_stack(128, 128, synth.uniform_angles(64), 3)
    x = gpu(rng.standard_normal((3, 128, 128)), dev)
    s1 = plan.fwd(x).clone()
    s2 = plan.fwd(x)
    assert torch.equal(s1, s2)
    g1 = plan.adj(s1).clone()
    g2 = plan.adj(s1)
    assert rel(g1.cpu().numpy(), g2.cpu().numpy()) < 1e-6


def test_error_paths(dev):
    from paper_2304_12934_amd import Plan
    from paper_2304_12934_amd._lib import NrError
    say("case: error paths")
    plan = Plan.uniform_stack(32, 32, synth.uniform_angles(8), 1)
    with pytest.raises(TypeError):
        plan.fwd(torch.zeros((1, 32, 32), dtype=torch.float64, device=dev))
    with pytest.raises(ValueError):
        plan.fwd(torch.zeros((1, 16, 16), dtype=torch.float32, device=dev))
    with pytest.raises(NrError):
        Plan.uniform_stack(48, 48, synth.uniform_angles(8), 1)
