"""GPU parity of the rotation-axis offset and of radon_fbp against the FP64 oracle.

Both ride on the radial transforms: the offset is a phase on each radial
line (forward) and its conjugate (adjoint); the back-projection filter is a
real weight on the adjoint's radial line.  Tolerance: float32 relative L2
<= 1e-5, as for the plain operator.
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
    L.lib()
    return torch.device("cuda", 0)


def gpu(a, dev):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev)


@pytest.mark.parametrize("c", [2.37, -5.0, 40.5, -63.25])
def test_offset_forward_and_adjoint(dev, c):
    from paper_2304_12934_amd import Plan
    say(f"case: 128x128, 90 angles, rotation axis offset {c}")
    n = nd = 128
    ang = synth.uniform_angles(90)
    f = synth.ellipse_phantom(1, 0, n, 8).numpy()
    plan = Plan.uniform_stack(n, nd, ang, 1, center=c)
    s = plan.fwd(gpu(f[None], dev)).cpu().numpy()[0]
    e = rel(s, ora.radon_fwd(f, ang, nd, center=c))
    assert e < TOL, e
    y = np.random.default_rng(30).standard_normal((90, nd))
    g = plan.adj(gpu(y[None], dev)).cpu().numpy()[0]
    e = rel(g, ora.radon_adj(y, ang, n, center=c))
    assert e < TOL, e


def test_offsets_per_slice_in_an_uneven_stack(dev):
    """Slices with different offsets (and some sharing one) in one plan."""
    from paper_2304_12934_amd import Plan, SliceGeometry
    say("case: uneven stack, per-slice rotation axis offsets")
    rng = np.random.default_rng(31)
    spec = [(64, 64, 0.0), (80, 80, 3.5), (64, 64, -1.25), (128, 128, 3.5), (80, 80, 0.0)]
    geoms, fs, ys = [], [], []
    for i, (n, nd, c) in enumerate(spec):
        ang = rng.uniform(0, np.pi, 40 + 7 * i)
        geoms.append(SliceGeometry(n, nd, ang, c))
        fs.append(synth.ellipse_phantom(1, 10 + i, n, 6).numpy())
        ys.append(rng.standard_normal((len(ang), nd)))
    plan = Plan(geoms, device=dev)
    s = plan.fwd(gpu(np.concatenate([f.ravel() for f in fs]), dev)).cpu().numpy()
    g = plan.adj(gpu(np.concatenate([y.ravel() for y in ys]), dev)).cpu().numpy()
    for i, gm in enumerate(geoms):
        so, vo = plan.sino_offsets[i], plan.vol_offsets[i]
        si = s[so:so + len(gm.angles) * gm.n_det].reshape(len(gm.angles), gm.n_det)
        gi = g[vo:vo + gm.n * gm.n].reshape(gm.n, gm.n)
        assert rel(si, ora.radon_fwd(fs[i], gm.angles, gm.n_det, gm.center)) < TOL, i
        assert rel(gi, ora.radon_adj(ys[i], gm.angles, gm.n, gm.center)) < TOL, i


def test_offset_dot_product(dev):
    from paper_2304_12934_amd import Plan
    say("case: dot test with offset 7.3, 256x256, 97 angles")
    n, na = 256, 97
    rng = np.random.default_rng(32)
    plan = Plan.uniform_stack(n, n, rng.uniform(0, np.pi, na), 1, center=7.3)
    x = gpu(rng.standard_normal((1, n, n)), dev)
    y = gpu(rng.standard_normal((1, na, n)), dev)
    Rx = plan.fwd(x).double()
    lhs = float((Rx * y.double()).sum())
    rhs = float((x.double() * plan.adj(y).double()).sum())
    scale = float(torch.linalg.vector_norm(Rx) * torch.linalg.vector_norm(y.double()))
    assert abs(lhs - rhs) / scale < 1e-7


@pytest.mark.parametrize("filt,c", [("ramp", 0.0), ("butterworth", 0.0), ("ramp", 1.5), ("butterworth", -12.75)])
def test_fbp_against_oracle(dev, filt, c):
    from paper_2304_12934_amd import Plan
    say(f"case: fbp {filt}, 128x128, 180 angles, offset {c}")
    n = nd = 128
    ang = synth.uniform_angles(180)
    f = synth.ellipse_phantom(1, 3, n, 8).numpy()
    y = ora.radon_fwd(f, ang, nd, center=c) + 0.01 * np.random.default_rng(33).standard_normal((180, nd))
    plan = Plan.uniform_stack(n, nd, ang, 1, center=c)
    g = plan.fbp(gpu(y[None], dev), filter=filt, order=2, cutoff=0.25).cpu().numpy()[0]
    e = rel(g, ora.fbp(y, ang, n, filt=filt, order=2, cutoff=0.25, center=c))
    say(f"fbp rel L2 {e:.3e}")
    assert e < TOL


def test_fbp_rejects_bad_filters(dev):
    from paper_2304_12934_amd import Plan
    from paper_2304_12934_amd._lib import NrError
    plan = Plan.uniform_stack(32, 32, synth.uniform_angles(8), 1)
    y = torch.zeros(plan.sino_shape(), dtype=torch.float32, device=dev)
    with pytest.raises(NrError):
        plan.fbp(y, filter="butterworth", cutoff=0.0)
    with pytest.raises(NrError):
        plan.fbp(y, filter="butterworth", order=0)
    with pytest.raises(ValueError):
        plan.fbp(y, filter="hann")


def test_fbp_full_size_sampled(dev):
    """2560^2, 1024 angles: data on 4 angles only, so the oracle's FBP over those
    angles, rescaled from pi/4 to pi/1024, is the expected result."""
    from paper_2304_12934_amd import Plan
    say("case: fbp 2560^2, 1024 angles, sampled, Butterworth, offset 3.25")
    n, na = 2560, 1024
    ang = synth.uniform_angles(na)
    sample = np.array([0, 341, 682, 1023])
    plan = Plan.uniform_stack(n, n, ang, 1, center=3.25)
    y = np.zeros((na, n))
    y[sample] = np.random.default_rng(34).standard_normal((len(sample), n))
    g = plan.fbp(gpu(y[None], dev), filter="butterworth").cpu().numpy()[0]
    ref = ora.fbp(y[sample], ang[sample], n, filt="butterworth", center=3.25) * (len(sample) / na)
    e = rel(g, ref)
    say(f"fbp 2560 rel L2 {e:.3e}")
    assert e < TOL
