"""Parity at the benchmark's full size: 2560 x 2560 slices, 1024 angles, 2560 bins.

The FP64 oracle is evaluated on sampled angles (its cost is linear in the
angle count) or on sampled pixels (the closed form costs N_theta N_t per
pixel); properties that hold at any size (mass conservation per angle) are
checked on every angle.  The dense adjoint cases put data on every angle,
so the cells around the spectrum's origin receive the low frequencies of all
1024 angles (the spreading's heaviest tiles).
"""

import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import synth
from oracle import radon as ora
from tests.analytic import ellipse_projection

pytestmark = pytest.mark.gpu
TOL = 1e-5
N, NA = 2560, 1024
SAMPLE = np.arange(0, NA, 64)          # 16 angles: a = 0, 64, ..., 960


def adj_entries(y, ang, n, pixels):
    """oracle.radon_adj_entries over chunks of pixels on host threads (numpy
    releases the GIL inside its array operations)."""
    chunks = [pixels[i::16] for i in range(16)]
    with ThreadPoolExecutor(16) as ex:
        parts = list(ex.map(lambda c: ora.radon_adj_entries(y, ang, n, c), chunks))
    out = np.empty(len(pixels))
    for i, part in enumerate(parts):
        out[i::16] = part
    return out


def sample_pixels(seed, n, block):
    """A block x block square at the centre and 48 pixels drawn over the inscribed disc."""
    c = n // 2
    px = [(c - block // 2 + i, c - block // 2 + j) for i in range(block) for j in range(block)]
    rng = np.random.default_rng(seed)
    while len(px) < block * block + 48:
        iy, ix = rng.integers(0, n, 2)
        if (iy - c) ** 2 + (ix - c) ** 2 < (0.45 * n) ** 2:
            px.append((int(iy), int(ix)))
    return px


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def setup():
    from paper_2304_12934_amd import Plan
    print("case: 2560^2, 1024 angles, 20 ellipses", flush=True)
    dev = torch.device("cuda", 0)
    ang = synth.uniform_angles(NA)
    f = synth.ellipse_phantom(2, 0, N, 20).numpy()
    plan = Plan.uniform_stack(N, N, ang, 1, device=dev)
    return dev, ang, f, plan


def test_forward_sampled_angles(setup):
    dev, ang, f, plan = setup
    s = plan.fwd(torch.as_tensor(f[None], dtype=torch.float32, device=dev)).cpu().numpy()[0]
    sys.stdout.flush()
    ref = ora.radon_fwd(f, ang[SAMPLE], N)
    e = rel(s[SAMPLE], ref)
    print(f"fwd rel L2 on {len(SAMPLE)} angles: {e:.3e}", flush=True)
    assert e < TOL
    # every angle conserves mass: sum_m s[a, m] = sum f
    mass = s.astype(np.float64).sum(axis=1)
    assert np.abs(mass - f.sum()).max() / f.sum() < TOL


def test_adjoint_sampled_angles(setup):
    dev, ang, f, plan = setup
    rng = np.random.default_rng(7)
    y = np.zeros((NA, N))
    y[SAMPLE] = rng.standard_normal((len(SAMPLE), N))
    g = plan.adj(torch.as_tensor(y[None], dtype=torch.float32, device=dev)).cpu().numpy()[0]
    ref = ora.radon_adj(y[SAMPLE], ang[SAMPLE], N)
    e = rel(g, ref)
    print(f"adj rel L2 (y on {len(SAMPLE)} angles): {e:.3e}", flush=True)
    assert e < TOL


@pytest.mark.parametrize("kind", ["ellipse projections", "random"])
def test_adjoint_dense_sampled_pixels(setup, kind):
    """Adjoint of data on all 1024 angles: the analytic projections of an
    ellipse phantom (non-negative, dominated by low frequencies) and white
    noise, against the closed form on a 16 x 16 block at the centre and 48
    pixels over the disc."""
    dev, ang, f, plan = setup
    print(f"case: dense adjoint, {kind}, 2560^2, 1024 angles", flush=True)
    if kind == "random":
        y = np.random.default_rng(11).standard_normal((NA, N))
    else:
        params = synth.ellipse_params(synth.rng_for(2, 5), N, 20)
        y = ellipse_projection(params, ang, ora.pixel_coords(N))
    g = plan.adj(torch.as_tensor(y[None], dtype=torch.float32, device=dev)).cpu().numpy()[0]
    px = sample_pixels(12, N, 16)
    ref = adj_entries(y, ang, N, px)
    got = np.array([g[iy, ix] for iy, ix in px])
    e = rel(got, ref)
    e_c = rel(got[:256], ref[:256])
    print(f"dense adj rel L2 ({kind}): {e:.3e} on {len(px)} pixels, centre block {e_c:.3e}", flush=True)
    assert e < TOL and e_c < TOL


def test_2048_forward_and_adjoint_sampled():
    """2048^2 slices (4096-point grid transforms), 512 angles, sampled against the oracle."""
    from paper_2304_12934_amd import Plan
    print("case: 2048^2, 512 angles, sampled fwd/adj", flush=True)
    dev = torch.device("cuda", 0)
    n, na = 2048, 512
    ang = synth.uniform_angles(na)
    f = synth.ellipse_phantom(2, 1, n, 20).numpy()
    plan = Plan.uniform_stack(n, n, ang, 1, device=dev)
    sample = np.array([0, 129, 300, 511])
    s = plan.fwd(torch.as_tensor(f[None], dtype=torch.float32, device=dev)).cpu().numpy()[0]
    e = rel(s[sample], ora.radon_fwd(f, ang[sample], n))
    print(f"2048 fwd rel L2: {e:.3e}", flush=True)
    assert e < TOL
    rng = np.random.default_rng(8)
    y = np.zeros((na, n))
    y[sample] = rng.standard_normal((len(sample), n))
    g = plan.adj(torch.as_tensor(y[None], dtype=torch.float32, device=dev)).cpu().numpy()[0]
    e = rel(g, ora.radon_adj(y[sample], ang[sample], n))
    print(f"2048 adj rel L2: {e:.3e}", flush=True)
    assert e < TOL


@pytest.mark.parametrize("n,nd,na,sample", [(4096, 4096, 96, [0, 47]), (1024, 8192, 64, [5, 40])])
def test_largest_transform_lengths_sampled(n, nd, na, sample):
    """The longest built FFT length, 8192: as the grid transform (4096^2 slices,
    G = 8192) and as the radial transform (8192 detector bins)."""
    from paper_2304_12934_amd import Plan
    print(f"case: {n}^2, {nd} bins, {na} angles, sampled fwd/adj", flush=True)
    dev = torch.device("cuda", 0)
    ang = synth.uniform_angles(na)
    f = synth.ellipse_phantom(2, 7, n, 20).numpy()
    plan = Plan.uniform_stack(n, nd, ang, 1, device=dev)
    sample = np.array(sample)
    s = plan.fwd(torch.as_tensor(f[None], dtype=torch.float32, device=dev)).cpu().numpy()[0]
    e = rel(s[sample], ora.radon_fwd(f, ang[sample], nd))
    print(f"fwd rel L2: {e:.3e}", flush=True)
    assert e < TOL
    assert np.abs(s.astype(np.float64).sum(axis=1) - f.sum()).max() / f.sum() < TOL
    y = np.zeros((na, nd))
    y[sample] = np.random.default_rng(9).standard_normal((len(sample), nd))
    g = plan.adj(torch.as_tensor(y[None], dtype=torch.float32, device=dev)).cpu().numpy()[0]
    e = rel(g, ora.radon_adj(y[sample], ang[sample], n))
    print(f"adj rel L2: {e:.3e}", flush=True)
    assert e < TOL


def test_batch_above_last_level_cache(setup):
    """Two 2560^2 slices in one batch (about 282 MB of grids, above the 256 MiB
    last-level cache, so the forward column transform and the spreading store
    their rows with non-temporal stores) against the same slices in one-slice
    batches (plain stores), and the batched forward against the oracle on
    sampled angles."""
    from paper_2304_12934_amd import Plan
    dev, ang, f, _ = setup
    print("case: 2 x 2560^2 in one batch vs one-slice batches", flush=True)
    f2 = np.stack([f, synth.ellipse_phantom(2, 3, N, 20).numpy()])
    x = torch.as_tensor(f2, dtype=torch.float32, device=dev)
    big = Plan.uniform_stack(N, N, ang, 2, device=dev, tuning={"batch_mb": 400})
    small = Plan.uniform_stack(N, N, ang, 2, device=dev, tuning={"batch_mb": 160})
    assert big.info()["batches"] == 1 and small.info()["batches"] == 2
    sb, gb = (t.cpu().numpy() for t in big.normal(x))
    ss, gs = (t.cpu().numpy() for t in small.normal(x))
    big.close()
    small.close()
    e_s, e_g = rel(sb, ss), rel(gb, gs)
    print(f"one batch vs two: fwd {e_s:.3e}, normal {e_g:.3e}", flush=True)
    # the same kernels and sums; only split tiles add in a different order
    assert e_s < 1e-6 and e_g < 1e-6
    e = rel(sb[1][SAMPLE], ora.radon_fwd(f2[1], ang[SAMPLE], N))
    print(f"batched fwd rel L2 on {len(SAMPLE)} angles: {e:.3e}", flush=True)
    assert e < TOL
