"""The uneven stack at its real sizes: 96 slices of 512^2, 1024^2 or 2048^2
with 128 to 1500 angles each (half sparse with a random offset, half
limited-view), detector width equal to the slice width.

The batched plan's captured graph is compared with its eager calls and with
a plan that runs every slice alone; four slices (one of each size and the one
with the most angles) are compared with the FP64 oracle: the forward on
sampled angles, the adjoint of seeded random data on sampled pixels.  The
persistent execution (each batch one kernel over per-XCD work queues) is
compared with the per-stage launches and with the oracle the same way, in
three batches and with the whole stack as one batch (one launch).
"""

import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import synth
from oracle import radon as ora

pytestmark = pytest.mark.gpu
TOL = 1e-5
TUNING = {"batch_mb": 2048, "streams": 2}     # three batches, as the autotuner usually picks


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def stack():
    from paper_2304_12934_amd import Plan, SliceGeometry
    say("case: uneven stack of 96 slices 512^2..2048^2, 128..1500 angles")
    dev = torch.device("cuda", 0)
    geoms = [SliceGeometry(n, n, ang) for n, ang in synth.uneven_stack(synth.rng_for(3, 0), 96)]
    plan = Plan(geoms, device=dev, tuning=TUNING)
    vol = torch.empty(plan.vol_numel, dtype=torch.float32, device=dev)
    for i, g in enumerate(geoms):
        o = plan.vol_offsets[i]
        vol[o:o + g.n * g.n] = synth.ellipse_phantom(3, i, g.n, 20, device=dev).to(torch.float32).reshape(-1)
    y = torch.as_tensor(np.random.default_rng(90).standard_normal(plan.sino_numel), dtype=torch.float32,
                        device=dev)
    # one slice of each size and the one with the most angles
    picks = [next(i for i, g in enumerate(geoms) if g.n == n) for n in (512, 1024, 2048)]
    most = int(np.argmax([len(g.angles) for g in geoms]))
    picks.append(most if most not in picks else next(i for i in range(len(geoms)) if i not in picks))
    return dev, geoms, plan, vol, y, picks


def test_graph_equals_eager_and_per_slice(stack):
    from paper_2304_12934_amd import Plan
    dev, geoms, plan, vol, y, picks = stack
    assert plan.info()["batches"] > 1
    sino = torch.empty(plan.sino_numel, dtype=torch.float32, device=dev)
    back = torch.empty(plan.vol_numel, dtype=torch.float32, device=dev)
    with plan.capture("fwd+adj", vol, sino, back) as graph:
        graph.launch()
        torch.cuda.synchronize()
        s_eager, g_eager = plan.normal(vol)
        assert torch.equal(sino, s_eager)
        assert rel(back.cpu().numpy(), g_eager.cpu().numpy()) < 1e-6
        with Plan(geoms, device=dev, tuning={"batch": 1}) as per:
            s1, g1 = per.normal(vol)
            say(f"graph vs per-slice: fwd equal {torch.equal(sino, s1)}, "
                f"adj rel {rel(back.cpu().numpy(), g1.cpu().numpy()):.2e}")
            assert torch.equal(sino, s1)          # the forward does not depend on batching
            assert rel(back.cpu().numpy(), g1.cpu().numpy()) < 1e-6


def test_forward_against_oracle(stack):
    dev, geoms, plan, vol, y, picks = stack
    sino = torch.empty(plan.sino_numel, dtype=torch.float32, device=dev)
    with plan.capture("fwd", vol, sino) as graph:
        graph.launch()
        torch.cuda.synchronize()
    s_all = sino.cpu().numpy()
    v_all = vol.cpu().numpy()
    for i in picks:
        g = geoms[i]
        na = len(g.angles)
        s = s_all[plan.sino_offsets[i]:plan.sino_offsets[i] + na * g.n_det].reshape(na, g.n_det)
        f = v_all[plan.vol_offsets[i]:plan.vol_offsets[i] + g.n * g.n].reshape(g.n, g.n).astype(np.float64)
        sample = np.array([0, na // 3, na - 1])
        e = rel(s[sample], ora.radon_fwd(f, g.angles[sample], g.n_det))
        say(f"slice {i}: {g.n}^2, {na} angles, fwd rel L2 {e:.3e}")
        assert e < TOL


def test_adjoint_against_oracle(stack):
    dev, geoms, plan, vol, y, picks = stack
    back = torch.empty(plan.vol_numel, dtype=torch.float32, device=dev)
    with plan.capture("adj", sino=y, vol_out=back) as graph:
        graph.launch()
        torch.cuda.synchronize()
    g_all = back.cpu().numpy()
    y_all = y.cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(91)
    for i in picks:
        g = geoms[i]
        na = len(g.angles)
        yi = y_all[plan.sino_offsets[i]:plan.sino_offsets[i] + na * g.n_det].reshape(na, g.n_det)
        gi = g_all[plan.vol_offsets[i]:plan.vol_offsets[i] + g.n * g.n].reshape(g.n, g.n)
        c = g.n // 2
        px = [(c - 4 + k // 8, c - 4 + k % 8) for k in range(64)]
        px += [(int(a), int(b)) for a, b in rng.integers(0, g.n, (32, 2))]
        chunks = [px[k::16] for k in range(16)]
        with ThreadPoolExecutor(16) as ex:
            parts = list(ex.map(lambda ch: ora.radon_adj_entries(yi, g.angles, g.n, ch), chunks))
        ref = np.empty(len(px))
        for k, part in enumerate(parts):
            ref[k::16] = part
        got = np.array([gi[a, b] for a, b in px])
        e = rel(got, ref)
        say(f"slice {i}: {g.n}^2, {na} angles, adj rel L2 {e:.3e} on {len(px)} pixels")
        assert e < TOL


def adj_oracle(yi, g, px):
    chunks = [px[k::16] for k in range(16)]
    with ThreadPoolExecutor(16) as ex:
        parts = list(ex.map(lambda ch: ora.radon_adj_entries(yi, g.angles, g.n, ch), chunks))
    ref = np.empty(len(px))
    for k, part in enumerate(parts):
        ref[k::16] = part
    return ref


@pytest.mark.parametrize("batch_mb", [2048, 1 << 20])
def test_persistent_equals_stages_and_oracle(stack, batch_mb):
    """radon_normal with b = R f - y gives R f - b = y and R^T y: the persistent
    pass against the per-stage pass (the forward bit-equal, the adjoint to
    float32 rounding of the spreading sums) and both halves against the oracle
    on the sampled slices (the adjoint against the oracle's transpose of the
    residual the kernels produced)."""
    from paper_2304_12934_amd import Plan
    dev, geoms, plan, vol, y, picks = stack
    v = vol * 1e-3
    s_ref = torch.empty(plan.sino_numel, dtype=torch.float32, device=dev)
    plan.fwd(v, s_ref)
    b = s_ref - y
    r_ref, g_ref = plan.normal(v, b)
    tuning = {"batch_mb": batch_mb, "streams": 2, "persistent": 1}
    with Plan(geoms, device=dev, tuning=tuning) as pp:
        info = pp.info()
        say(f"case: persistent, batch_mb {batch_mb}: {info['batches']} batches, {info['launches']} launches per pass")
        assert info["launches"] == 2 * info["batches"]
        sino = torch.empty(pp.sino_numel, dtype=torch.float32, device=dev)
        back = torch.empty(pp.vol_numel, dtype=torch.float32, device=dev)
        r_e, g_e = pp.normal(v, b)
        pp.check()
        graph = pp.capture("fwd+adj", v, sino, back)
        try:
            for _ in range(2):   # replays of the captured persistent pass
                back.zero_()
                graph.launch()
                pp.check()
                assert torch.equal(sino, s_ref)
        finally:
            graph.close()
        # the graph's forward+adjoint (no b) against the per-stage forward + adjoint
        g_plain = plan.normal(v)[1]
        e_graph = rel(back.cpu().numpy(), g_plain.cpu().numpy())
        e_fwd = torch.equal(r_e, r_ref)
        e_adj = rel(g_e.cpu().numpy(), g_ref.cpu().numpy())
        say(f"persistent vs stages: residual equal {e_fwd}, adj rel {e_adj:.2e}, graph adj rel {e_graph:.2e}")
        assert e_fwd and e_adj < 1e-6 and e_graph < 1e-6
        r_all = r_e.cpu().numpy().astype(np.float64)
        g_all = g_e.cpu().numpy()
        s_all = (r_e + b).cpu().numpy()
        v_all = v.cpu().numpy()
        rng = np.random.default_rng(92)
        for i in picks:
            g = geoms[i]
            na = len(g.angles)
            so = plan.sino_offsets[i]
            s_i = s_all[so:so + na * g.n_det].reshape(na, g.n_det)
            f = v_all[plan.vol_offsets[i]:plan.vol_offsets[i] + g.n * g.n].reshape(g.n, g.n).astype(np.float64)
            sample = np.array([0, na // 2, na - 1])
            e_f = rel(s_i[sample], ora.radon_fwd(f, g.angles[sample], g.n_det))
            yi = r_all[so:so + na * g.n_det].reshape(na, g.n_det)
            gi = g_all[plan.vol_offsets[i]:plan.vol_offsets[i] + g.n * g.n].reshape(g.n, g.n)
            c = g.n // 2
            px = [(c - 4 + k // 8, c - 4 + k % 8) for k in range(64)]
            px += [(int(a), int(bb)) for a, bb in rng.integers(0, g.n, (32, 2))]
            e_a = rel(np.array([gi[a, bb] for a, bb in px]), adj_oracle(yi, g, px))
            say(f"slice {i}: {g.n}^2, {na} angles, persistent fwd rel L2 {e_f:.3e}, adj rel L2 {e_a:.3e}")
            assert e_f < TOL and e_a < TOL
