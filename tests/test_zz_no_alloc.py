"""mbir_step_noalloc (the MBIR step whose residual sinogram lives in the
library's own per-device scratch array) against mbir_step with a caller
scratch buffer, through the C ABI: two calls in a row, the second on a
smaller problem, and the refusal of a plan whose sinogram exceeds the array."""

import ctypes
import sys

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = a.double().cpu().numpy().ravel()
    b = b.double().cpu().numpy().ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def problem(dev, n, nz, na, seed):
    from paper_2304_12934_amd import Plan
    ang = synth.uniform_angles(na)
    plan = Plan.uniform_stack(n, n, ang, nz, device=dev)
    f = np.stack([synth.ellipse_phantom(seed, z, n, 6).numpy() for z in range(nz)])
    b = plan.fwd(torch.as_tensor(f, dtype=torch.float32, device=dev))
    return plan, b


def states(dev, plan, seed):
    """x, x_prev, y, grad and the float64 state, x = y random (one warm state)."""
    from paper_2304_12934_amd._lib import NR_MBIR_STATE_DOUBLES, check, lib
    from paper_2304_12934_amd.radon import _ptr, _stream
    g = torch.Generator(device="cpu").manual_seed(seed)
    x = torch.rand(plan.vol_shape(), generator=g).to(dev)
    bufs = [x.clone(), x.clone(), x.clone(), torch.zeros_like(x)]
    st = torch.empty(NR_MBIR_STATE_DOUBLES, dtype=torch.float64, device=dev)
    check(lib().mbir_state_init(_ptr(st), _stream(dev)), "mbir_state_init")
    return bufs, st


@pytest.mark.parametrize("monotone", [0, 1])
def test_noalloc_matches_mbir_step(monotone):
    from paper_2304_12934_amd import Prior
    from paper_2304_12934_amd._lib import NrMbir, check, lib
    from paper_2304_12934_amd.radon import _ptr, _stream
    dev = torch.device("cuda", 0)
    prior = Prior(lam=0.5)
    pc = prior.as_c()
    # two calls in a row: 3 x 80^2 slices, 60 angles, then 2 x 64^2 slices, 30 angles
    for (n, nz, na, seed) in [(80, 3, 60, 1), (64, 2, 30, 2)]:
        say(f"case: mbir_step_noalloc monotone={monotone} {nz}x{n}^2, {na} angles")
        plan, b = problem(dev, n, nz, na, seed)
        params = NrMbir()
        check(lib().nr_mbir_params(ctypes.c_double(4.0 * n), ctypes.byref(pc), 1, 0, monotone,
                                   ctypes.byref(params)), "nr_mbir_params")
        (x1, xp1, y1, g1), st1 = states(dev, plan, seed)
        (x2, xp2, y2, g2), st2 = states(dev, plan, seed)
        scratch = torch.empty(plan.sino_shape(), dtype=torch.float32, device=dev)
        s = _stream(dev)
        for _ in range(2):
            check(lib().mbir_step(plan._h, ctypes.byref(pc), ctypes.byref(params), _ptr(b), _ptr(x1), _ptr(xp1),
                                  _ptr(y1), _ptr(g1), _ptr(scratch), _ptr(st1), s), "mbir_step")
            check(lib().mbir_step_noalloc(plan._h, ctypes.byref(pc), ctypes.byref(params), _ptr(b), _ptr(x2),
                                          _ptr(xp2), _ptr(y2), _ptr(g2), _ptr(st2), s), "mbir_step_noalloc")
        torch.cuda.synchronize()
        for name, u, v in (("x", x2, x1), ("x_prev", xp2, xp1), ("y", y2, y1), ("grad", g2, g1)):
            e = rel(u, v)
            say(f"  {name}: rel L2 {e:.3e}")
            assert e < 1e-5, (name, e)
        t1, t2 = st1.cpu().numpy(), st2.cpu().numpy()
        assert abs(t1[0] - t2[0]) < 1e-9 and t1[2] == 0 and t2[2] == 0
        plan.close()


def test_noalloc_refuses_oversized_sinogram():
    from paper_2304_12934_amd import Plan, Prior
    from paper_2304_12934_amd._lib import NR_INVALID_ARG, NrMbir, check, lib
    from paper_2304_12934_amd.radon import _ptr, _stream
    dev = torch.device("cuda", 0)
    say("case: mbir_step_noalloc with a 68.8 MB sinogram (2100 x 64^2, 128 angles)")
    plan = Plan.uniform_stack(64, 64, synth.uniform_angles(128), 2100, device=dev)
    pc = Prior(lam=0.5).as_c()
    params = NrMbir()
    check(lib().nr_mbir_params(ctypes.c_double(100.0), ctypes.byref(pc), 1, 0, 0, ctypes.byref(params)),
          "nr_mbir_params")
    v = torch.zeros(plan.vol_shape(), dtype=torch.float32, device=dev)
    b = torch.zeros(plan.sino_shape(), dtype=torch.float32, device=dev)
    st = torch.zeros(16, dtype=torch.float64, device=dev)
    r = lib().mbir_step_noalloc(plan._h, ctypes.byref(pc), ctypes.byref(params), _ptr(b), _ptr(v), _ptr(v),
                                _ptr(v), _ptr(v), _ptr(st), _stream(dev))
    assert r == NR_INVALID_ARG
    assert b"scratch" in lib().nr_last_error()
    plan.close()
