"""GPU parity of the host-resident MBIR iteration (mbir_stream_iterate): against
the FP64 oracle's iterates and against the device-resident mbir_step."""

import sys

import numpy as np
import pytest
import torch

import synth
from oracle import mbir as omb

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


def pinned(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32).contiguous().pin_memory()


def test_host_mbir_matches_oracle_iterates(dev):
    """6 slices of 32^2 streamed as 3 chunks of 2 (every chunk has a halo on
    at least one side), 8 iterations against the oracle's loop over the whole
    volume (the prior couples the chunks)."""
    from paper_2304_12934_amd import HostMBIR, Plan, Prior
    say("case: host MBIR vs oracle, 3 chunks x 2 slices of 32^2, 48 angles, 8 iterations")
    rng = np.random.default_rng(60)
    n, nzc, chunks, na = 32, 2, 3, 48
    nz = nzc * chunks
    vol = synth.rasterize_ellipsoids(synth.ellipsoid_params(rng, n, nz, 5), n, nz).numpy()
    ang = synth.uniform_angles(na)
    A, At = omb.radon_ops(ang, n, n)
    b = A(vol) + 0.01 * rng.standard_normal((nz, na, n))
    oprior = omb.Prior(p=1.2, sigma=1.0, c=0.01, lam=0.5)
    L = omb.power_lipschitz(A, At, vol.shape, iters=60) + oprior.lipschitz()
    ref = omb.State(np.zeros(vol.shape), np.zeros(vol.shape))
    plan = Plan.uniform_stack(n, n, ang, nzc, device=dev)
    m = HostMBIR(plan, pinned(b).reshape(-1), chunks, Prior(p=1.2, sigma=1.0, c=0.01, lam=0.5), L=L)
    for k in range(8):
        ref = omb.step(ref, b, A, At, oprior, L)
        m.step()
        assert rel(m.x.numpy(), ref.x) < 1e-5, k
        assert abs(float(m.state[0].item()) - ref.t) < 1e-12
    assert m.restarts == ref.restarts
    assert not m.nonfinite


@pytest.mark.parametrize("nzc,chunks,nonneg", [(3, 4, False), (1, 5, True), (6, 1, False)])
def test_host_mbir_equals_device_mbir(dev, nzc, chunks, nonneg):
    """The streamed iteration against mbir_step on the whole volume held on
    the device: one-slice chunks (halo slices on both sides), a single chunk,
    and the nonneg clamp; 10 iterations of Poisson data."""
    from paper_2304_12934_amd import MBIR, HostMBIR, Plan, Prior, power_lipschitz
    n, na = 64, 90
    nz = nzc * chunks
    say(f"case: host vs device MBIR, {chunks} chunks x {nzc} slices of {n}^2, nonneg={nonneg}")
    rng = np.random.default_rng(61 + nzc)
    vol = synth.rasterize_ellipsoids(synth.ellipsoid_params(rng, n, nz, 6), n, nz)
    ang = synth.uniform_angles(na)
    full = Plan.uniform_stack(n, n, ang, nz, device=dev)
    b_true = full.fwd(vol.to(dev).to(torch.float32).contiguous())
    b = torch.as_tensor(synth.poisson_log_data(b_true * (2.0 / float(b_true.max())), rng, 1.0e4),
                        dtype=torch.float32).contiguous()
    prior = Prior(lam=0.2, c=0.01, sigma=1.0)
    ld = power_lipschitz(full, 40)
    m_dev = MBIR(full, b.to(dev), prior, L_data=ld, nonneg=nonneg)
    chunk = Plan.uniform_stack(n, n, ang, nzc, device=dev)
    m_host = HostMBIR(chunk, b.reshape(-1).pin_memory(), chunks, prior, L_data=ld, nonneg=nonneg)
    assert abs(m_host.params.inv_L - m_dev.params.inv_L) == 0.0
    for k in range(10):
        m_dev.step()
        m_host.step()
        e = rel(m_host.x.numpy(), m_dev.x.cpu().numpy())
        assert e < 1e-5, (k, e)
    assert m_host.restarts == m_dev.restarts
    assert not m_host.nonfinite


def test_host_mbir_errors(dev):
    import ctypes

    from paper_2304_12934_amd import HostMBIR, Plan, Prior
    from paper_2304_12934_amd._lib import NR_INVALID_ARG, NrMbir, lib
    say("case: host MBIR error paths")
    n, na = 32, 16
    plan = Plan.uniform_stack(n, n, synth.uniform_angles(na), 2, device=dev)
    b = torch.zeros(2 * plan.sino_numel, dtype=torch.float32).pin_memory()
    with pytest.raises(ValueError):
        HostMBIR(plan, b[:-1], 2, Prior(), L=10.0)
    m = HostMBIR(plan, b, 2, Prior(), L=10.0)
    p = NrMbir(m.params.inv_L, 1, 0, 1)     # monotone is not supported
    st = torch.cuda.current_stream(dev).cuda_stream
    x = m._x
    args = (plan._h, ctypes.byref(m._prior_c), ctypes.byref(p), 2, ctypes.c_void_p(b.data_ptr()),
            ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(m._x_prev.data_ptr()),
            ctypes.c_void_p(m._x_next.data_ptr()), ctypes.c_void_p(m.work.data_ptr()), m.work.numel(),
            ctypes.c_void_p(m.state.data_ptr()), ctypes.c_void_p(st))
    assert lib().mbir_stream_iterate(*args) == NR_INVALID_ARG
    small = list(args)
    small[2] = ctypes.byref(m.params)
    small[9] = m.work.numel() - 1
    assert lib().mbir_stream_iterate(*small) != 0          # work area too small
    alias = list(args)
    alias[2] = ctypes.byref(m.params)
    alias[7] = ctypes.c_void_p(x.data_ptr())               # output aliases x_k
    assert lib().mbir_stream_iterate(*alias) == NR_INVALID_ARG
    m.step()                                                # still usable
    assert not m.nonfinite
