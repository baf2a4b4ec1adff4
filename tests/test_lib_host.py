"""Host-only checks of libnufftradon (no GPU): exports, Kaiser-Bessel tables, plan validation."""

import ctypes
import os
import re

import numpy as np
import pytest
from scipy import integrate, special

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nufftradon.h")


@pytest.fixture(scope="module")
def L():
    from paper_2304_12934_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    return _lib.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:nr_status|const char\*)\s+(\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("radon_fwd", "radon_adj", "mbir_step", "qggmrf_grad", "nr_plan_create", "nr_plan_bind"):
        assert must in names


def test_library_exports_every_declared_symbol(L):
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_signatures_cover_header():
    from paper_2304_12934_amd import _lib
    assert set(declared_functions()) <= set(_lib.SIGNATURES)


# P7 — Kaiser-Bessel kernel and its Fourier transform
@pytest.mark.parametrize("W", [6, 7, 8])
def test_kaiser_bessel_tables(L, W):
    from paper_2304_12934_amd import kb_eval
    beta = np.pi * np.sqrt((W / 2.0) ** 2 * 1.5 ** 2 - 0.8)
    u = np.linspace(-W / 2 + 1e-6, W / 2 - 1e-6, 501)
    xi = np.linspace(0.0, 0.25, 26)
    phi, phihat, poly = kb_eval(W, 0.0, u, xi)
    ref = special.i0(beta * np.sqrt(1 - (2 * u / W) ** 2)) / special.i0(beta)
    assert np.abs(phi - ref).max() < 1e-13
    # continuous Fourier transform by quadrature of the kernel itself
    f = lambda x: special.i0(beta * np.sqrt(max(0.0, 1 - (2 * x / W) ** 2))) / special.i0(beta)  # noqa: E731
    quad = np.array([integrate.quad(lambda x: f(x) * np.cos(2 * np.pi * k * x), -W / 2, W / 2,
                                    epsabs=1e-14, epsrel=1e-13, limit=200)[0] for k in xi])
    assert np.abs(phihat - quad).max() / quad.max() < 1e-11
    # device polynomial: float32 coefficients, error at float32 resolution
    assert np.abs(poly - ref).max() < 1e-7


def _slices(*rows):
    from paper_2304_12934_amd._lib import NrSlice
    arr = (NrSlice * len(rows))()
    for i, r in enumerate(rows):
        arr[i] = NrSlice(*r)
    return arr


def _create(L, rows, angles, width=7):
    from paper_2304_12934_amd._lib import NrNufft
    h = ctypes.c_void_p()
    ang = np.ascontiguousarray(angles, dtype=np.float64)
    st = L.nr_plan_create(_slices(*rows), len(rows), ang.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                          ctypes.byref(NrNufft(2.0, width, 0.0)), ctypes.byref(h))
    return st, h


def test_plan_validation_status_codes(L):
    from paper_2304_12934_amd import _lib
    ang = np.linspace(0, np.pi, 10, endpoint=False)
    assert _create(L, [(127, 128, 10, 0, 0, 0)], ang)[0] == _lib.NR_INVALID_ARG       # odd N
    assert _create(L, [(128, 6, 10, 0, 0, 0)], ang)[0] == _lib.NR_INVALID_ARG         # N_t < 8
    assert _create(L, [(128, 128, 0, 0, 0, 0)], ang)[0] == _lib.NR_INVALID_ARG        # no angles
    assert _create(L, [(48, 128, 10, 0, 0, 0)], ang)[0] == _lib.NR_UNSUPPORTED_SIZE   # G = 96
    assert _create(L, [(128, 96, 10, 0, 0, 0)], ang)[0] == _lib.NR_UNSUPPORTED_SIZE   # N_t = 96
    assert _create(L, [(128, 128, 10, 0, 0, 0)], ang, width=9)[0] == _lib.NR_UNSUPPORTED_SIZE
    # point codes (angle << ceil(log2(N_t/2 + 1))) | j must fit 31 bits: with
    # N_t = 8192 (13 bits of j) at most 2^18 - 1 angles
    many = np.linspace(0, np.pi, 1 << 18, endpoint=False)
    assert _create(L, [(128, 8192, 1 << 18, 0, 0, 0)], many)[0] == _lib.NR_UNSUPPORTED_SIZE
    bad = ang.copy()
    bad[3] = np.nan
    assert _create(L, [(128, 128, 10, 0, 0, 0)], bad)[0] == _lib.NR_INVALID_ARG
    assert L.nr_last_error()
    # an empty stack is refused (there is nothing to plan)
    h0 = ctypes.c_void_p()
    assert L.nr_plan_create(_slices((128, 128, 10, 0, 0, 0)), 0, ang.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                            None, ctypes.byref(h0)) == _lib.NR_INVALID_ARG
    # rotation-axis offset: finite and within half the detector
    assert _create(L, [(128, 128, 10, 0, 0, 0, float("nan"))], ang)[0] == _lib.NR_INVALID_ARG
    assert _create(L, [(128, 128, 10, 0, 0, 0, 64.5)], ang)[0] == _lib.NR_INVALID_ARG
    st, h = _create(L, [(128, 128, 10, 0, 0, 0, -64.0)], ang)
    assert st == _lib.NR_OK
    L.nr_plan_destroy(h)
    st, h = _create(L, [(128, 128, 10, 0, 0, 0)], ang)
    assert st == _lib.NR_OK
    # binding a NULL workspace is refused before any device work
    assert L.nr_plan_bind(h, None, 0, None) == _lib.NR_INVALID_ARG
    assert L.radon_fwd(h, ctypes.c_void_p(8), ctypes.c_void_p(8), None) == _lib.NR_INVALID_ARG  # not bound
    ramp = _lib.NrFbp(_lib.NR_FBP_RAMP, 0, 0.0)
    assert L.radon_fbp(h, ctypes.byref(ramp), ctypes.c_void_p(8), ctypes.c_void_p(8), None) == _lib.NR_INVALID_ARG
    bufs = (ctypes.c_void_p * 2)(8, 16)
    assert L.radon_stream(h, _lib.NR_STREAM_FWD, None, ctypes.c_void_p(8), ctypes.c_void_p(8), 1, bufs, bufs,
                          None) == _lib.NR_INVALID_ARG
    L.nr_plan_destroy(h)


def test_plan_info_and_workspace(L):
    from paper_2304_12934_amd import _lib
    ang = np.linspace(0, np.pi, 90, endpoint=False)
    st, h = _create(L, [(128, 128, 90, 0, 0, 0), (128, 128, 90, 128 * 128, 90 * 128, 0)], ang)
    assert st == _lib.NR_OK
    info = (ctypes.c_int64 * 8)()
    assert L.nr_plan_info(h, 1, info, 8) == _lib.NR_OK
    G, tiles, entries, items, degree, slots, batches, launches = list(info)
    assert G == 256 and degree == 9
    assert slots == 2 and batches == 1          # both small slices share one batch
    assert launches == 4 + 5                     # forward 4, adjoint 4 + the tile clear
    assert entries >= 90 * 64          # every point j >= 1 sits in at least one tile
    # every tile holding points has an item; tiles without points whose cells
    # all lie outside the disc the adjoint reads (the half-plane's corners) have none
    assert tiles // 2 <= items
    nbytes = ctypes.c_size_t()
    assert L.nr_plan_workspace_bytes(h, ctypes.byref(nbytes)) == _lib.NR_OK
    # at least the extended half-plane grid (G/2 + 1 + 8 rows of G + 8 complex)
    assert nbytes.value >= (G // 2 + 9) * (G + 8) * 8
    # tuning: one slice per batch on one stream halves the scratch; on two
    # streams each keeps its own scratch; an unknown tile is refused
    assert L.nr_plan_tune(h, b"streams", 1) == _lib.NR_OK
    assert L.nr_plan_tune(h, b"batch", 1) == _lib.NR_OK
    small = ctypes.c_size_t()
    assert L.nr_plan_workspace_bytes(h, ctypes.byref(small)) == _lib.NR_OK
    assert small.value < nbytes.value
    assert L.nr_plan_info(h, 0, info, 8) == _lib.NR_OK and info[5] == 1 and info[6] == 2
    assert L.nr_plan_tune(h, b"streams", 2) == _lib.NR_OK
    lanes = ctypes.c_size_t()
    assert L.nr_plan_workspace_bytes(h, ctypes.byref(lanes)) == _lib.NR_OK
    assert lanes.value > small.value
    assert L.nr_plan_tune(h, b"streams", 9) == _lib.NR_INVALID_ARG
    assert L.nr_plan_tune(h, b"streams", 1) == _lib.NR_OK
    assert L.nr_plan_tune(h, b"tile_w", 48) == _lib.NR_OK
    assert L.nr_plan_workspace_bytes(h, ctypes.byref(small)) == _lib.NR_UNSUPPORTED_SIZE
    assert L.nr_plan_tune(h, b"tile_w", 32) == _lib.NR_OK
    assert L.nr_plan_workspace_bytes(h, ctypes.byref(small)) == _lib.NR_OK
    assert L.nr_plan_tune(h, b"no_such_key", 1) == _lib.NR_INVALID_ARG
    # direct interpolation: one forward launch fewer (interpolation and radial pass fused)
    assert L.nr_plan_tune(h, b"interp_mode", 2) == _lib.NR_INVALID_ARG
    assert L.nr_plan_tune(h, b"interp_mode", 1) == _lib.NR_OK
    assert L.nr_plan_info(h, 0, info, 8) == _lib.NR_OK and info[7] == 2 * (3 + 5)   # two batches
    L.nr_plan_destroy(h)


def test_prior_weights_and_lipschitz_in_the_library(L):
    """nr_prior_init's weights and nr_prior_lipschitz against the oracle's readings."""
    from oracle import mbir as omb
    from oracle import qggmrf as oq
    from paper_2304_12934_amd import Prior
    from paper_2304_12934_amd._lib import NrMbir, NrPrior
    for kind, ref in (("inv_distance", oq.inverse_distance_weights()), ("gaussian", oq.gaussian_weights())):
        c = Prior(p=1.2, sigma=1.0 / 0.7, c=1e-4, lam=0.7, weights=kind).as_c()
        got = (c.w_face, c.w_edge, c.w_corner)
        assert np.allclose(got, (ref[1], ref[2], ref[3]), rtol=1e-6, atol=0)
    # float32 parameters: equal to float32 rounding
    assert abs(Prior(lam=0.7).lipschitz() - omb.Prior(lam=0.7).lipschitz()) < 1e-6 * omb.Prior(lam=0.7).lipschitz()
    with pytest.raises(ValueError):
        Prior(weights="box").as_c()
    out = NrMbir()
    pr = Prior(lam=0.5, c=0.01, sigma=1.0).as_c()
    assert L.nr_mbir_params(3.0, ctypes.byref(pr), 1, 0, 1, ctypes.byref(out)) == 0
    assert abs(out.inv_L - 1.0 / (3.0 + 8 * 0.5 / 0.01)) < 1e-9 and out.restart == 1 and out.monotone == 1
    assert L.nr_mbir_params(-1.0, None, 1, 0, 0, ctypes.byref(out)) != 0
    assert L.nr_mbir_params(2.0, None, 1, 2, 0, ctypes.byref(out)) != 0      # flags are 0 or 1
    bad = NrPrior(0.5, 1.0, 1e-4, 1.0, 0.1, 0.1, 0.1)                          # p < 1
    v = ctypes.c_double()
    assert L.nr_prior_lipschitz(ctypes.byref(bad), ctypes.byref(v)) != 0


def test_autotune_scratch_and_tuning_keys(L):
    """Host side of the autotuner: the scratch bound covers every candidate
    layout, and the tuning keys read back."""
    from paper_2304_12934_amd import _lib
    ang = np.linspace(0, np.pi, 40, endpoint=False)
    st, h = _create(L, [(128, 128, 40, 0, 0, 0), (64, 64, 40, 128 * 128, 40 * 128, 0)], ang)
    assert st == _lib.NR_OK
    need = ctypes.c_size_t()
    assert L.nr_autotune_scratch_bytes(h, ctypes.byref(need)) == _lib.NR_OK
    v = ctypes.c_int64()
    for key, want in (("tile_w", 64), ("tile_h", 32), ("chunk", 1024), ("batch_mb", 160), ("streams", 2),
                      ("autotune_us", -1), ("autotune_trials", 0)):
        assert L.nr_plan_get_tune(h, key.encode(), ctypes.byref(v)) == _lib.NR_OK and v.value == want, key
    assert L.nr_plan_get_tune(h, b"no_such_key", ctypes.byref(v)) == _lib.NR_INVALID_ARG
    for mb in (1, 160, 640, 1400, 2048):
        for ns in (1, 2, 3, 6):
            for tw, th in ((64, 32), (32, 32), (64, 64), (128, 32)):
                assert L.nr_plan_tune(h, b"batch_mb", mb) == 0 and L.nr_plan_tune(h, b"streams", ns) == 0
                assert L.nr_plan_tune(h, b"tile_w", tw) == 0 and L.nr_plan_tune(h, b"tile_h", th) == 0
                ws = ctypes.c_size_t()
                assert L.nr_plan_workspace_bytes(h, ctypes.byref(ws)) == 0
                assert ws.value + 2 * 4 * (128 * 128 + 64 * 64) + 4 * 40 * 192 <= need.value
    # without a device the tuner itself stops at its first HIP call with a status, not a crash
    L.nr_plan_destroy(h)


def test_host_mbir_work_area(L):
    """mbir_stream_work_bytes: two input sets of 2 (nz + 2) slices and one chunk
    of data, the extended y and prior gradient, the gradient, the residual and
    two output chunks, each 256-byte aligned; uneven plans are refused."""
    from paper_2304_12934_amd import _lib
    n, na, nz = 128, 90, 3
    ang = np.linspace(0, np.pi, na, endpoint=False)
    st, h = _create(L, [(n, n, na, z * n * n, z * na * n, 0) for z in range(nz)], ang)
    assert st == _lib.NR_OK
    got = ctypes.c_size_t()
    assert L.mbir_stream_work_bytes(h, ctypes.byref(got)) == _lib.NR_OK

    def a(v):
        return (v + 255) // 256 * 256

    ext, vol, sino = 4 * (nz + 2) * n * n, 4 * nz * n * n, 4 * nz * na * n
    assert got.value == 2 * (2 * a(ext) + a(sino)) + 2 * a(ext) + a(vol) + a(sino) + 2 * a(vol)
    assert L.mbir_stream_work_bytes(h, None) == _lib.NR_INVALID_ARG
    L.nr_plan_destroy(h)
    st, h = _create(L, [(n, n, na, 0, 0, 0), (64, 64, na, n * n, na * n, 0)], ang)
    assert st == _lib.NR_OK
    assert L.mbir_stream_work_bytes(h, ctypes.byref(got)) == _lib.NR_INVALID_ARG
    L.nr_plan_destroy(h)
