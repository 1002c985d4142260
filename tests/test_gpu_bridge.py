"""Parity of the bridging of mask-separated regions (Section II-D) between
the HIP kernels and the oracle, through the C ABI: region numbers, the
bridged cycle counts and phi, bit for bit."""
import numpy as np
import pytest

import oracle
from paper_2609_36267_amd import binding as ww
from paper_2609_36267_amd import synth
from tests.helpers import np_

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    ww.load()
    return torch


def smooth_truth(m, n, seed):
    rng = np.random.default_rng(seed)
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    true = 0.02 * j + 0.01 * i + 1.5 * np.sin(i / 17.0) + rng.uniform(-40, 40)
    psi = np.angle(np.exp(1j * true)).astype(np.float32)
    Kt = np.round((true - psi.astype(np.float64)) / (2 * np.pi)).astype(np.int32)
    return psi, Kt


def check(psi, valid, K, h=32):
    Ko, phio, Ro = oracle.bridge(psi, valid, K, half_window=h, nodata=-9.0)
    Kg, phig, Rg, reg = ww.bridge(psi, valid, K, ww.default_bridge_params(half_window=h),
                                  nodata=-9.0, want_regions=True)
    lab, _ = oracle.regions(valid)
    assert Rg == Ro
    assert np.array_equal(np_(reg).view(np.uint32), lab)
    assert np.array_equal(np_(Kg), Ko)
    assert np_(phig).tobytes() == phio.tobytes()
    return Ko, Ro


@pytest.mark.parametrize("shape,width", [((70, 90), 6), ((64, 64), 4), ((129, 203), 8),
                                         ((300, 400), 10)])
def test_bridge_parity_offsets(torch_cuda, shape, width):
    m, n = shape
    rng = np.random.default_rng(m + n)
    valid = synth.river_mask(m, n, rng, width=width)
    psi, Kt = smooth_truth(m, n, m)
    lab, R = oracle.regions(valid)
    off = rng.integers(-9, 10, R + 1)
    K = (Kt + off[lab]).astype(np.int32)
    Kb, R2 = check(psi, valid, K)
    assert R2 == R >= 3
    d = (Kb.astype(np.int64) - Kt)[valid.astype(bool)]
    assert np.all(d == d[0])  # every region back on one level


@pytest.mark.parametrize("h", [0, 5, 32])
def test_bridge_parity_noise_and_windows(torch_cuda, h):
    rng = np.random.default_rng(40 + h)
    m, n = 97, 131
    valid = synth.river_mask(m, n, rng, width=5, lakes=9)
    psi = rng.uniform(-np.pi, np.pi, (m, n)).astype(np.float32)
    K = rng.integers(-5, 6, (m, n)).astype(np.int32)
    check(psi, valid, K, h=h)


def test_bridge_many_small_regions(torch_cuda):
    """Speckled mask: hundreds of regions, many of one pixel, equal sizes
    ranked by number."""
    rng = np.random.default_rng(5)
    m, n = 60, 75
    valid = (rng.random((m, n)) > 0.45).astype(np.uint8)
    psi = rng.uniform(-np.pi, np.pi, (m, n)).astype(np.float32)
    K = rng.integers(-3, 4, (m, n)).astype(np.int32)
    _, R = check(psi, valid, K)
    assert R > 100


def test_bridge_degenerate(torch_cuda):
    psi, Kt = smooth_truth(20, 30, 1)
    # one region: unchanged
    Kb, R = check(psi, np.ones(psi.shape, np.uint8), Kt)
    assert R == 1 and np.array_equal(Kb, Kt)
    # no valid pixel
    Kb, R = check(psi, np.zeros(psi.shape, np.uint8), Kt)
    assert R == 0
    # single row and single column with gaps
    p1, k1 = smooth_truth(1, 40, 2)
    v = np.ones((1, 40), np.uint8)
    v[0, 10:12] = 0
    v[0, 25] = 0
    _, R = check(p1, v, k1 + (np.arange(40)[None, :] > 20).astype(np.int32))
    assert R == 3
    p2, k2 = smooth_truth(20, 1, 3)
    v = np.ones((20, 1), np.uint8)
    v[7, 0] = 0
    _, R = check(p2, v, k2)
    assert R == 2


def test_bridge_in_place(torch_cuda):
    import torch
    rng = np.random.default_rng(2)
    m, n = 80, 100
    valid = synth.river_mask(m, n, rng, width=6)
    psi, Kt = smooth_truth(m, n, 3)
    K = (Kt + rng.integers(-3, 4)).astype(np.int32)
    want = np_(ww.bridge(psi, valid, K)[0])
    t = torch.from_numpy(K.copy()).cuda()
    phi = torch.empty_like(t, dtype=torch.float32)
    ww.bridge(psi, valid, t, out=(t, phi))
    assert np.array_equal(np_(t), want)


def test_bridge_after_unwrap_full_path(torch_cuda):
    """ww_unwrap then ww_bridge on a river-masked 512 x 640 scene: the
    oracle's whole path and bridging give the same K and phi."""
    sc = synth.make(512, 640, looks=9, seed=11, peak=20.0, ramp=0.05)
    valid = synth.river_mask(512, 640, np.random.default_rng(11), width=8)
    K, phi, tot = ww.unwrap(sc.psi, sc.coh, valid, 9)
    out = oracle.unwrap(sc.psi, sc.coh, valid, 9, want=True)
    assert tot == out["total"]
    Ko, phio, Ro = oracle.bridge(sc.psi, valid, out["K"])
    # the GPU's K can differ from the oracle's only on uncertified pixels of
    # equal-cost optima; bridge the oracle's K on both sides for parity
    Kg, phig, Rg = ww.bridge(sc.psi, valid, out["K"])
    assert Rg == Ro and np.array_equal(np_(Kg), Ko)
    assert np_(phig).tobytes() == phio.tobytes()
