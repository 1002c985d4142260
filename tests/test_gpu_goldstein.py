"""Parity of the Goldstein preprocessing (Section II-D) between the HIP
kernels and the oracle, through the C ABI.

The filter runs in FP32 on the GPU and in FP64 in the oracle, so the
filtered phase is compared within a bound set by the conditioning of the
argument: an absolute error e in the complex sum S moves its phase by at
most e / |S|.  The kernels' FP32 error in S stays below 3e-6 for unit
phasors and patches up to 64 (radix-2 transforms of log2(N^2) stages with
rounding 2^-24 per operation, plus the power and the taper), so each pixel
must satisfy |dphi| <= 3e-6 / |S| + 2e-7 (the last term for the rounding
of the float32 output); pixels with |S| < 1e-3 (ill-conditioned, a handful
per scene) are counted but not compared.

The cycle-count transfer is integer work and is compared bit for bit, as is
the whole filtered path when both sides start from the oracle's filtered
phase.  ww_unwrap_filtered is checked against the composition of the three
GPU entry points it fuses."""
import math

import numpy as np
import pytest

import oracle
from paper_2609_36267_amd import binding as ww
from paper_2609_36267_amd import synth
from tests.helpers import np_

pytestmark = pytest.mark.gpu

E_ABS = 3e-6
E_OUT = 2e-7
S_MIN = 1e-3


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    ww.load()
    return torch


def noisy_scene(seed, m, n, sigma=0.8, mask=0.1):
    rng = np.random.default_rng(seed)
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    clean = 0.21 * j + 0.13 * i + 3.0 * np.sin(i / 11.0) * np.cos(j / 13.0)
    psi = np.angle(np.exp(1j * (clean + rng.normal(0, sigma, (m, n))))).astype(np.float32)
    valid = (rng.random((m, n)) > mask).astype(np.uint8)
    return psi, valid


def wrapdiff(a, b):
    return np.angle(np.exp(1j * (np.asarray(a, np.float64) - np.asarray(b, np.float64))))


def compare_filter(psi, valid, **kw):
    f_o, S = oracle.goldstein(psi, valid, want_sum=True, **kw)
    p = ww.default_filter_params(**kw)
    f_g = np_(ww.goldstein_filter(psi, valid, p))
    v = np.ones(psi.shape, bool) if valid is None else valid.astype(bool)
    assert np.array_equal(f_g[~v], psi[~v])  # invalid pixels keep psi, bit for bit
    mag = np.abs(S)
    ok = v & (mag >= S_MIN)
    err = np.abs(wrapdiff(f_g, f_o))
    bound = E_ABS / np.maximum(mag, S_MIN) + E_OUT
    worst = float((err[ok] / bound[ok]).max()) if ok.any() else 0.0
    print(f"filter {psi.shape} {kw}: worst err/bound {worst:.3f}, "
          f"ill-conditioned {int((v & ~ok).sum())}", flush=True)
    assert worst <= 1.0
    assert int((v & ~ok).sum()) <= max(3, v.sum() // 1000)
    return f_g, f_o


@pytest.mark.parametrize("shape", [(1, 1), (3, 70), (37, 45), (65, 97), (130, 257)])
def test_filter_parity_shapes(torch_cuda, shape):
    psi, valid = noisy_scene(shape[0] * 7 + shape[1], *shape)
    compare_filter(psi, valid)


@pytest.mark.parametrize("patch", [16, 32, 64])
@pytest.mark.parametrize("smooth", [1, 3, 5])
def test_filter_parity_patch_and_smoothing(torch_cuda, patch, smooth):
    psi, valid = noisy_scene(patch + smooth, 90, 141)
    compare_filter(psi, valid, patch=patch, smooth=smooth, alpha=0.7)


@pytest.mark.parametrize("alpha", [0.0, 0.25, 1.0, 2.5])
def test_filter_parity_alpha(torch_cuda, alpha):
    psi, valid = noisy_scene(int(alpha * 8) + 3, 77, 96)
    f_g, _ = compare_filter(psi, valid, alpha=alpha)
    if alpha == 0.0:  # the identity
        v = valid.astype(bool)
        assert np.abs(wrapdiff(f_g, psi)[v]).max() < 1e-5


def test_filter_without_mask_and_all_invalid(torch_cuda):
    psi, _ = noisy_scene(4, 64, 64)
    compare_filter(psi, None)
    zero = np.zeros(psi.shape, np.uint8)
    assert np.array_equal(np_(ww.goldstein_filter(psi, zero)), psi)


def test_filter_in_place(torch_cuda):
    import torch
    psi, valid = noisy_scene(8, 50, 83)
    want = np_(ww.goldstein_filter(psi, valid))
    t = torch.from_numpy(psi.copy()).cuda()
    ww.goldstein_filter(t, valid, out=t)
    assert np.array_equal(np_(t), want)


def test_filter_c0_scene(torch_cuda):
    sc = synth.config("c0", keep_truth=False)
    compare_filter(sc.psi, sc.valid)


def test_filter_bad_params(torch_cuda):
    psi, valid = noisy_scene(1, 8, 8)
    for kw in (dict(patch=24), dict(smooth=2), dict(alpha=-0.5), dict(alpha=5.0)):
        with pytest.raises(ww.WWError):
            ww.goldstein_filter(psi, valid, ww.default_filter_params(**kw))


# ---------------------------------------------------------- cycle transfer ---

@pytest.mark.parametrize("ref", [None, (0, 0), (13, 7)])
@pytest.mark.parametrize("masked", [False, True])
def test_transfer_parity(torch_cuda, ref, masked):
    rng = np.random.default_rng(31)
    m, n = 47, 66
    psi = rng.uniform(-np.pi, np.pi, (m, n)).astype(np.float32)
    psi_f = np.angle(np.exp(1j * (psi + rng.normal(0, 1.5, (m, n))))).astype(np.float32)
    # differences at and around +-pi exactly
    psi[0, :4] = np.float32(np.pi)
    psi_f[0, :4] = np.float32(-np.pi), np.float32(0.0), np.nextafter(np.float32(0), 1), np.float32(np.pi)
    K_f = rng.integers(-6, 7, (m, n)).astype(np.int32)
    valid = (rng.random((m, n)) > 0.2).astype(np.uint8) if masked else None
    K_o, phi_o = oracle.transfer_ambiguity(psi, valid, psi_f, K_f, ref=ref, nodata=-3.0)
    K_g, phi_g = ww.transfer_ambiguity(psi, valid, psi_f, K_f, ref=ref, nodata=-3.0)
    assert np.array_equal(np_(K_g), K_o)
    assert np_(phi_g).tobytes() == phi_o.tobytes()


# -------------------------------------------------------- whole filtered path ---

def test_filtered_path_parity_from_the_oracle_filter(torch_cuda):
    """Both sides unwrap the oracle's filtered phase of the 256 x 256 scene and
    move the cycle counts onto the original phase: K and phi bit for bit on
    certified pixels, the same optimum, and phi congruent to psi."""
    from tests.helpers import assert_same_on_certified_pixels
    sc = synth.config("c0", keep_truth=False)
    m, n = sc.psi.shape
    out = oracle.unwrap_filtered(sc.psi, sc.coh, sc.valid, 9, want=True)
    K_f, phi_f, tot = ww.unwrap(out["psi_f"], sc.coh, sc.valid, 9)
    assert tot == out["total"]
    ref = divmod(oracle.ref_index(sc.valid, m, n), n)
    K_g, phi_g = ww.transfer_ambiguity(sc.psi, sc.valid, out["psi_f"], K_f, ref=ref)
    fx, fy = oracle.fixed_edges(out["costs"], out["dkx"], out["dky"], out["pot"])
    share = assert_same_on_certified_pixels(np_(K_f), out["K_f"], fx, fy,
                                            oracle.ref_index(sc.valid, m, n))
    assert share > 0.5
    # the transfer is pixelwise: wherever K_f agrees, K and phi agree
    same = np_(K_f) == out["K_f"]
    assert np.array_equal(np_(K_g)[same], out["K"][same])
    v = sc.valid.astype(bool)
    cyc = (np_(phi_g).astype(np.float64) - sc.psi) / (2 * math.pi)
    assert np.abs(cyc[v] - np.round(cyc[v])).max() < 1e-4
    assert np_(K_g)[ref] == 0


def test_unwrap_filtered_equals_its_parts(torch_cuda):
    """ww_unwrap_filtered = filter, unwrap, transfer with the integration's
    reference pixel, bit for bit; fewer residues than the raw phase."""
    sc = synth.config("c0", keep_truth=False)
    m, n = sc.psi.shape
    K, phi, tot = ww.unwrap_filtered(sc.psi, sc.coh, sc.valid, 9)
    f = ww.goldstein_filter(sc.psi, sc.valid)
    K_f, _, tot_f = ww.unwrap(f, sc.coh, sc.valid, 9)
    assert tot == tot_f
    ref = divmod(oracle.ref_index(sc.valid, m, n), n)
    K2, phi2 = ww.transfer_ambiguity(sc.psi, sc.valid, f, K_f, ref=ref)
    assert np.array_equal(np_(K), np_(K2))
    assert np_(phi).tobytes() == np_(phi2).tobytes()
    r_raw = int(np.abs(np_(ww.residues(sc.psi, sc.valid)[0])).sum())
    r_f = int(np.abs(np_(ww.residues(f, sc.valid)[0])).sum())
    assert r_f * 5 < r_raw
