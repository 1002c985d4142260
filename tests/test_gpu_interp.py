"""Parity of the interpolated table lookup (Section II-B, the cost table read
between its bin centres) between the HIP cost kernels and the oracle,
element by element: the streaming kernel (box half-widths 0..4, tables up to
8192 entries), the tile kernel (wider boxes, larger tables), and the whole
path through ww_unwrap."""
import numpy as np
import pytest

import oracle
from paper_2609_36267_amd import binding as ww
from paper_2609_36267_amd import synth
from tests.helpers import np_, phase_tolerance_ok

pytestmark = pytest.mark.gpu

PFIX = 3294199


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    ww.load()
    return torch


@pytest.fixture(scope="module")
def lut9():
    return oracle.build_lut(9)


def scene(seed, m, n):
    rng = np.random.default_rng(seed)
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    smooth = np.angle(np.exp(1j * (0.4 * j - 0.2 * i + 4 * np.sin(i / 9.0)))).astype(np.float32)
    noise = rng.uniform(-np.pi, np.pi, (m, n)).astype(np.float32)
    psi = np.where(rng.random((m, n)) < 0.75, smooth, noise).astype(np.float32)
    coh = rng.uniform(-0.05, 1.05, (m, n)).astype(np.float32)
    if m * n > 4:
        coh.reshape(-1)[rng.integers(0, m * n, 3)] = np.nan
    valid = (rng.random((m, n)) > 0.1).astype(np.uint8)
    return psi, coh, valid


def check(psi, coh, valid, T, lp=None, **kw):
    cp = ww.default_cost_params(lut_interp=1, **kw)
    got = ww.edge_costs(psi, coh, valid, T, cp, lp)
    want = oracle.edge_costs(psi, coh, valid, T, interp=1, **kw)
    for g, w in zip(got, want):
        assert np.array_equal(np_(g), w)
    return want


@pytest.mark.parametrize("shape", [(1, 9), (9, 1), (2, 2), (37, 45), (65, 97), (130, 257)])
@pytest.mark.parametrize("h", [0, 2])
def test_interp_costs_parity(torch_cuda, lut9, shape, h):
    psi, coh, valid = scene(3 + shape[0] * 17 + shape[1], *shape)
    want = check(psi, coh, valid, lut9, box_half=h)
    if min(shape) > 8:
        near = oracle.edge_costs(psi, coh, valid, lut9, box_half=h)
        assert any(not np.array_equal(a, b) for a, b in zip(want, near))


@pytest.mark.parametrize("h", [1, 3, 4, 5, 8])
def test_interp_costs_parity_box_sizes(torch_cuda, lut9, h):
    """h <= 4 runs the streaming kernel, h > 4 the tile kernel."""
    psi, coh, valid = scene(40 + h, 77, 150)
    check(psi, coh, valid, lut9, box_half=h)


def test_interp_costs_parity_large_table(torch_cuda):
    """A 64 x 256 table (more entries than the streaming kernel stages in
    LDS) sends the lookup to the tile kernel."""
    p = ww.default_lut_params()
    p.n_alpha, p.n_gamma = 256, 64
    T = ww.build_cost_lut(9, p)
    T_o = oracle.build_lut(9, oracle.lut_params(256, 64, p.n_eta, p.n_gpanel, p.n_gnode,
                                                p.n_aquad, p.sigma_span))
    assert np.array_equal(T, T_o)
    psi, coh, valid = scene(77, 70, 130)
    check(psi, coh, valid, T, lp=p)


def test_interp_costs_parity_near_centres(torch_cuda, lut9):
    """Uniform ramps whose box mean lands next to slope-bin centres and
    next to the boundaries between bins, at coherences on and between
    coherence centres: fractions near 0 and near 1/2, where a rounding slip
    in the position would show."""
    NG, NA = lut9.shape
    m, n = 24, 3 * NA
    rows = []
    for k in range(m):
        b = (k * 11) % NA
        q = ((2 * b + 1 + (k % 2)) - NA) * PFIX // NA  # centre, or the bin edge above it
        rows.append(np.cumsum(np.full(n, q, np.int64)))
    ramp = np.stack(rows).astype(np.float64) / 2.0 ** 20
    psi = np.angle(np.exp(1j * ramp)).astype(np.float32)
    coh = np.tile(((np.arange(n) % NG) + 0.5 * (np.arange(n) % 2)) / NG, (m, 1)).astype(np.float32)
    check(psi, coh, None, lut9, box_half=0, steep_rule=0)
    check(psi, coh, None, lut9, box_half=2, steep_rule=0)


def test_interp_steep_rule_parity(torch_cuda, lut9):
    rng = np.random.default_rng(8)
    m, n = 90, 110
    psi = rng.uniform(-np.pi, np.pi, (m, n)).astype(np.float32)
    coh = np.full((m, n), 0.9, np.float32)
    (_, st) = oracle.edge_costs(psi, coh, None, lut9, want_stats=True, interp=1)
    assert st["steep_candidates"] > st["steep_zeroed"] > 0
    check(psi, coh, None, lut9)


def test_interp_unwrap_end_to_end(torch_cuda, lut9):
    """ww_unwrap with the interpolated lookup reaches the oracle's optimum on
    the 256 x 256 scene."""
    sc = synth.config("c0", keep_truth=False)
    cp = ww.default_cost_params(lut_interp=1)
    K, phi, tot = ww.unwrap(sc.psi, sc.coh, sc.valid, 9, cp)
    out = oracle.unwrap(sc.psi, sc.coh, sc.valid, 9, lut=lut9, want=True, interp=1)
    assert tot == out["total"]
    near = oracle.unwrap(sc.psi, sc.coh, sc.valid, 9, lut=lut9, want=True)
    assert near["total"] != out["total"]
    ok, err = phase_tolerance_ok(np_(phi), sc.psi, np_(K), sc.valid)
    assert ok, err


def test_interp_rejects_bad_flag(torch_cuda, lut9):
    psi, coh, valid = scene(1, 8, 8)
    with pytest.raises(RuntimeError):
        ww.edge_costs(psi, coh, valid, lut9, ww.default_cost_params(lut_interp=2))


# ------------------------------------------------- non-integer looks (L) ---

@pytest.mark.parametrize("q", [(9 << 16) | 0x8000, (2 << 16) | 1, (15 << 16) | 40000,
                               (63 << 16) | 65535, 64 << 16, 7 << 16])
def test_lut_at_non_integer_looks_parity(torch_cuda, q):
    """The device's blend of two integer tables equals the oracle's, entry
    for entry (integer nodes included)."""
    assert np.array_equal(ww.build_cost_lut_q16(q), oracle.build_lut_q16(q))


def test_unwrap_at_non_integer_looks(torch_cuda):
    """ww_unwrap with looks = 9 + 0.3 (looks_frac16 = 19661): the same cost
    planes and optimal cost as the oracle's path on the blended table."""
    from tests.helpers import np_
    sc = synth.make(120, 170, looks=9, seed=21, mask_frac=0.05, disks=1, disk_radius=(10, 20),
                    keep_truth=False, workers=1)
    q = (9 << 16) | 19661
    T = oracle.build_lut_q16(q)
    out = oracle.unwrap(sc.psi, sc.coh, sc.valid, 9, lut=T, want=True)
    costs_g = ww.edge_costs(sc.psi, sc.coh, sc.valid, ww.build_cost_lut_q16(q))
    for a, b in zip(costs_g, out["costs"]):
        assert np.array_equal(np_(a), b)
    cp = ww.default_cost_params(looks_frac16=19661)
    K, phi, tot = ww.unwrap(sc.psi, sc.coh, sc.valid, 9, params=cp)
    assert tot == out["total"]
    with pytest.raises(ww.WWError):
        ww.unwrap(sc.psi, sc.coh, sc.valid, 64, params=cp)
