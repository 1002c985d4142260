"""Pins of the oracle's per-edge integer costs (Section II-B: box-filtered slope,
edge coherence = min of endpoints, table lookup, mirrored reverse arc, mask
rule, steep-gradient rule)."""
import numpy as np
import pytest

import oracle

PI_D = np.pi
PFIX = 3294199


def _box(a, h):
    """Clipped (2h+1)^2 box sums by integral image (different route from the
    oracle's direct loops)."""
    m, n = a.shape
    ii = np.zeros((m + 1, n + 1), np.int64)
    ii[1:, 1:] = np.cumsum(np.cumsum(a.astype(np.int64), 0), 1)
    r0 = np.clip(np.arange(m) - h, 0, m)
    r1 = np.clip(np.arange(m) + h + 1, 0, m)
    c0 = np.clip(np.arange(n) - h, 0, n)
    c1 = np.clip(np.arange(n) + h + 1, 0, n)
    return (ii[r1][:, c1] - ii[r0][:, c1] - ii[r1][:, c0] + ii[r0][:, c0])


def numpy_costs(psi, coh, valid, T, h=2, steep=True, thresh=1.0, cap_pct=3):
    NG, NA = T.shape
    p = psi.astype(np.float64).copy()
    v = np.ones(psi.shape, bool) if valid is None else valid.astype(bool)
    p[~v] = 0.0
    c = coh.astype(np.float64)
    c = np.where(np.isnan(c) | (c < 0), 0.0, np.minimum(c, 1.0))
    out = []
    ds, vs = [], []
    for axis in (1, 0):
        if axis == 1:
            diff = p[:, 1:] - p[:, :-1]
            ve = v[:, 1:] & v[:, :-1]
            g = np.minimum(c[:, 1:], c[:, :-1])
        else:
            diff = p[1:, :] - p[:-1, :]
            ve = v[1:, :] & v[:-1, :]
            g = np.minimum(c[1:, :], c[:-1, :])
        w = (diff > PI_D).astype(int) - (diff <= -PI_D).astype(int)
        d = diff - 2 * PI_D * w
        q = np.floor(d * 2.0 ** 20).astype(np.int64)
        S = _box(np.where(ve, q, 0), h)
        cnt = _box(ve.astype(np.int64), h)
        safe = np.maximum(cnt, 1)
        ba = np.clip(((S + safe * PFIX) * NA) // (2 * safe * PFIX), 0, NA - 1)
        bg = np.minimum(NG - 1, np.floor(g * NG).astype(np.int64))
        cp = np.where(ve, T[bg, ba], 0).astype(np.int16)
        cn = np.where(ve, T[bg, NA - 1 - ba], 0).astype(np.int16)
        out += [cp, cn]
        ds.append(d)
        vs.append(ve)
    cxp, cxn, cyp, cyn = out
    nvalid = int(vs[0].sum() + vs[1].sum())
    if steep:
        keys = np.concatenate([np.abs(ds[0]).ravel(), np.abs(ds[1]).ravel()])
        ok = np.concatenate([vs[0].ravel(), vs[1].ravel()]) & (keys > thresh)
        ids = np.flatnonzero(ok)
        cap = nvalid * cap_pct // 100
        if ids.size > cap:
            order = np.lexsort((ids, -keys[ids]))
            ids = ids[order[:cap]]
        nx = cxp.size
        for arr_p, arr_n, sel in ((cxp, cxn, ids[ids < nx]), (cyp, cyn, ids[ids >= nx] - nx)):
            arr_p.reshape(-1)[sel] = 0
            arr_n.reshape(-1)[sel] = 0
    return cxp, cxn, cyp, cyn


@pytest.mark.parametrize("h", [0, 1, 2, 3])
def test_costs_match_independent_recomputation(h, lut9):
    rng = np.random.default_rng(h)
    m, n = 37, 45
    psi = rng.uniform(-np.pi, np.pi, (m, n)).astype(np.float32)
    coh = rng.uniform(-0.1, 1.1, (m, n)).astype(np.float32)
    coh[3, 4] = np.nan
    valid = (rng.random((m, n)) > 0.15).astype(np.uint8)
    got = oracle.edge_costs(psi, coh, valid, lut9, box_half=h, steep_rule=0)
    want = numpy_costs(psi, coh, valid, lut9, h=h, steep=False)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)


def test_costs_on_c0_match_recomputation(scene_c0, lut9):
    sc = scene_c0
    got, st = oracle.edge_costs(sc.psi, sc.coh, sc.valid, lut9, want_stats=True)
    want = numpy_costs(sc.psi, sc.coh, sc.valid, lut9)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)
    assert st["valid_edges"] == 2 * 256 * 255


def test_steep_cap_binds_and_picks_largest(lut9):
    """Noise so strong that far more than 3% of edges exceed 1 rad: exactly
    floor(3% of valid edges) are zeroed, the largest |d| first."""
    rng = np.random.default_rng(11)
    m, n = 40, 50
    psi = rng.uniform(-np.pi, np.pi, (m, n)).astype(np.float32)
    coh = np.full((m, n), 0.9, np.float32)
    valid = np.ones((m, n), np.uint8)
    base = oracle.edge_costs(psi, coh, valid, lut9, steep_rule=0)
    got, st = oracle.edge_costs(psi, coh, valid, lut9, want_stats=True)
    cap = st["valid_edges"] * 3 // 100
    assert st["steep_candidates"] > cap
    assert st["steep_zeroed"] == cap
    want = numpy_costs(psi, coh, valid, lut9)
    for g, w in zip(got, want):
        assert np.array_equal(g, w)
    changed = sum(int(((b != g) ).sum()) for b, g in zip(base[::2], got[::2]))
    assert changed <= cap


def test_steep_all_candidates_when_under_cap(lut9):
    m, n = 30, 30
    psi = np.zeros((m, n), np.float32)
    psi[10, 10] = 2.0  # four edges with |d| = 2 > 1 rad
    coh = np.full((m, n), 0.95, np.float32)
    got, st = oracle.edge_costs(psi, coh, None, lut9, want_stats=True)
    assert st["steep_candidates"] == 4 and st["steep_zeroed"] == 4
    cxp, cxn, cyp, cyn = got
    assert cxp[10, 9] == 0 and cxp[10, 10] == 0 and cyp[9, 10] == 0 and cyp[10, 10] == 0
    assert cxp[5, 5] > 0


def test_mask_rule_zero_cost(lut9):
    rng = np.random.default_rng(5)
    m, n = 20, 20
    psi = rng.uniform(-1, 1, (m, n)).astype(np.float32)
    coh = np.full((m, n), 0.95, np.float32)
    valid = np.ones((m, n), np.uint8)
    valid[5:9, 6:12] = 0
    cxp, cxn, cyp, cyn = oracle.edge_costs(psi, coh, valid, lut9, steep_rule=0)
    vx = valid[:, 1:] & valid[:, :-1]
    vy = valid[1:, :] & valid[:-1, :]
    assert np.all(cxp[vx == 0] == 0) and np.all(cxn[vx == 0] == 0)
    assert np.all(cyp[vy == 0] == 0) and np.all(cyn[vy == 0] == 0)
    assert np.all(cxp[vx == 1] > 0)


def test_reverse_arc_uses_mirrored_slope(lut9):
    """A uniform ramp of slope a gives c+ = T[bg][b(a)] and c- = T[bg][b(-a)]
    read from the table directly (Section II-B: the reverse correction is the
    +1 correction of the opposite slope)."""
    m, n = 16, 16
    a = 1.1
    j = np.arange(n)[None, :]
    psi = np.angle(np.exp(1j * a * j * np.ones((m, 1)))).astype(np.float32)
    coh = np.full((m, n), 0.7, np.float32)
    cxp, cxn, _, _ = oracle.edge_costs(psi, coh, None, lut9, steep_rule=0)
    NG, NA = lut9.shape
    bg = int(np.floor(np.float32(0.7) * np.float64(NG)))
    b = int(np.floor((a + np.pi) / (2 * np.pi) * NA))
    assert cxp[8, 8] == lut9[bg, b]
    assert cxn[8, 8] == lut9[bg, NA - 1 - b]
    assert cxp[8, 8] < cxn[8, 8]  # slope towards +pi: a +1 correction is cheaper


# ------------------------------------------------- interpolated table lookup --

def _interp_costs(psi, coh, valid, T, h=2):
    """Edge costs with the table interpolated at run time, recomputed in
    float64 with scipy's linear grid interpolator over the bin centres
    (positions clamped to the outermost centres, the result rounded down)."""
    from scipy.interpolate import RegularGridInterpolator
    NG, NA = T.shape
    F = RegularGridInterpolator((np.arange(NG) + 0.5, np.arange(NA) + 0.5), T.astype(np.float64))
    p = psi.astype(np.float64).copy()
    v = np.ones(psi.shape, bool) if valid is None else valid.astype(bool)
    p[~v] = 0.0
    c = coh.astype(np.float64)
    c = np.where(np.isnan(c) | (c < 0), 0.0, np.minimum(c, 1.0))
    out = []
    for axis in (1, 0):
        if axis == 1:
            diff, ve, g = p[:, 1:] - p[:, :-1], v[:, 1:] & v[:, :-1], np.minimum(c[:, 1:], c[:, :-1])
        else:
            diff, ve, g = p[1:, :] - p[:-1, :], v[1:, :] & v[:-1, :], np.minimum(c[1:, :], c[:-1, :])
        w = (diff > PI_D).astype(int) - (diff <= -PI_D).astype(int)
        q = np.floor((diff - 2 * PI_D * w) * 2.0 ** 20).astype(np.int64)
        S = _box(np.where(ve, q, 0), h)
        cnt = np.maximum(_box(ve.astype(np.int64), h), 1)
        s = (S + cnt * PFIX) * NA / (2.0 * cnt * PFIX)
        gp = np.clip(g * NG, 0.5, NG - 0.5)
        for pos in (s, NA - s):
            val = F(np.stack([gp.ravel(), np.clip(pos, 0.5, NA - 0.5).ravel()], 1)).reshape(s.shape)
            out.append(np.where(ve, np.floor(val), 0).astype(np.int64))
    return out


def test_interp_at_bin_centres_is_the_table(lut9):
    """With K = N_alpha samples and S = ((2b+1) - N_alpha) P the slope position
    is exactly the centre of bin b; a power-of-two N_gamma puts g = (k+1/2)/N_gamma
    on a coherence centre: the interpolated pair is then the table's entries."""
    NG, NA = lut9.shape
    rng = np.random.default_rng(3)
    for _ in range(200):
        b, k = int(rng.integers(NA)), int(rng.integers(NG))
        S = ((2 * b + 1) - NA) * PFIX
        g = (k + 0.5) / NG
        cp, cn = oracle.lut_pair(lut9, S, NA, g, interp=1)
        assert (cp, cn) == (int(lut9[k, b]), int(lut9[k, NA - 1 - b]))
        assert oracle.lut_pair(lut9, S, NA, g, interp=0) == (cp, cn)


def test_interp_lies_between_neighbours(lut9):
    """Halfway between two slope centres the blend is the floor of their
    mean; anywhere it stays within the four surrounding entries."""
    NG, NA = lut9.shape
    k = NG // 2
    g = (k + 0.5) / NG
    for b in range(NA - 1):
        S = (2 * (b + 1) - NA) * PFIX  # s = b + 1: the edge between bins b and b+1
        cp, _ = oracle.lut_pair(lut9, S, NA, g, interp=1)
        assert cp == (int(lut9[k, b]) + int(lut9[k, b + 1])) // 2
    rng = np.random.default_rng(4)
    for _ in range(500):
        K = int(rng.integers(1, 26))
        S = int(rng.integers(-K * PFIX, K * PFIX))
        g = float(rng.random())
        cp, cn = oracle.lut_pair(lut9, S, K, g, interp=1)
        assert lut9.min() <= cp <= lut9.max() and lut9.min() <= cn <= lut9.max()


@pytest.mark.parametrize("h", [0, 2])
def test_interp_costs_match_float_interpolation(h, lut9):
    """The fixed-point blend agrees with float64 bilinear interpolation over
    the bin centres within one cost unit at every edge (masked edges are 0
    on both sides), and differs from the nearest-bin lookup somewhere."""
    rng = np.random.default_rng(20 + h)
    m, n = 33, 41
    psi = rng.uniform(-np.pi, np.pi, (m, n)).astype(np.float32)
    coh = rng.uniform(-0.1, 1.1, (m, n)).astype(np.float32)
    valid = (rng.random((m, n)) > 0.1).astype(np.uint8)
    got = oracle.edge_costs(psi, coh, valid, lut9, box_half=h, steep_rule=0, interp=1)
    want = _interp_costs(psi, coh, valid, lut9, h=h)
    near = oracle.edge_costs(psi, coh, valid, lut9, box_half=h, steep_rule=0, interp=0)
    for g, w in zip(got, want):
        assert np.abs(g.astype(np.int64) - w).max() <= 1
    assert any(not np.array_equal(g, nb) for g, nb in zip(got, near))


def test_interp_keeps_steep_and_mask_rules(lut9):
    """The steep-gradient and mask rules act on the same edges whichever
    lookup is used."""
    rng = np.random.default_rng(11)
    m, n = 40, 50
    psi = rng.uniform(-np.pi, np.pi, (m, n)).astype(np.float32)
    coh = np.full((m, n), 0.9, np.float32)
    valid = (rng.random((m, n)) > 0.1).astype(np.uint8)
    vx = (valid[:, 1:] & valid[:, :-1]).astype(bool)
    vy = (valid[1:, :] & valid[:-1, :]).astype(bool)
    runs = []
    for interp in (0, 1):
        full, st = oracle.edge_costs(psi, coh, valid, lut9, want_stats=True, interp=interp)
        free = oracle.edge_costs(psi, coh, valid, lut9, steep_rule=0, interp=interp)
        for c, ve in zip(free, (vx, vx, vy, vy)):
            assert np.all(c[~ve] == 0)
        runs.append((full, free, st))
    assert runs[0][2] == runs[1][2] and runs[0][2]["steep_zeroed"] > 0
    # one set of edges zeroed by the steep rule, the same for both lookups
    hit = [(a != b) | (c != d) for a, b, c, d in zip(runs[0][0], runs[0][1], runs[1][0], runs[1][1])]
    # (each zeroed edge clears both of its arcs)
    assert 0 < sum(int((x | y).sum()) for x, y in (hit[0:2], hit[2:4])) <= runs[0][2]["steep_zeroed"]
    for full, free, _ in runs:
        for f, c, x in zip(full, free, hit):
            assert np.array_equal(f, np.where(x, 0, c))
