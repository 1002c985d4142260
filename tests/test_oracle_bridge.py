"""Pins of the oracle's bridging of mask-separated regions (Section II-D):
size-ordered spanning tree, closest pixel pairs, window medians and rounded
cycle offsets."""
import numpy as np
import pytest
from scipy import ndimage

import oracle


def gentle_truth(m, n, c=13.0):
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    true = 0.02 * j + 0.01 * i + 1.5 * np.sin(i / 17.0) + c
    psi = np.angle(np.exp(1j * true)).astype(np.float32)
    Kt = np.round((true - psi.astype(np.float64)) / (2 * np.pi)).astype(np.int32)
    return psi, Kt


def river_mask(m, n, seed):
    rng = np.random.default_rng(seed)
    valid = np.ones((m, n), np.uint8)
    valid[:, n // 2 - 3:n // 2 + 3] = 0                 # a river
    valid[m // 3:m // 3 + 4, :n // 2] = 0                # a canal
    for _ in range(6):                                   # lakes with islands
        a = int(rng.integers(0, m - 14))
        b = int(rng.integers(0, n - 14))
        valid[a:a + 14, b:b + 14] = 0
        valid[a + 4:a + 10, b + 4:b + 10] = 1
    return valid


def test_regions_are_the_valid_components():
    valid = river_mask(60, 80, 1)
    lab, R = oracle.regions(valid)
    ref, nref = ndimage.label(valid)
    assert R == nref
    # same partition, numbered by first pixel
    firsts = [np.flatnonzero(lab.ravel() == r)[0] for r in range(1, R + 1)]
    assert firsts == sorted(firsts)
    for r in range(1, R + 1):
        assert len(np.unique(ref[lab == r])) == 1


def test_recovers_region_offsets_on_a_smooth_field():
    """Each region's cycle counts shifted by a different integer are brought
    back to one consistent level when the phase is smooth over a window."""
    m, n = 70, 90
    psi, Kt = gentle_truth(m, n)
    valid = river_mask(m, n, 2)
    lab, R = oracle.regions(valid)
    assert R >= 4
    rng = np.random.default_rng(3)
    off = rng.integers(-7, 8, R + 1)
    K = (Kt + off[lab]).astype(np.int32)
    Kb, phi, R2 = oracle.bridge(psi, valid, K)
    assert R2 == R
    v = valid.astype(bool)
    d = (Kb.astype(np.int64) - Kt)[v]
    assert np.all(d == d[0])


def test_closest_pairs_against_distance_transform():
    """The chosen pair of every region is a closest pixel pair to the
    regions ranked before it (scipy's exact Euclidean distance transform),
    with the smallest child index, then the smallest parent index."""
    m, n = 50, 64
    valid = river_mask(m, n, 4)
    psi, Kt = gentle_truth(m, n)
    _, _, R, edges = oracle.bridge(psi, valid, Kt, want=True)
    lab, _ = oracle.regions(valid)
    sizes = np.bincount(lab.ravel())[1:]
    order = sorted(range(1, R + 1), key=lambda r: (-int(sizes[r - 1]), r))
    assert len(edges) == R - 1
    for (k, p, q, kp, d, s) in edges:
        r = order[k]
        lower = np.isin(lab, order[:k])
        dist = ndimage.distance_transform_edt(~lower)
        own = lab == r
        d2min = int(round(float((dist[own] ** 2).min())))
        pi, pj = divmod(p, n)
        qi, qj = divmod(q, n)
        assert lab[pi, pj] == r and lower[qi, qj] and kp < k
        assert (pi - qi) ** 2 + (pj - qj) ** 2 == d2min
        # smallest p achieving d2min, then smallest q at d2min from p
        ps = np.flatnonzero(own.ravel() & (np.round(dist.ravel() ** 2) == d2min))
        assert p == ps.min()
        qs = np.flatnonzero(lower.ravel())
        qd = (qs // n - pi) ** 2 + (qs % n - pj) ** 2
        assert q == qs[qd == d2min].min()
        assert order.index(int(lab[qi, qj])) == kp


def test_median_offset_closed_form():
    """Two regions of constant phase: the offset is the rounded difference
    of their (constant) medians, whatever the window."""
    m, n = 20, 30
    valid = np.ones((m, n), np.uint8)
    valid[:, 14:16] = 0
    psi = np.zeros((m, n), np.float32)
    psi[:, :14] = 0.4
    psi[:, 16:] = -0.3
    K = np.zeros((m, n), np.int32)
    K[:, 16:] = 4  # right region 4 cycles too high; equal sizes, so the left (label 1) is the root
    Kb, phi, R, edges = oracle.bridge(psi, valid, K, want=True)
    assert R == 2
    (k, p, q, kp, d, s), = edges
    assert d == int(np.floor((0.4 - (-0.3 + 8 * np.pi)) / (2 * np.pi) + 0.5)) == -4
    assert np.all(Kb[:, 16:] == 0) and np.all(Kb[:, :14] == 0)


def test_ranking_by_size_then_label():
    valid = np.zeros((10, 30), np.uint8)
    valid[1:4, 1:4] = 1      # 9 px, label 1
    valid[1:4, 10:13] = 1    # 9 px, label 2
    valid[5:9, 20:25] = 1    # 20 px, label 3 -> rank 0
    psi = np.zeros(valid.shape, np.float32)
    K = np.zeros(valid.shape, np.int32)
    _, _, R, edges = oracle.bridge(psi, valid, K, want=True)
    lab, _ = oracle.regions(valid)
    assert R == 3
    got = {k: int(lab.ravel()[p]) for (k, p, q, kp, d, s) in edges}
    assert got == {1: 1, 2: 2}


def test_identity_cases():
    psi, Kt = gentle_truth(30, 40)
    Kb, phi, R = oracle.bridge(psi, np.ones(psi.shape, np.uint8), Kt)
    assert R == 1 and np.array_equal(Kb, Kt)
    Kb, phi, R = oracle.bridge(psi, np.zeros(psi.shape, np.uint8), Kt)
    assert R == 0 and np.array_equal(Kb, Kt) and np.all(np.isnan(phi))


def test_invariants_on_noise():
    rng = np.random.default_rng(9)
    m, n = 48, 56
    valid = river_mask(m, n, 9)
    psi = rng.uniform(-np.pi, np.pi, (m, n)).astype(np.float32)
    K = rng.integers(-4, 5, (m, n)).astype(np.int32)
    Kb, phi, R, edges = oracle.bridge(psi, valid, K, want=True)
    lab, _ = oracle.regions(valid)
    sizes = np.bincount(lab.ravel())[1:]
    root = sorted(range(1, R + 1), key=lambda r: (-int(sizes[r - 1]), r))[0]
    for r in range(1, R + 1):
        d = (Kb.astype(np.int64) - K)[lab == r]
        assert np.all(d == d[0])
        if r == root:
            assert d[0] == 0
    assert np.array_equal(Kb[valid == 0], K[valid == 0])
    v = valid.astype(bool)
    cyc = (phi.astype(np.float64) - psi) / (2 * np.pi)
    assert np.abs(cyc[v] - Kb[v]).max() < 1e-4
