"""Pins of the oracle's connected components of reliably unwrapped pixels
(Section II-D): the components of the reliable-edge graph as scipy's graph
routine finds them, the labelling invariants and special cases."""
import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

import oracle


def reliable_masks(dkx, dky, costs, valid, T):
    """Reliable edges written out from the definition: both pixels valid,
    dk = 0 and both costs above T."""
    cxp, cxn, cyp, cyn = costs
    m, n = dkx.shape[0], dky.shape[1]
    v = np.ones((m, n), bool) if valid is None else valid.astype(bool)
    rx = (dkx == 0) & (cxp > T) & (cxn > T) & v[:, :-1] & v[:, 1:]
    ry = (dky == 0) & (cyp > T) & (cyn > T) & v[:-1, :] & v[1:, :]
    return rx, ry


def library_labels(m, n, rx, ry, valid, min_size):
    """Components by scipy's connected_components on the reliable-edge
    graph; numbered in row-major order of their first pixel, small ones and
    invalid pixels 0."""
    idx = np.arange(m * n).reshape(m, n)
    rows = np.concatenate([idx[:, :-1][rx], idx[:-1, :][ry]])
    cols = np.concatenate([idx[:, 1:][rx], idx[1:, :][ry]])
    g = coo_matrix((np.ones(rows.size), (rows, cols)), shape=(m * n, m * n))
    _, comp = connected_components(g, directed=False)
    comp = comp.reshape(-1)
    v = np.ones(m * n, bool) if valid is None else valid.reshape(-1).astype(bool)
    out = np.zeros(m * n, np.uint32)
    seen, nxt = {}, 0
    sizes = np.bincount(comp[v], minlength=comp.max() + 1)
    for p in range(m * n):
        if not v[p]:
            continue
        c = comp[p]
        if c not in seen:
            if sizes[c] >= min_size:
                nxt += 1
                seen[c] = nxt
            else:
                seen[c] = 0
        out[p] = seen[c]
    return out.reshape(m, n), nxt


def random_solution(seed, m, n, zero_frac=0.8):
    rng = np.random.default_rng(seed)
    dkx = np.where(rng.random((m, n - 1)) < zero_frac, 0, rng.choice([-1, 1], (m, n - 1))).astype(np.int8)
    dky = np.where(rng.random((m - 1, n)) < zero_frac, 0, rng.choice([-1, 1], (m - 1, n))).astype(np.int8)
    costs = [rng.integers(0, 700, s).astype(np.int16) for s in ((m, n - 1), (m, n - 1), (m - 1, n), (m - 1, n))]
    valid = (rng.random((m, n)) > 0.1).astype(np.uint8)
    return dkx, dky, costs, valid


@pytest.mark.parametrize("seed,m,n,T,frac", [(1, 12, 17, 300, 0.0), (2, 30, 25, 300, 0.02),
                                              (3, 9, 40, 100, 0.0), (4, 40, 40, 500, 0.005),
                                              (5, 1, 30, 300, 0.0), (6, 25, 1, 0, 0.0)])
def test_components_equal_library_graph_components(seed, m, n, T, frac):
    dkx, dky, costs, valid = random_solution(seed, m, n)
    for v in (valid, None):
        lab, nc = oracle.connected_components(dkx, dky, costs, v, threshold=T, min_size_frac=frac)
        rx, ry = reliable_masks(dkx, dky, costs, v, T)
        ms = oracle.cc_min_size(v, m, n, frac)
        want, nw = library_labels(m, n, rx, ry, v, ms)
        assert nc == nw
        assert np.array_equal(lab, want)


def test_labels_constant_across_reliable_edges_and_numbered_in_order():
    dkx, dky, costs, valid = random_solution(9, 50, 60, zero_frac=0.95)
    lab, nc = oracle.connected_components(dkx, dky, costs, valid, threshold=200, min_size_frac=0.0)
    rx, ry = reliable_masks(dkx, dky, costs, valid, 200)
    assert np.all(lab[:, :-1][rx] == lab[:, 1:][rx])
    assert np.all(lab[:-1, :][ry] == lab[1:, :][ry])
    assert np.all(lab[valid == 0] == 0) and np.all(lab[valid == 1] >= 1)
    # first appearance of labels 1, 2, ... in row-major order
    flat = lab.reshape(-1)
    firsts = [flat[flat == k].size and np.argmax(flat == k) for k in range(1, nc + 1)]
    assert firsts == sorted(firsts) and lab.max() == nc


def test_special_cases():
    m, n = 6, 7
    z = lambda s: np.zeros(s, np.int8)  # noqa: E731
    hi = [np.full(s, 1000, np.int16) for s in ((m, n - 1), (m, n - 1), (m - 1, n), (m - 1, n))]
    lo = [np.full(s, 10, np.int16) for s in ((m, n - 1), (m, n - 1), (m - 1, n), (m - 1, n))]
    # expensive, uncorrected edges everywhere: one component
    lab, nc = oracle.connected_components(z((m, n - 1)), z((m - 1, n)), hi, None)
    assert nc == 1 and np.all(lab == 1)
    # cheap edges: every pixel alone, numbered row-major when all are kept
    lab, nc = oracle.connected_components(z((m, n - 1)), z((m - 1, n)), lo, None, min_size_frac=0.0)
    assert nc == m * n and np.array_equal(lab.reshape(-1), np.arange(1, m * n + 1))
    # corrected edges are never reliable: a full column of corrections splits the image
    dkx = z((m, n - 1))
    dkx[:, 3] = 1
    lab, nc = oracle.connected_components(dkx, z((m - 1, n)), hi, None)
    assert nc == 2 and np.all(lab[:, :4] == 1) and np.all(lab[:, 4:] == 2)
    # the size threshold drops the small side
    lab, nc = oracle.connected_components(dkx, z((m - 1, n)), hi, None, min_size_frac=0.5)
    assert nc == 1 and np.all(lab[:, :4] == 1) and np.all(lab[:, 4:] == 0)
