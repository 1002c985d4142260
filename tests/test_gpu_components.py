"""Connected components of reliably unwrapped pixels on the GPU
(ww_connected_components) against the oracle's breadth-first search: labels
bit-identical and the same number of components, on random solutions of
many shapes and on the oracle's own solution of a seeded scene."""
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


def random_solution(seed, m, n, zero_frac=0.8, cmax=700, invalid=0.1):
    rng = np.random.default_rng(seed)
    dkx = np.where(rng.random((m, n - 1)) < zero_frac, 0, rng.choice([-1, 1], (m, n - 1))).astype(np.int8)
    dky = np.where(rng.random((m - 1, n)) < zero_frac, 0, rng.choice([-1, 1], (m - 1, n))).astype(np.int8)
    costs = [rng.integers(0, cmax, s).astype(np.int16)
             for s in ((m, n - 1), (m, n - 1), (m - 1, n), (m - 1, n))]
    valid = (rng.random((m, n)) > invalid).astype(np.uint8)
    return dkx, dky, costs, valid


def check(dkx, dky, costs, valid, T, frac):
    lab_o, nc_o = oracle.connected_components(dkx, dky, costs, valid, threshold=T, min_size_frac=frac)
    p = ww.default_cc_params(threshold=T, min_size_frac=frac)
    lab_g, nc_g = ww.connected_components(dkx, dky, costs, valid, p)
    assert nc_g == nc_o
    assert np.array_equal(np_(lab_g).view(np.uint32), lab_o)


@pytest.mark.parametrize("shape", [(1, 1), (1, 40), (40, 1), (2, 2), (37, 45), (130, 257), (300, 77)])
@pytest.mark.parametrize("T,frac", [(300, 0.0), (100, 0.01), (0, 0.0), (650, 0.002)])
def test_components_random(torch_cuda, shape, T, frac):
    m, n = shape
    dkx, dky, costs, valid = random_solution(m * 131 + n + T, m, n)
    for v in (valid, None):
        check(dkx, dky, costs, v, T, frac)


def test_components_long_snakes(torch_cuda):
    """Serpentine components (long chains of unions) need many rounds."""
    m, n = 64, 96
    dkx = np.zeros((m, n - 1), np.int8)
    dky = np.zeros((m - 1, n), np.int8)
    hi = [np.full(s, 1000, np.int16) for s in ((m, n - 1), (m, n - 1), (m - 1, n), (m - 1, n))]
    # walls: every second row of y-edges corrected except one end, alternating
    for i in range(0, m - 1):
        dky[i, :] = 1
        dky[i, (n - 1) if i % 2 == 0 else 0] = 0
    check(dkx, dky, hi, None, 300, 0.0)


@pytest.mark.parametrize("transpose", [False, True])
def test_components_snake_across_tiles(torch_cuda, transpose):
    """One serpentine component over many tiles: every row (or column) is
    joined to the next at alternating ends, so the unions form chains
    across tile borders in both directions."""
    m, n = (200, 333) if not transpose else (333, 200)
    dkx = np.zeros((m, n - 1), np.int8)
    dky = np.zeros((m - 1, n), np.int8)
    hi = [np.full(s, 1000, np.int16) for s in ((m, n - 1), (m, n - 1), (m - 1, n), (m - 1, n))]
    if not transpose:
        for i in range(m - 1):
            dky[i, :] = 1
            dky[i, (n - 1) if i % 2 == 0 else 0] = 0
    else:
        for j in range(n - 1):
            dkx[:, j] = 1
            dkx[(m - 1) if j % 2 == 0 else 0, j] = 0
    check(dkx, dky, hi, None, 300, 0.0)
    lab, nc = ww.connected_components(dkx, dky, hi, np.ones((m, n), np.uint8),
                                      ww.default_cc_params(threshold=300, min_size_frac=0.0))
    assert nc == 1


@pytest.mark.parametrize("seed", [1, 2])
def test_components_large_with_holes(torch_cuda, seed):
    """Few large components with scattered holes and single-pixel islands
    over hundreds of tiles: many border edges join the same two roots."""
    m, n = 701, 1103
    dkx, dky, costs, valid = random_solution(seed, m, n, zero_frac=0.997, cmax=30000, invalid=0.02)
    # T = 8000 leaves about 54 % of the edges reliable: near percolation,
    # large fractal components
    for T, frac in ((10, 0.0), (10, 0.001), (8000, 0.0), (20000, 0.0)):
        check(dkx, dky, costs, valid, T, frac)
    check(dkx, dky, costs, None, 10, 0.0)


def test_components_of_the_oracle_solution(torch_cuda):
    sc = synth.make(200, 230, looks=9, seed=21, mask_frac=0.05, disks=2, disk_radius=(15, 30),
                    keep_truth=False, workers=1)
    out = oracle.unwrap(sc.psi, sc.coh, sc.valid, 9, want=True)
    for T, frac in ((300, 0.001), (100, 0.0), (1000, 0.01)):
        check(out["dkx"], out["dky"], out["costs"], sc.valid, T, frac)


def test_components_bad_args(torch_cuda):
    dkx, dky, costs, valid = random_solution(1, 10, 12)
    with pytest.raises(ww.WWError):
        ww.connected_components(dkx, dky, costs, valid, ww.default_cc_params(threshold=-1))
    with pytest.raises(ww.WWError):
        ww.connected_components(dkx, dky, costs, valid, ww.default_cc_params(min_size_frac=1.5))
