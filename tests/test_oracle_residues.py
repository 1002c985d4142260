"""Pins of the oracle's residues (Section II-A, eq. 1) against exact rational
arithmetic, the vortex closed form and the discrete Stokes identity."""
from fractions import Fraction

import numpy as np
import pytest

import oracle

# pi to 50 digits as an exact rational
PI50 = Fraction("3.14159265358979323846264338327950288419716939937510")


def exact_wrap_count(a: float, b: float) -> int:
    """Cycles removed by wrap(b - a) into (-pi, pi], in exact rationals."""
    d = Fraction(b) - Fraction(a)
    if d > PI50:
        return 1
    if d <= -PI50:
        return -1
    return 0


def exact_residues(psi, valid=None):
    m, n = psi.shape
    p = psi.astype(np.float64).copy()
    if valid is not None:
        p[valid == 0] = 0.0
    res = np.zeros((m - 1, n - 1), np.int64)
    for i in range(m - 1):
        for j in range(n - 1):
            w1 = exact_wrap_count(p[i, j], p[i, j + 1])
            w2 = exact_wrap_count(p[i, j + 1], p[i + 1, j + 1])
            w3 = exact_wrap_count(p[i + 1, j], p[i + 1, j + 1])
            w4 = exact_wrap_count(p[i, j], p[i + 1, j])
            # loop (i,j)->(i,j+1)->(i+1,j+1)->(i+1,j)->(i,j): sum of wrapped
            # differences = -2pi * (w1 + w2 - w3 - w4)
            res[i, j] = -(w1 + w2 - w3 - w4)
    return res


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_residues_match_exact_rationals_random(seed):
    rng = np.random.default_rng(seed)
    psi = rng.uniform(-np.pi, np.pi, (17, 23)).astype(np.float32)
    res, _, _ = oracle.residues(psi)
    assert np.array_equal(res, exact_residues(psi))
    assert set(np.unique(res)) <= {-1, 0, 1}


def test_residues_adversarial_near_pi():
    """Differences within a few float32 ulps of +-pi, and exactly +-pi_f32."""
    rng = np.random.default_rng(7)
    pf = np.float32(np.pi)
    vals = [pf, -pf, np.float32(0.0), np.nextafter(pf, np.float32(0)),
            np.nextafter(-pf, np.float32(0)), np.float32(1e-30), np.float32(-1e-30)]
    psi = rng.choice(np.array(vals, np.float32), size=(9, 9))
    # include rows where neighbours differ by nearly 2pi and by nearly pi
    psi[0, :] = [pf, -pf, pf, -pf, 0, pf, 0, -pf, 0]
    psi[1, :] = np.float32(np.pi / 2) * np.array([0, 2, 0, -2, 0, 2, 1, -1, 0], np.float32)
    res, _, _ = oracle.residues(psi)
    assert np.array_equal(res, exact_residues(psi))


def test_residues_with_mask_read_as_zero():
    rng = np.random.default_rng(3)
    psi = rng.uniform(-np.pi, np.pi, (12, 14)).astype(np.float32)
    valid = (rng.random((12, 14)) > 0.3).astype(np.uint8)
    res, _, _ = oracle.residues(psi, valid)
    assert np.array_equal(res, exact_residues(psi, valid))


@pytest.mark.parametrize("ci,cj,sign", [(4.5, 6.5, 1), (2.3, 3.7, 1), (7.6, 1.2, -1)])
def test_vortex_closed_form(ci, cj, sign):
    """psi = sign * atan2(i - ci, j - cj) winds once around (ci, cj): exactly
    the loop containing the centre carries charge `sign` (the loop order
    (i,j)->(i,j+1)->(i+1,j+1)->(i+1,j) turns the angle by +2pi)."""
    m, n = 10, 10
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    psi = (sign * np.arctan2(i - ci, j - cj)).astype(np.float32)
    res, perim, ground = oracle.residues(psi)
    want = np.zeros((m - 1, n - 1), np.int64)
    want[int(np.floor(ci)), int(np.floor(cj))] = sign
    assert np.array_equal(res, want)
    # the ground node balances the single charge
    assert ground == -sign


@pytest.mark.parametrize("seed", [0, 5])
def test_stokes_identity(seed):
    """Sum of loop charges plus the one-sided boundary charges is zero; the
    boundary charges are recomputed here with numpy from the wrap counts."""
    rng = np.random.default_rng(seed)
    m, n = 31, 27
    psi = rng.uniform(-np.pi, np.pi, (m, n)).astype(np.float32)
    res, perim, ground = oracle.residues(psi)
    p = psi.astype(np.float64)
    dx = p[:, 1:] - p[:, :-1]
    dy = p[1:, :] - p[:-1, :]
    wx = (dx > np.pi).astype(int) - (dx <= -np.pi).astype(int)
    wy = (dy > np.pi).astype(int) - (dy <= -np.pi).astype(int)
    boundary = wx[0, :].sum() - wx[m - 1, :].sum() - wy[:, 0].sum() + wy[:, n - 1].sum()
    assert int(res.sum()) + int(boundary) == 0
    assert int(perim.sum()) == int(boundary)
    assert ground == -int(res.sum())


def test_degenerate_shapes():
    psi = np.linspace(-3, 3, 7, dtype=np.float32)[None, :]
    res, perim, ground = oracle.residues(psi)
    assert res.size == 0 and ground == 0
    # top and bottom ring charges of a single row cancel
    assert perim.sum() == 0
