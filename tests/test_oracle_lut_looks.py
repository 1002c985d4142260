"""Pins of the cost table at a non-integer number of looks (Section II-B:
the table is precomputed on a grid that includes L and read by interpolation
at run time).  The grid over L is the integers; an effective L = l0 + f/2^16
blends the two neighbouring tables in 2^-16 fixed point, rounded down."""
import math

import numpy as np
import pytest

import oracle


@pytest.fixture(scope="module")
def tables():
    return {L: oracle.build_lut(L) for L in (8, 9, 10, 11, 63, 64)}


def test_integer_looks_are_the_tables_themselves(tables):
    for L in (9, 10, 64):
        assert np.array_equal(oracle.build_lut_q16(L << 16), tables[L])


def test_halfway_is_floor_of_the_mean(tables):
    got = oracle.lut_blend_looks(tables[9], tables[10], 1 << 15)
    want = (tables[9].astype(np.int64) + tables[10].astype(np.int64)) // 2
    assert np.array_equal(got, want)


def test_blend_between_neighbours_and_monotone(tables):
    a, b = tables[9].astype(np.int64), tables[10].astype(np.int64)
    prev = a
    for f in (1, 1000, 16384, 32768, 50000, 65535):
        got = oracle.lut_blend_looks(tables[9], tables[10], f).astype(np.int64)
        assert (got >= np.minimum(a, b)).all() and (got <= np.maximum(a, b)).all()
        # moving towards the upper table never goes back
        assert ((got - prev) * np.sign(b - a) >= 0).all()
        prev = got
    assert np.array_equal(oracle.build_lut_q16((63 << 16) | 65535),
                          oracle.lut_blend_looks(tables[63], tables[64], 65535))


def test_blend_agrees_with_numpy_linear_interpolation(tables):
    """numpy.interp over the two integer nodes, in float64, then floored:
    equal wherever its value is not within rounding of an integer."""
    a, b = tables[10].astype(np.float64), tables[11].astype(np.float64)
    for f in (3, 12345, 40000, 65000):
        t = 10 + f / 65536.0
        ref = np.empty_like(a)
        for idx in np.ndindex(a.shape):
            ref[idx] = np.interp(t, [10.0, 11.0], [a[idx], b[idx]])
        got = oracle.lut_blend_looks(tables[10], tables[11], f).astype(np.float64)
        clear = np.abs(ref - np.round(ref)) > 1e-9
        assert np.array_equal(got[clear], np.floor(ref[clear]))
        assert np.abs(got - np.floor(ref)).max() <= 1


def test_out_of_range_looks_rejected():
    for q in (1 << 16, (1 << 16) | 5, (64 << 16) | 1, 65 << 16):
        with pytest.raises(oracle.OracleError):
            oracle.build_lut_q16(q)


@pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")
def test_blend_tracks_the_model_at_half_integer_looks(tables):
    """The cost model of eqs. 4-7 evaluated directly at L = 9.5 (published
    densities with Gamma functions and the hypergeometric function, which
    hold at non-integer L) lies within the interpolation error of the
    blended table: one unit for the floors plus an eighth of the table's
    second difference over L."""
    from tests.test_oracle_lut_composition import independent_entries
    Tb = oracle.build_lut_q16((9 << 16) | 0x8000)
    for c in (10, 25, 45, 58):
        for b, (_, _, c100) in zip((40, 60, 70), independent_entries(9.5, c, [40, 60, 70])):
            t = [int(tables[L][c, b]) for L in (8, 9, 10, 11)]
            d2 = max(abs(t[0] - 2 * t[1] + t[2]), abs(t[1] - 2 * t[2] + t[3]))
            assert abs(math.floor(c100) - int(Tb[c, b])) <= 1 + math.ceil(d2 / 8), (c, b)
