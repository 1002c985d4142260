"""Host model of the steep rule's two-level selection, checked against the
plain definition (Section II-B: of the valid edges whose wrapped gradient
exceeds the threshold, the steepest ones, at most a fixed share of all valid
edges, cost nothing; ties in |d| go to the lower edge index).

The selection runs in two levels.  A pre-pass histograms the candidate keys
(the bits of |d|, which order like the values for non-negative doubles)
into 4096 coarse bins, bin = min(4095, (key - bits(thr) - 1) >> shift),
with shift chosen so that the bins cover the keys up to bits(pi).  The
boundary bin b* is the largest bin whose candidates in bins >= b* number at
least cap; the edges above it are selected outright (key >= kzero), and the
remaining places go to the boundary bin's candidates (kbound <= key < kzero)
by an exact radix select over (key, ~id), eight-bit digits from the top,
which stops early once a digit's whole bucket is taken.  The model follows
those steps and must select exactly the set the definition names."""
import struct

import numpy as np
import pytest

PI_D = float(np.pi)
BINS = 4096
NONE = (1 << 64) - 1


def bits(x: float) -> int:
    return struct.unpack("<Q", struct.pack("<d", x))[0]


def coarse_params(thr: float):
    base = bits(thr + 0.0)
    top = bits(PI_D)
    shift = 0
    if top > base:
        span = top - base
        shift = max(0, span.bit_length() - 12)
    return base, shift


def coarse_bin(key: int, base: int, shift: int) -> int:
    return min(BINS - 1, (key - base - 1) >> shift)


def radix_select(keys, ids, remaining):
    """The boundary select: the threshold (hi, lo) on (key, ~id), digits from
    the top, as the workgroup passes compute it."""
    ph = mh = pl = ml = 0
    for p in range(12):
        h = [0] * 256
        for k, e in zip(keys, ids):
            lo = ~e & 0xFFFFFFFF
            if (k & mh) != ph or (lo & ml) != pl:
                continue
            d = (k >> (8 * (7 - p))) & 0xFF if p < 8 else (lo >> (8 * (11 - p))) & 0xFF
            h[d] += 1
        suf = np.cumsum(h[::-1])[::-1]
        digit = max([d for d in range(256) if suf[d] >= remaining], default=0)
        above = int(suf[digit + 1]) if digit < 255 else 0
        take = remaining - above
        whole = take == h[digit]
        remaining = take
        if p < 8:
            ph |= digit << (8 * (7 - p))
            mh |= 0xFF << (8 * (7 - p))
        else:
            pl |= digit << (8 * (11 - p))
            ml |= 0xFF << (8 * (11 - p))
        if whole:
            break
    return ph, pl


def two_level(dd, thr, pct, nvalid):
    """Selected edge ids by the two-level scheme."""
    base, shift = coarse_params(thr)
    keys = [bits(float(x)) for x in dd]
    cand = [e for e, x in enumerate(dd) if x > thr]
    hist = [0] * BINS
    for e in cand:
        hist[coarse_bin(keys[e], base, shift)] += 1
    cap = nvalid * pct // 100
    ncand = len(cand)
    if cap > 0 and ncand > cap:
        suf = np.cumsum(hist[::-1])[::-1]
        bstar = max(b for b in range(BINS) if suf[b] >= cap)
        above = int(suf[bstar + 1]) if bstar < BINS - 1 else 0
        remaining = cap - above
        assert 1 <= remaining <= hist[bstar]
    else:
        bstar = BINS if cap == 0 else -1
        remaining = 0
    kzero = base + 1 if bstar < 0 else (NONE if bstar >= BINS - 1 else base + 1 + ((bstar + 1) << shift))
    kbound = NONE if (bstar < 0 or bstar >= BINS) else base + 1 + (bstar << shift)
    sel, bkeys, bids = set(), [], []
    for e in cand:
        k = keys[e]
        b = coarse_bin(k, base, shift)
        # the key bounds say the same as the bin comparison
        assert (k >= kzero) == (b > bstar)
        assert (kbound <= k < kzero) == (b == bstar)
        if k >= kzero:
            sel.add(e)
        elif k >= kbound:
            bkeys.append(k)
            bids.append(e)
    if remaining and bkeys:
        if len(bkeys) <= remaining:
            sel.update(bids)
        else:
            th, tl = radix_select(bkeys, bids, remaining)
            for k, e in zip(bkeys, bids):
                lo = ~e & 0xFFFFFFFF
                if k > th or (k == th and lo >= tl):
                    sel.add(e)
    return sel


def by_definition(dd, thr, pct, nvalid):
    cand = [e for e, x in enumerate(dd) if x > thr]
    cap = nvalid * pct // 100
    cand.sort(key=lambda e: (-dd[e], e))
    return set(cand[:cap])


def draw(rng, kind, n):
    if kind == "uniform":
        return rng.uniform(0, PI_D, n)
    if kind == "ties":  # few distinct values: ties decided by the edge index
        return rng.choice([0.5, 1.25, 1.5, 2.0, 3.0], n)
    if kind == "narrow":  # every candidate in one coarse bin
        return 1.7 + rng.integers(0, 50, n) * 2.0 ** -40
    if kind == "wide":  # inputs outside one cycle: gradients beyond pi share the last bin
        return np.abs(rng.normal(0, 3.0, n))
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["uniform", "ties", "narrow", "wide"])
@pytest.mark.parametrize("thr,pct", [(1.0, 3), (1.0, 40), (0.0, 10), (2.5, 100), (3.5, 50),
                                     (1.0, 0)])
def test_two_level_selects_the_defined_set(kind, thr, pct):
    rng = np.random.default_rng(hash((kind, thr, pct)) & 0xFFFF)
    n = 3000
    dd = draw(rng, kind, n)
    nvalid = n + int(rng.integers(0, 500))  # some valid edges carry no gradient here
    assert two_level(dd, thr, pct, nvalid) == by_definition(dd, thr, pct, nvalid)


def test_fewer_candidates_than_cap_selects_all():
    dd = np.array([0.1, 2.0, 0.3, 1.5, 3.0])
    assert two_level(dd, 1.0, 100, 5) == {1, 3, 4}


def test_negative_zero_threshold_orders_like_zero():
    dd = np.array([0.0, 1e-300, 0.5, 0.5, 2.0])
    for thr in (0.0, -0.0):
        assert two_level(dd, thr, 60, 5) == by_definition(dd, thr, 60, 5) == {4, 2, 3}
