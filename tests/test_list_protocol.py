"""Host-side model of the solver's tile-list protocol, with assertions on
every list bound.

The relaxation rounds keep three rotating lists of tile entries, each of
capacity NT (the number of tiles).  Round r reads list r % 3 (its length
count[r % 3]), resets count[(r + 2) % 3] (the list the previous round
read) in one thread at its start, and appends to list (r + 1) % 3 through
activate(): an exchange of the tile's round stamp act[t] with r + 1, and a
slot reservation only when the old stamp differs.  Between batches of
rounds the host may run the pass set-up and the requeue of parked tiles,
which activate into the next round rr the same way.  Batches have any
length (the model draws 4 to 16 rounds per batch, with empty rounds at a
window's end).

The model draws, for every round, an arbitrary set of activation requests
(repeats, tiles already listed, every tile at once) in an arbitrary order,
and checks that no list ever holds more than NT entries, that every entry
is a tile index below NT, that a tile appears at most once in a list, and
that the lengths the host reads after a batch are those of the lists the
next round will read.
"""
import numpy as np
import pytest


class Protocol:
    def __init__(self, NT):
        self.NT = NT
        self.act = np.zeros(NT, np.int64)      # round stamps, 0 = never listed
        self.lists = np.full((3, NT), -1, np.int64)
        self.count = [0, 0, 0]

    def activate(self, t, r):
        assert 0 <= t < self.NT
        old = self.act[t]
        self.act[t] = r
        if old != r:
            pos = self.count[r % 3]
            self.count[r % 3] += 1
            assert pos < self.NT, f"list {r % 3} overflows at round {r}"
            self.lists[r % 3, pos] = t

    def round(self, r, rng, wants):
        """Round r: read its list, reset the list read by round r - 1,
        activate the requested tiles for round r + 1 in a shuffled order."""
        cnt = self.count[r % 3]
        assert cnt <= self.NT
        listed = self.lists[r % 3, :cnt].copy()
        assert (listed >= 0).all() and (listed < self.NT).all()
        assert len(set(listed.tolist())) == cnt, "a tile listed twice"
        # every listed tile carries this round's stamp
        assert (self.act[listed] == r).all()
        self.count[(r + 2) % 3] = 0
        reqs = list(wants(listed, rng))
        rng.shuffle(reqs)
        for t in reqs:
            self.activate(t, r + 1)
        return listed


def wants_random(NT):
    def f(listed, rng):
        k = int(rng.integers(0, 3 * NT + 1))
        out = rng.integers(0, NT, k).tolist()
        # a visit re-lists itself when unconverged, and its neighbours
        out += [t for t in listed.tolist() if rng.random() < 0.5]
        if rng.random() < 0.05:
            out += list(range(NT)) * 2   # everything, twice
        return out
    return f


@pytest.mark.parametrize("NT", [1, 2, 15, 64, 257])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_lists_never_overflow(NT, seed):
    rng = np.random.default_rng(seed * 1000 + NT)
    P = Protocol(NT)
    rr = 1
    wants = wants_random(NT)
    for window in range(40):
        # pass set-up or requeue: activations into round rr, whose list the
        # host has just read as empty (a window ends only then)
        assert P.count[rr % 3] == 0
        for t in rng.integers(0, NT, int(rng.integers(0, 2 * NT + 1))).tolist():
            P.activate(t, rr)
        while True:
            batch = int(rng.integers(4, 17))
            for _ in range(batch):
                P.round(rr, rng, wants)
                rr += 1
            # the host reads count[rr % 3]: the list the next round reads
            assert P.count[rr % 3] <= NT
            if P.count[rr % 3] == 0 or rng.random() < 0.3:
                # drain: rounds with no new activations until the list is empty
                while P.count[rr % 3]:
                    P.round(rr, rng, lambda listed, rng: [])
                    rr += 1
                break


def test_quiet_rounds_reach_an_empty_list():
    """Without activations the lists empty after one round and stay empty,
    so a window's trailing batch of launches finds nothing to relax."""
    rng = np.random.default_rng(5)
    P = Protocol(10)
    for t in range(10):
        P.activate(t, 1)
    P.round(1, rng, lambda listed, rng: [])
    for r in range(2, 30):
        assert P.count[r % 3] == 0
        P.round(r, rng, lambda listed, rng: [])
