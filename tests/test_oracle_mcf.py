"""Pins of the oracle's min-cost-flow solve (Section II-A eq. 2, Section II-C):
brute-force enumeration of the integer cycle field, an LP solver (the
constraint matrix is totally unimodular), network simplex, the optimality
self-certificate and closed-form special cases."""
import itertools

import numpy as np
import pytest

import oracle


def wraps_from_psi(psi):
    p = psi.astype(np.float64)
    dx = p[:, 1:] - p[:, :-1]
    dy = p[1:, :] - p[:-1, :]
    wx = ((dx > np.pi).astype(int) - (dx <= -np.pi).astype(int)).astype(np.int8)
    wy = ((dy > np.pi).astype(int) - (dy <= -np.pi).astype(int)).astype(np.int8)
    return wx, wy


def residues_from_wraps(wx, wy):
    # loop (i,j): -(wx[i,j] + wy[i,j+1] - wx[i+1,j] - wy[i,j])
    return (-(wx[:-1, :] + wy[:, 1:] - wx[1:, :] - wy[:, :-1])).astype(np.int8)


def random_costs(rng, m, n, hi, zero_frac=0.0):
    out = []
    for shape in ((m, n - 1), (m, n - 1), (m - 1, n), (m - 1, n)):
        c = rng.integers(0, hi + 1, shape).astype(np.int16)
        if zero_frac:
            c[rng.random(shape) < zero_frac] = 0
        out.append(c)
    return tuple(out)


def flow_cost(dkx, dky, costs):
    cxp, cxn, cyp, cyn = costs
    return int(np.where(dkx > 0, cxp, np.where(dkx < 0, cxn, 0)).sum()
               + np.where(dky > 0, cyp, np.where(dky < 0, cyn, 0)).sum())


def all_optima_dk(wx, wy, costs, best):
    """Every optimal (dk_x, dk_y) by depth-first enumeration of K (tiny
    grids), pruned by the optimal cost."""
    cxp, cxn, cyp, cyn = costs
    m, n = wx.shape[0], wy.shape[1]
    N = m * n
    K = np.zeros(N, np.int64)
    sols = []

    def c_of(dk, cp, cn):
        return int(cp) if dk > 0 else (int(cn) if dk < 0 else 0)

    def rec(a, cost):
        if cost > best:
            return
        if a == N:
            Kf = K.reshape(m, n)
            sols.append((Kf[:, 1:] - Kf[:, :-1] + wx, Kf[1:, :] - Kf[:-1, :] + wy))
            return
        i, j = divmod(a, n)
        cands = None
        if j > 0:
            base = K[a - 1] - wx[i, j - 1]
            cands = {base - 1, base, base + 1}
        if i > 0:
            base = K[a - n] - wy[i - 1, j]
            c2 = {base - 1, base, base + 1}
            cands = c2 if cands is None else cands & c2
        for k in sorted(cands):
            c = cost
            if j > 0:
                c += c_of(k - K[a - 1] + wx[i, j - 1], cxp[i, j - 1], cxn[i, j - 1])
            if i > 0:
                c += c_of(k - K[a - n] + wy[i - 1, j], cyp[i - 1, j], cyn[i - 1, j])
            K[a] = k
            rec(a + 1, c)

    rec(1, 0)
    return sols


SHAPES = [(2, 2), (2, 3), (3, 2), (3, 3), (2, 5), (4, 3), (3, 4), (4, 4), (2, 8), (1, 6), (5, 1)]


@pytest.mark.parametrize("shape", SHAPES)
def test_mcf_equals_bruteforce(shape):
    m, n = shape
    rng = np.random.default_rng(m * 100 + n)
    for trial in range(30):
        psi = rng.uniform(-np.pi, np.pi, (m, n)).astype(np.float32)
        wx, wy = wraps_from_psi(psi)
        hi = [3, 20, 1000][trial % 3]
        costs = random_costs(rng, m, n, hi, zero_frac=0.2 if trial % 4 == 0 else 0.0)
        best, count = oracle.bruteforce(wx, wy, costs)
        res, _, _ = oracle.residues(psi)
        dkx, dky, pot, total = oracle.mcf(res, costs, m=m, n=n)
        assert total == best, (trial, total, best)
        assert flow_cost(dkx, dky, costs) == total
        cert = oracle.check_optimal(res, costs, dkx, dky, pot)
        assert cert["ok"], cert
        # uniqueness certificate <=> exactly one optimal cycle field
        fx, fy = oracle.fixed_edges(costs, dkx, dky, pot)
        all_fixed = bool(fx.all() and fy.all())
        assert all_fixed == (count == 1), (trial, count, fx, fy)


@pytest.mark.parametrize("shape", [(3, 3), (3, 4), (4, 4)])
def test_fixed_edges_agree_across_all_optima(shape):
    """Edges the certificate calls fixed carry the same cycle difference in
    every optimum found by enumeration, and the others differ in some pair."""
    m, n = shape
    rng = np.random.default_rng(7 + m * n)
    checked = 0
    for trial in range(40):
        psi = rng.uniform(-np.pi, np.pi, (m, n)).astype(np.float32)
        wx, wy = wraps_from_psi(psi)
        costs = random_costs(rng, m, n, 2, zero_frac=0.3)
        best, count = oracle.bruteforce(wx, wy, costs)
        if count == 1 or count > 200:
            continue
        res, _, _ = oracle.residues(psi)
        dkx, dky, pot, total = oracle.mcf(res, costs, m=m, n=n)
        fx, fy = oracle.fixed_edges(costs, dkx, dky, pot)
        sols = all_optima_dk(wx, wy, costs, best)
        assert len(sols) == count
        sx = np.stack([s[0] for s in sols])
        sy = np.stack([s[1] for s in sols])
        same_x = (sx == sx[0]).all(0)
        same_y = (sy == sy[0]).all(0)
        assert np.array_equal(same_x, fx.astype(bool))
        assert np.array_equal(same_y, fy.astype(bool))
        checked += 1
    assert checked >= 5


def _lp_cost(res, costs, m, n):
    from scipy.optimize import linprog
    from scipy.sparse import lil_matrix
    cxp, cxn, cyp, cyn = costs
    R, C = m - 1, n - 1
    G = R * C

    def node_above(i, j):
        return (i - 1) * C + j if i > 0 else G

    def node_below(i, j):
        return i * C + j if i < R else G
    arcs = []  # (tail, head, cost)
    for i in range(m):
        for j in range(n - 1):
            up, dn = node_above(i, j), node_below(i, j)
            arcs.append((up, dn, int(cxp[i, j])))   # downward across hx: +1
            arcs.append((dn, up, int(cxn[i, j])))   # upward: -1
    for i in range(m - 1):
        for j in range(n):
            lf = i * C + j - 1 if j > 0 else G
            rt = i * C + j if j < C else G
            arcs.append((rt, lf, int(cyp[i, j])))   # leftward across vy: +1
            arcs.append((lf, rt, int(cyn[i, j])))   # rightward: -1
    A = lil_matrix((G, len(arcs)))
    for k, (t, h, _) in enumerate(arcs):
        if t < G:
            A[t, k] += 1
        if h < G:
            A[h, k] -= 1
    c = np.array([a[2] for a in arcs], float)
    r = lp = linprog(c, A_eq=A.tocsr(), b_eq=res.reshape(-1).astype(float), bounds=(0, 1),
                     method="highs")
    assert r.status == 0
    return lp.fun


@pytest.mark.parametrize("seed,m,n", [(0, 12, 12), (1, 20, 16), (2, 24, 24)])
def test_mcf_equals_lp_optimum(seed, m, n):
    rng = np.random.default_rng(seed)
    psi = rng.uniform(-np.pi, np.pi, (m, n)).astype(np.float32)
    costs = random_costs(rng, m, n, 500, zero_frac=0.05)
    res, _, _ = oracle.residues(psi)
    _, _, _, total = oracle.mcf(res, costs, m=m, n=n)
    assert abs(_lp_cost(res, costs, m, n) - total) < 1e-6


@pytest.mark.parametrize("seed", [0, 1])
def test_mcf_equals_network_simplex(seed, scene_c0, lut9):
    """networkx network simplex on a 64x64 crop of the c0 workload."""
    import networkx as nx
    sc = scene_c0
    # the two 64x64 windows (on a 32-px lattice) with the most residues
    full, _, _ = oracle.residues(sc.psi)
    cands = [(int(np.abs(full[i:i + 63, j:j + 63]).sum()), i, j)
             for i in range(0, 193, 32) for j in range(0, 193, 32)]
    cands.sort(reverse=True)
    _, i0, j0 = cands[seed]
    psi = sc.psi[i0:i0 + 64, j0:j0 + 64]
    coh = sc.coh[i0:i0 + 64, j0:j0 + 64]
    m, n = psi.shape
    costs = oracle.edge_costs(psi, coh, None, lut9)
    res, _, ground = oracle.residues(psi)
    _, _, _, total = oracle.mcf(res, costs, m=m, n=n)
    cxp, cxn, cyp, cyn = costs
    R, C = m - 1, n - 1
    g = nx.MultiDiGraph()
    for u in range(R * C):
        g.add_node(u, demand=-int(res.reshape(-1)[u]))
    g.add_node("G", demand=-int(ground))

    def nid(i, j):
        return i * C + j if (0 <= i < R and 0 <= j < C) else "G"
    for i in range(m):
        for j in range(n - 1):
            up, dn = nid(i - 1, j), nid(i, j)
            g.add_edge(up, dn, capacity=1, weight=int(cxp[i, j]))
            g.add_edge(dn, up, capacity=1, weight=int(cxn[i, j]))
    for i in range(m - 1):
        for j in range(n):
            lf, rt = nid(i, j - 1), nid(i, j)
            g.add_edge(rt, lf, capacity=1, weight=int(cyp[i, j]))
            g.add_edge(lf, rt, capacity=1, weight=int(cyn[i, j]))
    cost, _ = nx.network_simplex(g)
    assert cost == total
    assert np.abs(res).sum() > 10


def test_no_residues_zero_flow(lut9):
    m, n = 20, 30
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    psi = np.angle(np.exp(1j * (0.4 * j + 0.2 * i))).astype(np.float32)
    res, _, g = oracle.residues(psi)
    assert not res.any() and g == 0
    costs = oracle.edge_costs(psi, np.full((m, n), 0.8, np.float32), None, lut9)
    dkx, dky, pot, total = oracle.mcf(res, costs, m=m, n=n)
    assert total == 0 and not dkx.any() and not dky.any()


def test_isolated_dipole_takes_cheapest_crossing():
    """Residues +1 and -1 in adjacent loops, every other arc expensive: the
    optimum is the cheaper of the two arcs joining them directly."""
    m, n = 8, 9
    res = np.zeros((m - 1, n - 1), np.int8)
    res[3, 3], res[3, 4] = 1, -1
    costs = [np.full(s, 5000, np.int16) for s in ((m, n - 1),) * 2 + ((m - 1, n),) * 2]
    # the edge between loops (3,3) and (3,4) is vy(3,4); flow rightwards is -1
    costs[3][3, 4] = 17   # c- of vy(3,4)
    costs[2][3, 4] = 3    # c+ (leftward) is cheaper but goes the wrong way
    dkx, dky, pot, total = oracle.mcf(res, tuple(costs), m=m, n=n)
    assert total == 17
    assert dky[3, 4] == -1 and np.count_nonzero(dky) == 1 and not dkx.any()


def test_lone_residue_routes_to_ground_like_dijkstra():
    """A single +1 residue must reach the ground; the optimum equals a
    textbook shortest path (scipy csgraph) from it to the ground node."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra
    rng = np.random.default_rng(3)
    m, n = 15, 12
    R, C = m - 1, n - 1
    G = R * C
    res = np.zeros((R, C), np.int8)
    res[4, 7] = 1
    costs = random_costs(rng, m, n, 300)
    cxp, cxn, cyp, cyn = costs
    rows, cols, w = [], [], []

    def nid(i, j):
        return i * C + j if (0 <= i < R and 0 <= j < C) else G
    for i in range(m):
        for j in range(n - 1):
            rows += [nid(i - 1, j), nid(i, j)]
            cols += [nid(i, j), nid(i - 1, j)]
            w += [cxp[i, j], cxn[i, j]]
    for i in range(m - 1):
        for j in range(n):
            rows += [nid(i, j), nid(i, j - 1)]
            cols += [nid(i, j - 1), nid(i, j)]
            w += [cyp[i, j], cyn[i, j]]
    # keep the cheapest of parallel arcs (corner loops touch the ground twice);
    # weights cost*BIG + 1 keep zero-cost arcs as explicit entries while the
    # cost part of the shortest distance stays exact
    BIG = 1 << 20
    best = {}
    for r, c, x in zip(rows, cols, w):
        best[(r, c)] = min(best.get((r, c), 1 << 62), int(x) * BIG + 1)
    ks = list(best)
    mat = csr_matrix(([best[k] for k in ks], ([k[0] for k in ks], [k[1] for k in ks])),
                     shape=(G + 1, G + 1))
    d = dijkstra(mat, indices=4 * C + 7)
    dkx, dky, pot, total = oracle.mcf(res, costs, m=m, n=n)
    assert total == int(d[G]) // BIG


def test_c0_self_certificate(scene_c0, lut9):
    sc = scene_c0
    out = oracle.unwrap(sc.psi, sc.coh, sc.valid, 9, lut=lut9, want=True)
    cert = oracle.check_optimal(out["res"], out["costs"], out["dkx"], out["dky"], out["pot"])
    assert cert["ok"] and cert["min_reduced_cost"] >= 0
    assert out["total"] == flow_cost(out["dkx"], out["dky"], out["costs"])


# ----------------------------------------------------------------------------
# The optimality checker must reject what is not an optimum (Section II-C:
# successive shortest paths end at a flow whose residual arcs all have
# non-negative reduced cost and whose divergence equals the residues).  Each
# case starts from an optimum that brute-force enumeration confirms and breaks
# exactly one of the two conditions.
# ----------------------------------------------------------------------------

def _pinned_optimum(seed, m, n, hi=50):
    """A random grid whose optimum is unique (brute force), solved by the
    oracle; returns (res, costs, dkx, dky, pot)."""
    rng = np.random.default_rng(seed)
    for _ in range(200):
        psi = rng.uniform(-np.pi, np.pi, (m, n)).astype(np.float32)
        wx, wy = wraps_from_psi(psi)
        costs = random_costs(rng, m, n, hi)
        costs = tuple(np.maximum(c, 1).astype(np.int16) for c in costs)  # no zero-cost arc
        best, count = oracle.bruteforce(wx, wy, costs)
        res, _, _ = oracle.residues(psi)
        if count != 1 or not np.abs(res).sum():
            continue
        dkx, dky, pot, total = oracle.mcf(res, costs, m=m, n=n)
        assert total == best
        cert = oracle.check_optimal(res, costs, dkx, dky, pot)
        assert cert["ok"] and cert["divergence_violations"] == 0
        assert cert["negative_reduced_costs"] == 0
        return res, costs, dkx, dky, pot
    raise AssertionError("no unique-optimum grid found")


CHECK_CASES = [(11, 3, 4), (12, 4, 4), (13, 4, 3), (14, 3, 5)]


@pytest.mark.parametrize("seed,m,n", CHECK_CASES)
def test_check_rejects_flipped_edge(seed, m, n):
    """Changing one edge's cycle difference by one moves one unit of
    divergence at each of its two dual endpoints: two violations (an edge on
    the image border has the ground as one endpoint)."""
    res, costs, dkx, dky, pot = _pinned_optimum(seed, m, n)
    for plane, i, j in [("x", 0, 0), ("x", 1, n - 2), ("y", 0, 1), ("y", m - 2, n - 1)]:
        bx, by = dkx.copy(), dky.copy()
        b = bx if plane == "x" else by
        b[i, j] = 1 if b[i, j] <= 0 else 0
        cert = oracle.check_optimal(res, costs, bx, by, pot)
        assert not cert["ok"]
        assert cert["divergence_violations"] == 2, (plane, i, j, cert)


@pytest.mark.parametrize("seed,m,n", CHECK_CASES)
def test_check_rejects_out_of_range_cycle_difference(seed, m, n):
    """|dk| = 2 is not a flow of the unit-capacity problem."""
    res, costs, dkx, dky, pot = _pinned_optimum(seed, m, n)
    bx, by = dkx.copy(), dky.copy()
    # +1 then another +1 around the same loop keeps divergence intact only if
    # both are counted; the range check alone must already fail it
    bx[1, 0] = 2 if bx[1, 0] >= 0 else -2
    cert = oracle.check_optimal(res, costs, bx, by, pot)
    assert not cert["ok"] and cert["divergence_violations"] >= 1


@pytest.mark.parametrize("seed,m,n", CHECK_CASES)
def test_check_rejects_feasible_but_costlier_flow(seed, m, n):
    """One unit pushed around a residual cycle (the four loops around an
    interior pixel, which is K += 1 at that pixel) keeps the divergence but
    raises the cost; since the optimum is unique the cycle costs more than
    zero, so under the old potentials the reversed arcs of that cycle have
    negative reduced cost and the checker must say so."""
    res, costs, dkx, dky, pot = _pinned_optimum(seed, m, n)
    base = flow_cost(dkx, dky, costs)
    tried = 0
    for i in range(1, m - 1):
        for j in range(1, n - 1):
            for s in (1, -1):
                bx, by = dkx.astype(int), dky.astype(int)
                bx[i, j - 1] += s   # edge (i,j-1)->(i,j): K_v rises
                bx[i, j] -= s       # edge (i,j)->(i,j+1): K_u rises
                by[i - 1, j] += s
                by[i, j] -= s
                if np.abs(bx).max() > 1 or np.abs(by).max() > 1:
                    continue
                bx, by = bx.astype(np.int8), by.astype(np.int8)
                assert flow_cost(bx, by, costs) > base
                cert = oracle.check_optimal(res, costs, bx, by, pot)
                assert not cert["ok"]
                assert cert["divergence_violations"] == 0
                assert cert["negative_reduced_costs"] >= 1 and cert["min_reduced_cost"] < 0
                tried += 1
    assert tried >= 1


@pytest.mark.parametrize("seed,m,n", CHECK_CASES)
def test_check_rejects_perturbed_potential(seed, m, n):
    """Raising one node's potential by one, where an arc leaves it with
    reduced cost zero (a tight arc, which every shortest-path tree arc is),
    makes that arc's reduced cost -1."""
    res, costs, dkx, dky, pot = _pinned_optimum(seed, m, n)
    R, C = m - 1, n - 1
    cxp, cxn, cyp, cyn = costs
    found = 0
    for u in range(R * C):
        i, j = divmod(u, C)
        # the four arcs out of u with their heads and cycle-difference moves
        outs = [(0, i, j, -1, (i - 1) * C + j if i > 0 else R * C),
                (0, i + 1, j, +1, (i + 1) * C + j if i + 1 < R else R * C),
                (1, i, j, +1, u - 1 if j > 0 else R * C),
                (1, i, j + 1, -1, u + 1 if j + 1 < C else R * C)]
        tight = False
        for kind, ei, ej, d, v in outs:
            f = int((dkx if kind == 0 else dky)[ei, ej])
            cp = int((cxp if kind == 0 else cyp)[ei, ej])
            cn = int((cxn if kind == 0 else cyn)[ei, ej])
            if f == 0:
                c = cp if d > 0 else cn
            elif f == -d:
                c = -(cp if f > 0 else cn)
            else:
                continue
            if c - int(pot[u]) + int(pot[v]) == 0:
                tight = True
        if not tight:
            continue
        bp = pot.copy()
        bp[u] += 1
        cert = oracle.check_optimal(res, costs, dkx, dky, bp)
        assert not cert["ok"]
        assert cert["divergence_violations"] == 0
        assert cert["min_reduced_cost"] == -1 and cert["negative_reduced_costs"] >= 1
        found += 1
    assert found >= 1


@pytest.mark.parametrize("seed,m,n", CHECK_CASES)
def test_check_accepts_shifted_potentials(seed, m, n):
    """Positive control: adding one constant to every potential (ground
    included) changes no reduced cost."""
    res, costs, dkx, dky, pot = _pinned_optimum(seed, m, n)
    cert = oracle.check_optimal(res, costs, dkx, dky, pot + 12345)
    assert cert["ok"]


def test_mcf_reports_infeasible_when_supply_exceeds_cut():
    """A 5 x 5 block of +1 loops inside a 12 x 12 image: 25 units must leave
    the block, but only 20 unit-capacity arcs cross its boundary (5 per
    side), so no feasible flow exists (Section II-A, unit capacities)."""
    m = n = 12
    res = np.zeros((m - 1, n - 1), np.int8)
    res[3:8, 3:8] = 1
    rng = np.random.default_rng(5)
    costs = random_costs(rng, m, n, 100)
    with pytest.raises(oracle.OracleError) as e:
        oracle.mcf(res, costs, m=m, n=n)
    assert e.value.code == oracle.E_INFEASIBLE
    # with the centre 3 x 3 cleared, 16 supplies meet the same cut of 20:
    # feasible (every set holding the supplies has at least 20 arcs out)
    res2 = res.copy()
    res2[4:7, 4:7] = 0
    _, _, pot, total = oracle.mcf(res2, costs, m=m, n=n)
    assert total > 0
