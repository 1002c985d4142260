"""Shared checks for the GPU parity tests (oracle side on the host)."""
import numpy as np

import oracle


def np_(t):
    return t.detach().cpu().numpy()


def flow_cost(dkx, dky, costs):
    cxp, cxn, cyp, cyn = costs
    return int(np.where(dkx > 0, cxp, np.where(dkx < 0, cxn, 0)).astype(np.int64).sum()
               + np.where(dky > 0, cyp, np.where(dky < 0, cyn, 0)).astype(np.int64).sum())


def assert_same_on_fixed_edges(costs, dkx_o, dky_o, pot_o, dkx_g, dky_g):
    """Edges whose cycle difference is the same in every optimum (oracle
    certificate) must carry the oracle's value on the GPU too."""
    fx, fy = oracle.fixed_edges(costs, dkx_o, dky_o, pot_o)
    fx = fx.astype(bool)
    fy = fy.astype(bool)
    bad = int((dkx_g[fx] != dkx_o[fx]).sum() + (dky_g[fy] != dky_o[fy]).sum())
    assert bad == 0, f"{bad} certified edges differ"
    return fx, fy


def assert_same_on_certified_pixels(K_g, K_o, fx, fy, ref):
    """K equal on pixels joined to the reference by fixed edges, and equal up
    to one offset inside every other fixed-edge component."""
    cert, comp = oracle.certified_pixels(fx, fy, ref)
    assert np.array_equal(K_g[cert], K_o[cert])
    d = (K_g.astype(np.int64) - K_o.astype(np.int64)).reshape(-1)
    c = comp.reshape(-1)
    _, first = np.unique(c, return_index=True)
    off = np.zeros(c.max() + 1, np.int64)
    off[c[first]] = d[first]
    assert np.array_equal(d, off[c])
    return float(cert.mean())


def phase_tolerance_ok(phi, psi, K, valid):
    """|phi - (psi + 2 pi K)| <= max(1e-5, ulp32(phi)/2) at valid pixels
    (computed in double)."""
    v = np.ones(psi.shape, bool) if valid is None else valid.astype(bool)
    want = psi.astype(np.float64) + 2 * np.pi * K.astype(np.float64)
    err = np.abs(phi.astype(np.float64) - want)
    tol = np.maximum(1e-5, 0.5 * np.spacing(np.abs(phi).astype(np.float32)).astype(np.float64))
    ok = (err <= tol) | ~v
    return bool(ok.all()), float(err[v].max(initial=0.0))
