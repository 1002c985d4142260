"""CPU oracle for the MCF phase-unwrapping hot path (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It wraps ``ww_oracle.c`` (plain C,
single-threaded, FP64 and integer arithmetic, built with gcc -O2
-ffp-contract=off) and shares no code, header or table with the HIP library.

Parity status by function (the pins live in ``tests/test_oracle_*.py``):
  residues         pinned (exact rationals, vortex closed form, Stokes)
  f_eta, touzi     pinned (300-digit published forms, closed forms, norms)
  ftilde, mass     pinned (adaptive quadrature, normalisation, symmetry)
  sigma_alpha      parity unpinned as to the paper's formula (uniform limit pinned)
  build_lut        table values parity unpinned (the paper prints none);
                   shape properties of Section II-B pinned
  edge_costs       pinned (independent numpy recomputation, mirror, mask, cap)
  mcf              pinned (brute force, LP optimum, network simplex, certificate)
  integrate        pinned (path independence, congruence, exact recovery)
  connected_components  pinned (graph connected components of a library
                   routine, invariants, special cases)
  goldstein        pinned (identity at alpha = 0, plane waves on the DFT grid,
                   explicit DFT sums on tiny patches, conjugation symmetry)
  transfer_ambiguity  pinned (congruence, nearest value, brute force)
  regions, bridge  pinned (scipy labelling and exact distance transform,
                   offset recovery on smooth fields, closed-form medians,
                   ranking, invariants)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ww_oracle.c")
_LIB = os.path.join(_HERE, "libww_oracle.so")
_lock = threading.Lock()
_lib = None

OK, E_INVALID_ARG, E_OOM, E_INFEASIBLE, E_CERT = 0, -1, -2, -3, -6


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (single-threaded, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            _lib = C.CDLL(build())
            _declare(_lib)
    return _lib


P = C.c_void_p
I32 = C.c_int
I64 = C.c_int64
D = C.c_double


class LutParams(C.Structure):
    _fields_ = [("n_alpha", C.c_int32), ("n_gamma", C.c_int32), ("n_eta", C.c_int32),
                ("n_gpanel", C.c_int32), ("n_gnode", C.c_int32), ("n_aquad", C.c_int32),
                ("sigma_span", C.c_double)]


def lut_params(n_alpha=128, n_gamma=64, n_eta=2048, n_gpanel=64, n_gnode=16, n_aquad=513,
               sigma_span=8.0) -> LutParams:
    return LutParams(n_alpha, n_gamma, n_eta, n_gpanel, n_gnode, n_aquad, sigma_span)


def _declare(L):
    L.wwo_residues.argtypes = [P, P, I32, I32, P, P, P]
    L.wwo_f_eta.argtypes = [D, D, I32]
    L.wwo_f_eta.restype = D
    L.wwo_touzi.argtypes = [D, D, I32]
    L.wwo_touzi.restype = D
    L.wwo_gauss_legendre.argtypes = [I32, P, P]
    L.wwo_ftilde.argtypes = [I32, D, P, P]
    L.wwo_edge_mass.argtypes = [P, I32, P]
    L.wwo_branch_q.argtypes = [P, I32, D, P, P]
    L.wwo_slope_marginal.argtypes = [P, I32, D, D, I32, D, P, P]
    L.wwo_sigma_alpha.argtypes = [D, I32, I32]
    L.wwo_sigma_alpha.restype = D
    L.wwo_build_lut.argtypes = [I32, P, P, P, P, P]
    L.wwo_edge_costs.argtypes = [P, P, P, I32, I32, P, I32, I32, I32, I32, D, I32, I32, P, P, P, P, P]
    L.wwo_lut_pair.argtypes = [P, I32, I32, I64, I64, D, I32, P, P]
    L.wwo_lut_blend_looks.argtypes = [P, P, I64, I32, P]
    L.wwo_mcf.argtypes = [P, I32, I32, P, P, P, P, P, P, P, P, P]
    L.wwo_check_optimal.argtypes = [P, I32, I32, P, P, P, P, P, P, P, P]
    L.wwo_fixed_edges.argtypes = [I32, I32, P, P, P, P, P, P, P, P, P]
    L.wwo_integrate.argtypes = [P, P, P, P, I32, I32, I32, I32, C.c_float, P, P]
    L.wwo_certified_pixels.argtypes = [I32, I32, P, P, I64, P, P]
    L.wwo_bruteforce.argtypes = [I32, I32, P, P, P, P, P, P, P, P]
    L.wwo_connected_components.argtypes = [P, P, P, P, P, P, P, I32, I32, I32, I64, P, P]


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what} failed with status {code}")
        self.code = code


def _chk(rc, what):
    if rc != OK:
        raise OracleError(rc, what)


# ---------------------------------------------------------------- residues ---

def residues(psi, valid=None):
    """(res int8 [(m-1),(n-1)], perim int8 [2(n-1)+2(m-1)], ground int)."""
    psi = _c(psi, np.float32)
    valid = _c(valid, np.uint8)
    m, n = psi.shape
    res = np.zeros((max(m - 1, 0), max(n - 1, 0)), np.int8)
    perim = np.zeros(max(2 * (n - 1) + 2 * (m - 1), 0), np.int8)
    g = np.zeros(1, np.int64)
    _chk(lib().wwo_residues(_p(psi), _p(valid), m, n, _p(res), _p(perim), _p(g)), "residues")
    return res, perim, int(g[0])


# --------------------------------------------------------------------- LUT ---

def f_eta(eta, gamma, L):
    return lib().wwo_f_eta(float(eta), float(gamma), int(L))


def touzi(gh, gamma, L):
    return lib().wwo_touzi(float(gh), float(gamma), int(L))


def gauss_legendre(n):
    x = np.zeros(n)
    w = np.zeros(n)
    lib().wwo_gauss_legendre(n, _p(x), _p(w))
    return x, w


def ftilde(L, gh, params=None):
    params = params or lut_params()
    out = np.zeros(params.n_eta)
    _chk(lib().wwo_ftilde(L, float(gh), C.byref(params), _p(out)), "ftilde")
    return out


def edge_mass(ft):
    ft = _c(ft, np.float64)
    N = ft.shape[0]
    pm = np.zeros(2 * N - 1)
    lib().wwo_edge_mass(_p(ft), N, _p(pm))
    return pm


def branch_q(pm, alpha):
    pm = _c(pm, np.float64)
    N = (pm.shape[0] + 1) // 2
    q0 = np.zeros(1)
    qp = np.zeros(1)
    _chk(lib().wwo_branch_q(_p(pm), N, float(alpha), _p(q0), _p(qp)), "branch_q")
    return float(q0[0]), float(qp[0])


def slope_marginal(pm, alpha_hat, sigma, n_aquad=513, span=8.0):
    """(P0, P+) of eq. 7 for edge-noise masses pm."""
    pm = _c(pm, np.float64)
    N = (pm.shape[0] + 1) // 2
    P0 = np.zeros(1)
    Pp = np.zeros(1)
    _chk(lib().wwo_slope_marginal(_p(pm), N, float(alpha_hat), float(sigma), int(n_aquad),
                                  float(span), _p(P0), _p(Pp)), "slope_marginal")
    return float(P0[0]), float(Pp[0])


def sigma_alpha(gh, L, n_eta=2048):
    return lib().wwo_sigma_alpha(float(gh), int(L), int(n_eta))


def build_lut(L, params=None, want_probs=False):
    """int16 table [n_gamma, n_alpha] (+ P0, P+, sigma_alpha if asked)."""
    params = params or lut_params()
    T = np.zeros((params.n_gamma, params.n_alpha), np.int16)
    P0 = np.zeros((params.n_gamma, params.n_alpha)) if want_probs else None
    Pp = np.zeros((params.n_gamma, params.n_alpha)) if want_probs else None
    sg = np.zeros(params.n_gamma) if want_probs else None
    _chk(lib().wwo_build_lut(int(L), C.byref(params), _p(T), _p(P0), _p(Pp), _p(sg)), "build_lut")
    if want_probs:
        return T, P0, Pp, sg
    return T


def build_lut_q16(looks_q16, params=None):
    """Table at the effective number of looks looks_q16 / 2^16 (2 <= L <=
    64): the tables of the two neighbouring integers blended entry by entry
    in 2^-16 fixed point, rounded down (wwo_lut_blend_looks)."""
    l0, f = int(looks_q16) >> 16, int(looks_q16) & 0xffff
    if l0 < 2 or l0 > 64 or (l0 == 64 and f):
        raise OracleError(E_INVALID_ARG, "build_lut_q16")
    T0 = build_lut(l0, params)
    if f == 0:
        return T0
    T1 = build_lut(l0 + 1, params)
    return lut_blend_looks(T0, T1, f)


def lut_blend_looks(T0, T1, f):
    T0 = _c(T0, np.int16)
    T1 = _c(T1, np.int16)
    out = np.zeros_like(T0)
    lib().wwo_lut_blend_looks(_p(T0), _p(T1), int(T0.size), int(f), _p(out))
    return out


# ------------------------------------------------------------------- costs ---

def edge_costs(psi, coh, valid, lut, box_half=2, steep_rule=1, steep_thresh=1.0, steep_cap_pct=3,
               want_stats=False, interp=0):
    psi = _c(psi, np.float32)
    coh = _c(coh, np.float32)
    valid = _c(valid, np.uint8)
    lut = _c(lut, np.int16)
    m, n = psi.shape
    ng, na = lut.shape
    cxp = np.zeros((m, max(n - 1, 0)), np.int16)
    cxn = np.zeros_like(cxp)
    cyp = np.zeros((max(m - 1, 0), n), np.int16)
    cyn = np.zeros_like(cyp)
    st = np.zeros(3, np.int64)
    _chk(lib().wwo_edge_costs(_p(psi), _p(coh), _p(valid), m, n, _p(lut), na, ng, box_half,
                              steep_rule, float(steep_thresh), steep_cap_pct, int(interp),
                              _p(cxp), _p(cxn), _p(cyp), _p(cyn), _p(st)), "edge_costs")
    out = (cxp, cxn, cyp, cyn)
    if want_stats:
        return out, dict(valid_edges=int(st[0]), steep_candidates=int(st[1]), steep_zeroed=int(st[2]))
    return out


def lut_pair(lut, S, K, g, interp=1):
    """(c+, c-) of one edge from the table: slope sum S (2^-20 rad fixed point)
    over K valid samples, edge coherence g (Section II-B lookup, nearest bin
    when interp is 0, bilinear between bin centres otherwise)."""
    lut = _c(lut, np.int16)
    ng, na = lut.shape
    cp, cn = C.c_int16(0), C.c_int16(0)
    lib().wwo_lut_pair(_p(lut), na, ng, int(S), int(K), float(g), int(interp),
                       C.byref(cp), C.byref(cn))
    return int(cp.value), int(cn.value)


# --------------------------------------------------------------------- MCF ---

def mcf(res, costs, m=None, n=None, want_stats=False):
    """Successive shortest paths.  Returns (dk_x, dk_y, pot, total_cost)."""
    res = _c(res, np.int8)
    cxp, cxn, cyp, cyn = [_c(c, np.int16) for c in costs]
    if m is None:
        m, n = cxp.shape[0], cyp.shape[1]
    dkx = np.zeros((m, max(n - 1, 0)), np.int8)
    dky = np.zeros((max(m - 1, 0), n), np.int8)
    pot = np.zeros(max((m - 1) * (n - 1), 0) + 1, np.int64)
    tot = np.zeros(1, np.int64)
    st = np.zeros(3, np.int64)
    _chk(lib().wwo_mcf(_p(res), m, n, _p(cxp), _p(cxn), _p(cyp), _p(cyn), _p(dkx), _p(dky),
                       _p(pot), _p(tot), _p(st)), "mcf")
    out = (dkx, dky, pot, int(tot[0]))
    if want_stats:
        return out, dict(augmentations=int(st[0]), settled=int(st[1]), scanned=int(st[2]))
    return out


def check_optimal(res, costs, dkx, dky, pot):
    """Return dict(ok, divergence_violations, negative_reduced_costs, min_reduced_cost)."""
    res = _c(res, np.int8)
    cxp, cxn, cyp, cyn = [_c(c, np.int16) for c in costs]
    dkx = _c(dkx, np.int8)
    dky = _c(dky, np.int8)
    pot = _c(pot, np.int64)
    m, n = cxp.shape[0], cyp.shape[1]
    out = np.zeros(3, np.int64)
    rc = lib().wwo_check_optimal(_p(res), m, n, _p(cxp), _p(cxn), _p(cyp), _p(cyn), _p(dkx),
                                 _p(dky), _p(pot), _p(out))
    if rc not in (OK, E_CERT):
        raise OracleError(rc, "check_optimal")
    return dict(ok=rc == OK, divergence_violations=int(out[0]),
                negative_reduced_costs=int(out[1]), min_reduced_cost=int(out[2]))


def fixed_edges(costs, dkx, dky, pot):
    cxp, cxn, cyp, cyn = [_c(c, np.int16) for c in costs]
    dkx = _c(dkx, np.int8)
    dky = _c(dky, np.int8)
    pot = _c(pot, np.int64)
    m, n = cxp.shape[0], cyp.shape[1]
    fx = np.zeros(dkx.shape, np.uint8)
    fy = np.zeros(dky.shape, np.uint8)
    _chk(lib().wwo_fixed_edges(m, n, _p(cxp), _p(cxn), _p(cyp), _p(cyn), _p(dkx), _p(dky),
                               _p(pot), _p(fx), _p(fy)), "fixed_edges")
    return fx, fy


def certified_pixels(fx, fy, ref):
    fx = _c(fx, np.uint8)
    fy = _c(fy, np.uint8)
    m, n = fx.shape[0], fy.shape[1]
    cert = np.zeros((m, n), np.uint8)
    comp = np.zeros((m, n), np.int64)
    _chk(lib().wwo_certified_pixels(m, n, _p(fx), _p(fy), int(ref), _p(cert), _p(comp)),
         "certified_pixels")
    return cert.astype(bool), comp


# --------------------------------------------------------------- integrate ---

def integrate(psi, valid, dkx, dky, ref=None, nodata=float("nan")):
    psi = _c(psi, np.float32)
    valid = _c(valid, np.uint8)
    dkx = _c(dkx, np.int8)
    dky = _c(dky, np.int8)
    m, n = psi.shape
    K = np.zeros((m, n), np.int32)
    phi = np.zeros((m, n), np.float32)
    ri, rj = (-1, -1) if ref is None else ref
    _chk(lib().wwo_integrate(_p(psi), _p(valid), _p(dkx), _p(dky), m, n, ri, rj,
                             C.c_float(nodata), _p(K), _p(phi)), "integrate")
    return K, phi


def ref_index(valid, m, n):
    if valid is None:
        return 0
    v = np.asarray(valid).reshape(-1)
    nz = np.flatnonzero(v)
    return int(nz[0]) if nz.size else 0


# ------------------------------------------------------------- brute force ---

def bruteforce(wx, wy, costs):
    wx = _c(wx, np.int8)
    wy = _c(wy, np.int8)
    cxp, cxn, cyp, cyn = [_c(c, np.int16) for c in costs]
    m, n = cxp.shape[0], cyp.shape[1]
    best = np.zeros(1, np.int64)
    cnt = np.zeros(1, np.int64)
    _chk(lib().wwo_bruteforce(m, n, _p(wx), _p(wy), _p(cxp), _p(cxn), _p(cyp), _p(cyn),
                              _p(best), _p(cnt)), "bruteforce")
    return int(best[0]), int(cnt[0])


# ------------------------------------------------------------ whole path ----

def unwrap(psi, coh, valid, looks, lut=None, box_half=2, steep_rule=1, want=False, interp=0):
    """Residues -> LUT -> costs -> SSP -> integration, all on the CPU."""
    if lut is None:
        lut = build_lut(looks)
    res, perim, ground = residues(psi, valid)
    costs = edge_costs(psi, coh, valid, lut, box_half=box_half, steep_rule=steep_rule,
                       interp=interp)
    dkx, dky, pot, total = mcf(res, costs, m=psi.shape[0], n=psi.shape[1])
    K, phi = integrate(psi, valid, dkx, dky)
    if want:
        return dict(res=res, perim=perim, ground=ground, costs=costs, dkx=dkx, dky=dky, pot=pot,
                    total=total, K=K, phi=phi, lut=lut)
    return K, phi, total


def cc_min_size(valid, m, n, min_size_frac):
    """Smallest labelled component: max(1, ceil(frac * valid pixels))."""
    import math
    nv = int(m) * int(n) if valid is None else int(np.count_nonzero(valid))
    return max(1, int(math.ceil(float(min_size_frac) * nv)))


def connected_components(dkx, dky, costs, valid, threshold=300, min_size_frac=0.001):
    """Labels (uint32 [m, n]) of components of reliably unwrapped pixels and
    their number (Section II-D)."""
    dkx = _c(dkx, np.int8)
    dky = _c(dky, np.int8)
    cxp, cxn, cyp, cyn = [_c(c, np.int16) for c in costs]
    m, n = dkx.shape[0], dky.shape[1]
    valid = _c(valid, np.uint8)
    labels = np.zeros((m, n), np.uint32)
    nc = C.c_int64(0)
    _chk(lib().wwo_connected_components(_p(dkx), _p(dky), _p(cxp), _p(cxn), _p(cyp), _p(cyn),
                                        _p(valid), m, n, int(threshold),
                                        C.c_int64(cc_min_size(valid, m, n, min_size_frac)),
                                        _p(labels), C.byref(nc)), "connected_components")
    return labels, int(nc.value)


# ------------------------------------------------ Goldstein preprocessing ---

def triangle_taper(N):
    """Patch taper w(i) = 1 - |2i + 1 - N| / N, i = 0..N-1: positive, and two
    copies offset by N/2 sum to 1."""
    i = np.arange(N, dtype=np.float64)
    return 1.0 - np.abs(2.0 * i + 1.0 - N) / N


def goldstein(psi, valid=None, alpha=0.5, patch=32, smooth=3, want_sum=False):
    """Adaptive power-spectrum ("Goldstein") filter of the wrapped phase, the
    optional preprocessing of Section II-D, in float64.

    Unit phasors exp(i psi) at valid pixels, 0 elsewhere and outside the
    image.  Patches of N x N pixels (N = patch) sit on a grid of step N/2
    whose first patch starts N/2 rows above and N/2 columns left of the
    image, so that every pixel lies in four patches.  For each patch: the
    2-D DFT Z; B = the circular smooth x smooth mean of |Z|; Z is multiplied
    by H = (B / max B)^alpha (an all-zero patch contributes nothing); the
    inverse DFT is tapered by w(r) w(c) (triangle_taper) and added to the
    sum.  The filtered phase is the argument of the sum at valid pixels;
    invalid pixels keep psi.  Returns float32 [m, n] (and the complex sum
    when want_sum)."""
    psi = np.asarray(psi, np.float32)
    m, n = psi.shape
    v = np.ones((m, n), bool) if valid is None else np.asarray(valid).astype(bool)
    N = int(patch)
    S = N // 2
    z = np.where(v, np.exp(1j * psi.astype(np.float64)), 0.0)
    w = triangle_taper(N)
    w2 = np.outer(w, w)
    h = smooth // 2
    acc = np.zeros((m, n), np.complex128)
    for pi in range((m + S - 1) // S + 1):
        for pj in range((n + S - 1) // S + 1):
            r0, c0 = pi * S - S, pj * S - S
            blk = np.zeros((N, N), np.complex128)
            ra, rb = max(r0, 0), min(r0 + N, m)
            ca, cb = max(c0, 0), min(c0 + N, n)
            if ra >= rb or ca >= cb:
                continue
            blk[ra - r0:rb - r0, ca - c0:cb - c0] = z[ra:rb, ca:cb]
            Z = np.fft.fft2(blk)
            A = np.abs(Z)
            B = np.zeros_like(A)
            for du in range(-h, h + 1):
                for dv in range(-h, h + 1):
                    B += np.roll(np.roll(A, du, axis=0), dv, axis=1)
            B /= float(smooth * smooth)
            mx = B.max()
            if not mx > 0.0:
                continue
            H = (B / mx) ** float(alpha)
            zf = np.fft.ifft2(Z * H) * w2
            acc[ra:rb, ca:cb] += zf[ra - r0:rb - r0, ca - c0:cb - c0]
    out = np.where(v, np.arctan2(acc.imag, acc.real), psi.astype(np.float64)).astype(np.float32)
    if want_sum:
        return out, acc
    return out


def transfer_ambiguity(psi, valid, psi_f, K_f, ref=None, nodata=float("nan")):
    """Cycle counts on the original phase from those found on a filtered
    copy (Section II-D: the modified phase only estimates K).  At a valid
    pixel K = K_f + k with k the integer that puts psi + 2 pi K within
    (-pi, pi] of psi_f + 2 pi K_f, i.e. k = -wrap(psi - psi_f), wrap(x) =
    [x > pi] - [x <= -pi] in float64; elsewhere K = K_f.  With ref = (i, j)
    every K is then shifted so that K(i, j) = 0.  phi = float32 of
    psi + 2 pi K (float64) at valid pixels, nodata elsewhere."""
    psi = np.asarray(psi, np.float32).astype(np.float64)
    psi_f = np.asarray(psi_f, np.float32).astype(np.float64)
    K_f = np.asarray(K_f, np.int64)
    v = np.ones(psi.shape, bool) if valid is None else np.asarray(valid).astype(bool)
    x = psi - psi_f
    wrap = (x > np.pi).astype(np.int64) - (x <= -np.pi).astype(np.int64)
    K = np.where(v, K_f - wrap, K_f)
    if ref is not None:
        K = K - K[ref[0], ref[1]]
    K = K.astype(np.int32)
    phi = np.where(v, psi + 2.0 * np.pi * K.astype(np.float64), nodata).astype(np.float32)
    return K, phi


def unwrap_filtered(psi, coh, valid, looks, alpha=0.5, patch=32, smooth=3, lut=None, want=False):
    """Goldstein-filtered phase -> the whole path -> cycle counts moved back
    onto the original phase (Section II-D)."""
    psi_f = goldstein(psi, valid, alpha=alpha, patch=patch, smooth=smooth)
    out = unwrap(psi_f, coh, valid, looks, lut=lut, want=True)
    m, n = np.shape(psi)
    r = ref_index(valid, m, n)
    ref = divmod(int(r), n) if 0 <= r < m * n else None
    K, phi = transfer_ambiguity(psi, valid, psi_f, out["K"], ref=ref)
    if want:
        out.update(psi_f=psi_f, K_f=out["K"], K=K, phi=phi)
        return out
    return K, phi, out["total"]


# ----------------------------------------------------------------- bridging ---

def regions(valid):
    """4-connected regions of valid pixels, numbered 1, 2, ... in row-major
    order of their first pixel (0 = invalid): the component labelling of
    Section II-D with every edge between two valid pixels taken as reliable
    and no size cut.  Returns (labels uint32 [m, n], R)."""
    valid = np.ascontiguousarray(np.asarray(valid, np.uint8))
    m, n = valid.shape
    zx = np.zeros((m, max(n - 1, 0)), np.int8)
    zy = np.zeros((max(m - 1, 0), n), np.int8)
    big = [np.full(zx.shape, 32767, np.int16), np.full(zx.shape, 32767, np.int16),
           np.full(zy.shape, 32767, np.int16), np.full(zy.shape, 32767, np.int16)]
    return connected_components(zx, zy, big, valid, threshold=0, min_size_frac=0.0)


def _boundary(lab, r):
    """Pixels of region r with a 4-neighbour inside the image outside r: the
    only pixels that can be closest to anything outside r."""
    m, n = lab.shape
    own = lab == r
    out = np.zeros_like(own)
    out[:, 1:] |= own[:, 1:] & ~own[:, :-1]
    out[:, :-1] |= own[:, :-1] & ~own[:, 1:]
    out[1:, :] |= own[1:, :] & ~own[:-1, :]
    out[:-1, :] |= own[:-1, :] & ~own[1:, :]
    return np.flatnonzero(out)


def bridge(psi, valid, K, half_window=32, nodata=float("nan"), want=False):
    """Bridging of mask-separated regions (Section II-D), exact and slow.

    Regions (see regions()) are ranked by decreasing size, ties by label.
    Region k >= 1 attaches to the region of rank < k holding the pixel
    closest to it: the pair (p in region k, q of lower rank) minimising
    (|p - q|^2, index p, index q), indices row-major.  For each such edge the
    lower medians of phi = psi + 2 pi K (float64) over the pixels of the same
    region in the (2 half_window + 1)^2 square windows centred on q and on p
    give the offset d = floor((med_q - med_p) / 2 pi + 1/2); the region's
    shift is its parent's shift plus d, the largest region keeps 0.
    Returns (K + shift at valid pixels, phi, R) and, when want, the edges as
    a list of (rank, p, q, parent rank, d, shift)."""
    psi = np.asarray(psi, np.float32)
    m, n = psi.shape
    K = np.asarray(K, np.int64)
    lab, R = regions(valid)
    lab = lab.astype(np.int64)
    v = lab > 0
    Kout = K.copy()
    edges = []
    if R > 0:
        sizes = np.bincount(lab.ravel(), minlength=R + 1)[1:]
        order = sorted(range(1, R + 1), key=lambda r: (-int(sizes[r - 1]), r))
        rank_of = np.empty(R + 1, np.int64)
        for k, r in enumerate(order):
            rank_of[r] = k
        rank = np.where(v, rank_of[lab], -1)
        phi64 = psi.astype(np.float64) + 2.0 * np.pi * K.astype(np.float64)
        bnd = {r: _boundary(lab, r) for r in range(1, R + 1)}
        shift = np.zeros(R, np.int64)
        lower = np.zeros(0, np.int64)

        def lower_median(c, rr):
            i, j = divmod(int(c), n)
            sl = (slice(max(0, i - half_window), i + half_window + 1),
                  slice(max(0, j - half_window), j + half_window + 1))
            vals = np.sort(phi64[sl][lab[sl] == rr])
            return vals[(vals.size - 1) // 2]

        for k, r in enumerate(order):
            if k > 0:
                P = bnd[r]
                best = None
                for c0 in range(0, P.size, 256):
                    pp = P[c0:c0 + 256]
                    di = (pp[:, None] // n) - (lower[None, :] // n)
                    dj = (pp[:, None] % n) - (lower[None, :] % n)
                    d2 = di * di + dj * dj
                    a = np.lexsort((np.broadcast_to(lower[None, :], d2.shape).ravel(),
                                    np.broadcast_to(pp[:, None], d2.shape).ravel(), d2.ravel()))[0]
                    cand = (int(d2.ravel()[a]), int(pp[a // lower.size]), int(lower[a % lower.size]))
                    if best is None or cand < best:
                        best = cand
                _, p, q = best
                rq = int(lab.ravel()[q])
                d = int(np.floor((lower_median(q, rq) - lower_median(p, r)) / (2.0 * np.pi) + 0.5))
                shift[k] = shift[rank_of[rq]] + d
                edges.append((k, p, q, int(rank_of[rq]), d, int(shift[k])))
            lower = np.sort(np.concatenate([lower, bnd[r]]))
        Kout = np.where(v, K + shift[np.maximum(rank, 0)], K)
    Kout = Kout.astype(np.int32)
    phi = np.where(v, psi.astype(np.float64) + 2.0 * np.pi * Kout.astype(np.float64),
                   nodata).astype(np.float32)
    if want:
        return Kout, phi, int(R), edges
    return Kout, phi, int(R)
