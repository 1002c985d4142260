"""Pins of the oracle's cost-table construction (Section II-B, eqs. 4-7)."""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate as si
from scipy.special import erf

import oracle


def lee_published(eta, g, L, dps=300):
    """Lee et al. (1994) two-term multilook phase density at high precision
    (the naive form cancels catastrophically in the tails, so 300 digits)."""
    with mp.workdps(dps):
        eta, g = mp.mpf(eta), mp.mpf(g)
        b = g * mp.cos(eta)
        t1 = mp.gamma(L + mp.mpf(1) / 2) * (1 - g * g) ** L * b / (
            2 * mp.sqrt(mp.pi) * mp.gamma(L) * (1 - b * b) ** (L + mp.mpf(1) / 2))
        t2 = (1 - g * g) ** L / (2 * mp.pi) * mp.hyp2f1(L, 1, mp.mpf(1) / 2, b * b)
        return t1 + t2


@pytest.mark.parametrize("L", [2, 3, 9, 15, 64])
@pytest.mark.parametrize("g", [0.0, 0.3, 0.7, 0.95, 0.9999])
def test_f_eta_matches_published_form(L, g):
    for eta in [0.0, 0.2, 1.0, 1.7, 2.5, 3.0, math.pi]:
        ref = lee_published(eta, g, L)
        got = oracle.f_eta(eta, g, L)
        assert got > 0
        assert abs(got - float(ref)) <= 1e-12 * float(ref), (eta, got, ref)


def test_f_eta_single_look_closed_form():
    # L = 1: (1-g^2)/(2 pi (1-b^2)) [1 + b arccos(-b)/sqrt(1-b^2)]
    for g in [0.1, 0.5, 0.8]:
        for eta in np.linspace(-3.1, 3.1, 13):
            b = g * math.cos(eta)
            ref = (1 - g * g) / (2 * math.pi * (1 - b * b)) * (1 + b * math.acos(-b) / math.sqrt(1 - b * b))
            assert abs(oracle.f_eta(eta, g, 1) - ref) <= 1e-13 * ref


def test_f_eta_uniform_at_zero_coherence_and_normalised():
    for L in [2, 9, 40]:
        assert abs(oracle.f_eta(1.234, 0.0, L) - 1 / (2 * math.pi)) < 1e-15
        for g in [0.2, 0.6, 0.9]:
            val, _ = si.quad(lambda e: oracle.f_eta(e, g, L), -math.pi, math.pi, limit=400,
                             points=[0.0], epsabs=1e-14, epsrel=1e-13)
            assert abs(val - 1.0) < 1e-11


@pytest.mark.parametrize("L", [2, 5, 15, 64])
def test_touzi_normalised_and_finite_form(L):
    for g in [0.0, 0.4, 0.9]:
        val, _ = si.quad(lambda x: oracle.touzi(x, g, L), 0, 1, limit=400, epsabs=1e-13)
        assert abs(val - 1.0) < 1e-9
    with mp.workdps(40):
        for g, gh in [(0.3, 0.5), (0.9, 0.85), (0.99, 0.97)]:
            x = mp.mpf(g) ** 2 * mp.mpf(gh) ** 2
            ref = 2 * (L - 1) * (1 - mp.mpf(g) ** 2) ** L * gh * (1 - mp.mpf(gh) ** 2) ** (L - 2) \
                * mp.hyp2f1(L, L, 1, x)
            got = oracle.touzi(gh, g, L)
            assert abs(got - float(ref)) <= 1e-11 * float(ref)


def test_gauss_legendre_nodes():
    for n in [1, 2, 8, 16, 33]:
        x, w = oracle.gauss_legendre(n)
        xr, wr = np.polynomial.legendre.leggauss(n)
        assert np.allclose(x, xr, atol=1e-14) and np.allclose(w, wr, atol=1e-14)


def test_sigma_alpha_uniform_limit():
    """Section II-B: sigma_alpha -> pi/sqrt(3) as coherence -> 0."""
    s = oracle.sigma_alpha(0.0, 9)
    # midpoint rule of eta^2/(2pi) on 2048 cells: exact value minus deta^2/12
    deta = 2 * math.pi / 2048
    assert abs(s ** 2 - (math.pi ** 2 / 3 - deta ** 2 / 12)) < 1e-12
    assert abs(s - math.pi / math.sqrt(3)) < 1e-5
    # decreasing with coherence
    sig = [oracle.sigma_alpha(g, 9) for g in [0.0, 0.3, 0.6, 0.9, 0.99]]
    assert all(a > b for a, b in zip(sig, sig[1:]))


@pytest.mark.parametrize("L,gh", [(9, 0.3), (9, 0.85), (15, 0.6), (5, 0.97)])
def test_ftilde_against_adaptive_quadrature(L, gh):
    """eq. 5 by scipy's adaptive quadrature at a few eta, normalised by the
    same integral's mass (computed on the eta midpoints)."""
    ft = oracle.ftilde(L, gh)
    N = ft.size
    deta = 2 * math.pi / N
    assert abs(ft.sum() * deta - 1.0) < 1e-12
    assert np.allclose(ft, ft[::-1], rtol=1e-12)  # symmetric in eta

    def unnorm(eta):
        v, _ = si.quad(lambda g: oracle.f_eta(eta, g, L) * oracle.touzi(gh, g, L), 0, 1,
                       limit=500, epsabs=0, epsrel=1e-11, points=[gh])
        return v
    idx = [N // 2, N // 2 + 37, N // 2 + 300, N - 1]
    etas = [-math.pi + (i + 0.5) * deta for i in idx]
    # compare shapes (ratios), which do not depend on the normalisation
    vals = np.array([unnorm(e) for e in etas])
    ratio_ref = vals / vals[0]
    ratio_got = ft[idx] / ft[idx[0]]
    assert np.allclose(ratio_got, ratio_ref, rtol=2e-7), (ratio_got, ratio_ref)


def test_edge_mass_closed_form_for_uniform_noise():
    """Uniform phase noise: the difference density is the triangle on
    (-2pi, 2pi); on the cell lattice the mass of cell s is (N-|s|)/N^2."""
    N = 256
    ft = np.full(N, 1 / (2 * math.pi))
    pm = oracle.edge_mass(ft)
    s = np.arange(-(N - 1), N)
    assert np.allclose(pm, (N - np.abs(s)) / N ** 2, rtol=1e-13, atol=0)
    assert abs(pm.sum() - 1.0) < 1e-13


def test_edge_mass_matches_library_convolution():
    ft = oracle.ftilde(9, 0.7)
    N = ft.size
    deta = 2 * math.pi / N
    pm = oracle.edge_mass(ft)
    ref = np.convolve(ft, ft[::-1]) * deta * deta
    assert np.allclose(pm, ref, rtol=1e-12, atol=1e-300)
    assert abs(pm.sum() - 1.0) < 1e-12


def _tri_tail(a):
    """P(X > a) for the triangle density (2pi - |x|)/(4 pi^2) on (-2pi, 2pi)."""
    t = 2 * math.pi
    if a >= t:
        return 0.0
    if a <= -t:
        return 1.0
    if a >= 0:
        return (t - a) ** 2 / (2 * t * t)
    return 1.0 - (t + a) ** 2 / (2 * t * t)


def test_branch_probabilities_uniform_noise_closed_form():
    N = 2048
    pm = oracle.edge_mass(np.full(N, 1 / (2 * math.pi)))
    for alpha in [-5.0, -3.0, -1.0, 0.0, 0.4, 2.0, 3.1, 4.5, 7.0]:
        q0, qp = oracle.branch_q(pm, alpha)
        qp_ref = _tri_tail(math.pi - alpha)
        q0_ref = _tri_tail(-math.pi - alpha) - _tri_tail(math.pi - alpha)
        assert abs(qp - qp_ref) < 2e-6, (alpha, qp, qp_ref)
        assert abs(q0 - q0_ref) < 2e-6, (alpha, q0, q0_ref)


def test_branch_probabilities_sum_to_one():
    pm = oracle.edge_mass(oracle.ftilde(15, 0.9))
    for alpha in np.linspace(-9, 9, 41):
        q0, qp = oracle.branch_q(pm, alpha)
        _, qm = oracle.branch_q(pm, -alpha)  # P(G < -pi) = q+(-alpha) for symmetric noise
        assert abs(q0 + qp + qm - 1.0) < 1e-12
        assert q0 >= 0 and qp >= 0


def test_slope_marginal_uniform_noise_against_quadrature():
    """eq. 7 with uniform phase noise: integrate the closed-form q_j against
    the Gaussian truncated to +-8 sigma and renormalised."""
    N = 2048
    pm = oracle.edge_mass(np.full(N, 1 / (2 * math.pi)))
    sig = math.pi / math.sqrt(3)
    norm = erf(8 / math.sqrt(2))
    for ah in [-2.5, 0.0, 1.3, 3.0]:
        P0, Pp = oracle.slope_marginal(pm, ah, sig)

        def w(a):
            return math.exp(-0.5 * ((a - ah) / sig) ** 2) / (sig * math.sqrt(2 * math.pi) * norm)
        lo, hi = ah - 8 * sig, ah + 8 * sig
        brk = sorted(x for x in [-3 * math.pi, -math.pi, math.pi, 3 * math.pi] if lo < x < hi)
        Pp_ref, _ = si.quad(lambda a: _tri_tail(math.pi - a) * w(a), lo, hi, points=brk, limit=200)
        P0_ref, _ = si.quad(lambda a: (_tri_tail(-math.pi - a) - _tri_tail(math.pi - a)) * w(a),
                            lo, hi, points=brk, limit=200)
        assert abs(Pp - Pp_ref) < 1e-5 and abs(P0 - P0_ref) < 1e-5, (ah, Pp, Pp_ref, P0, P0_ref)


@pytest.fixture(scope="module")
def lut_probs():
    return oracle.build_lut(9, want_probs=True)


def test_lut_costs_match_probabilities(lut_probs):
    T, P0, Pp, _ = lut_probs
    c = np.maximum(0.0, -np.log(Pp / P0))
    want = np.minimum(32767, np.floor(100 * c)).astype(np.int16)
    assert np.array_equal(T, want)
    assert T.min() >= 0


def test_lut_shape_properties(lut_probs):
    """Section II-B: near +pi a +1 correction is cheap, near -pi expensive; a
    gradient near zero is expensive both ways; costs grow with coherence."""
    T, P0, Pp, _ = lut_probs
    NG, NA = T.shape
    for row in T:
        assert np.all(np.diff(row.astype(int)) <= 0)  # c+ non-increasing in alpha_hat
    mid = NA // 2
    assert np.all(np.diff(T[:, mid].astype(int)) >= 0)  # c(alpha~0) non-decreasing in gamma
    # -1 correction near -pi (mirror bin) cheaper than +1 there, at high coherence
    hi = NG - 8
    assert T[hi, NA - 1] < T[hi, 0]
    assert T[0, mid] < T[hi, mid]


def test_lut_rejects_bad_looks():
    with pytest.raises(oracle.OracleError):
        oracle.build_lut(1)
    with pytest.raises(oracle.OracleError):
        oracle.build_lut(65)


def test_generator_phase_matches_f_eta_monte_carlo():
    """The generator's L-look phase at fixed true coherence follows f_eta
    (chi-square on 32 bins), tying the synthetic inputs to the cost model."""
    from scipy.stats import chi2
    from paper_2609_36267_amd import synth
    L, g = 9, 0.6
    m = n = 256
    _, psi, coh = synth.simulate_looks(np.zeros((m, n)), np.full((m, n), g, np.float32), L, 123,
                                       workers=1)
    edges = np.linspace(-math.pi, math.pi, 33)
    obs, _ = np.histogram(psi.astype(np.float64), bins=edges)
    exp_ = np.array([si.quad(lambda e: oracle.f_eta(e, g, L), a, b)[0] for a, b in zip(edges, edges[1:])])
    exp_ *= psi.size
    stat = ((obs - exp_) ** 2 / exp_).sum()
    assert stat < chi2.ppf(0.999, 31)
    # and the sample coherence follows the Touzi density
    cedges = np.linspace(0, 1, 21)
    cobs, _ = np.histogram(coh.astype(np.float64), bins=cedges)
    cexp = np.array([si.quad(lambda x: oracle.touzi(x, g, L), a, b)[0] for a, b in zip(cedges, cedges[1:])])
    cexp *= coh.size
    keep = cexp > 5
    cstat = ((cobs[keep] - cexp[keep]) ** 2 / cexp[keep]).sum()
    assert cstat < chi2.ppf(0.999, keep.sum() - 1)
