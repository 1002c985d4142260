"""Pins of the oracle's Goldstein preprocessing and of the transfer of cycle
counts back to the original phase (Section II-D)."""
import numpy as np
import pytest

import oracle


def wrapdiff(a, b):
    d = np.asarray(a, np.float64) - np.asarray(b, np.float64)
    return np.angle(np.exp(1j * d))


def noisy_ramp(seed, m, n, sigma=0.8):
    rng = np.random.default_rng(seed)
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    clean = 0.21 * j + 0.13 * i + 3.0 * np.sin(i / 11.0) * np.cos(j / 13.0)
    noisy = clean + rng.normal(0, sigma, (m, n))
    return (np.angle(np.exp(1j * noisy)).astype(np.float32),
            np.angle(np.exp(1j * clean)).astype(np.float32))


def test_taper_is_a_partition_of_unity():
    for N in (4, 8, 32, 64):
        w = oracle.triangle_taper(N)
        assert np.all(w > 0)
        assert np.allclose(w[: N // 2] + w[N // 2:], 1.0, atol=0, rtol=0)


@pytest.mark.parametrize("N", [8, 32])
def test_alpha_zero_is_the_identity(N):
    """H = 1 everywhere: each patch returns its own phasors, and the taper
    only rescales the sum."""
    psi, _ = noisy_ramp(1, 45, 70)
    valid = (np.random.default_rng(2).random(psi.shape) > 0.2).astype(np.uint8)
    f = oracle.goldstein(psi, valid, alpha=0.0, patch=N)
    v = valid.astype(bool)
    assert np.abs(wrapdiff(f, psi)[v]).max() < 1e-6
    assert np.array_equal(f[~v], psi[~v])


@pytest.mark.parametrize("alpha", [0.5, 1.0, 2.0])
def test_plane_wave_on_the_dft_grid_passes_unchanged(alpha):
    """A plane wave with a whole number of cycles per patch has a one-bin
    spectrum there, where H = 1: patches that lie inside the image return it
    exactly, so pixels covered only by such patches keep their phase."""
    N, S = 32, 16
    m, n = 6 * S, 8 * S
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    psi = np.angle(np.exp(2j * np.pi * (3 * i + 5 * j) / N)).astype(np.float32)
    f = oracle.goldstein(psi, None, alpha=alpha, patch=N)
    inner = (slice(S, m - S), slice(S, n - S))
    assert np.abs(wrapdiff(f[inner], psi[inner])).max() < 1e-6


def _dft_filter_brute(psi, valid, alpha, N, smooth):
    """The same filter from explicit DFT sums and explicit loops (tiny N)."""
    m, n = psi.shape
    S = N // 2
    z = np.where(valid.astype(bool), np.exp(1j * psi.astype(np.float64)), 0)
    w = [1 - abs(2 * a + 1 - N) / N for a in range(N)]
    acc = np.zeros((m, n), complex)
    h = smooth // 2
    for pi in range((m + S - 1) // S + 1):
        for pj in range((n + S - 1) // S + 1):
            r0, c0 = pi * S - S, pj * S - S
            x = np.zeros((N, N), complex)
            for a in range(N):
                for b in range(N):
                    if 0 <= r0 + a < m and 0 <= c0 + b < n:
                        x[a, b] = z[r0 + a, c0 + b]
            Z = np.zeros((N, N), complex)
            for u in range(N):
                for v in range(N):
                    Z[u, v] = sum(x[a, b] * np.exp(-2j * np.pi * (u * a + v * b) / N)
                                  for a in range(N) for b in range(N))
            B = np.zeros((N, N))
            for u in range(N):
                for v in range(N):
                    B[u, v] = sum(abs(Z[(u + du) % N, (v + dv) % N])
                                  for du in range(-h, h + 1) for dv in range(-h, h + 1)) / smooth ** 2
            if B.max() <= 0:
                continue
            Y = Z * (B / B.max()) ** alpha
            for a in range(N):
                for b in range(N):
                    if 0 <= r0 + a < m and 0 <= c0 + b < n:
                        y = sum(Y[u, v] * np.exp(2j * np.pi * (u * a + v * b) / N)
                                for u in range(N) for v in range(N)) / N ** 2
                        acc[r0 + a, c0 + b] += w[a] * w[b] * y
    return acc


@pytest.mark.parametrize("N,smooth", [(4, 3), (8, 3), (8, 5)])
def test_matches_explicit_dft_sums(N, smooth):
    rng = np.random.default_rng(N + smooth)
    m, n = 11, 13
    psi = rng.uniform(-np.pi, np.pi, (m, n)).astype(np.float32)
    valid = (rng.random((m, n)) > 0.2).astype(np.uint8)
    f, acc = oracle.goldstein(psi, valid, alpha=0.7, patch=N, smooth=smooth, want_sum=True)
    want = _dft_filter_brute(psi, valid, 0.7, N, smooth)
    assert np.allclose(acc, want, rtol=0, atol=1e-11)


def test_conjugate_symmetry():
    psi, _ = noisy_ramp(5, 50, 60)
    f = oracle.goldstein(psi, None)
    g = oracle.goldstein(-psi, None)
    assert np.abs(wrapdiff(g, -f)).max() < 1e-5


def test_filter_removes_noise_and_residues():
    psi, clean = noisy_ramp(7, 128, 160)
    rms = lambda a: float(np.sqrt(np.mean(wrapdiff(a, clean) ** 2)))  # noqa: E731
    f5 = oracle.goldstein(psi, None, alpha=0.5)
    f1 = oracle.goldstein(psi, None, alpha=1.0)
    assert rms(f1) < rms(f5) < 0.6 * rms(psi)
    r = lambda a: int(np.abs(oracle.residues(a)[0]).sum())  # noqa: E731
    assert r(f1) <= r(f5) < r(psi) // 5


def test_invalid_pixels_keep_psi():
    psi, _ = noisy_ramp(9, 40, 40)
    valid = np.zeros(psi.shape, np.uint8)
    assert np.array_equal(oracle.goldstein(psi, valid), psi)
    valid[10:30, 5:35] = 1
    f = oracle.goldstein(psi, valid)
    assert np.array_equal(f[valid == 0], psi[valid == 0])


# ------------------------------------------------------- cycle transfer ---

def test_transfer_is_the_nearest_congruent_value():
    rng = np.random.default_rng(3)
    m, n = 40, 50
    psi = rng.uniform(-np.pi, np.pi, (m, n)).astype(np.float32)
    psi_f = np.angle(np.exp(1j * (psi + rng.normal(0, 1.2, (m, n))))).astype(np.float32)
    K_f = rng.integers(-5, 6, (m, n)).astype(np.int32)
    valid = (rng.random((m, n)) > 0.1).astype(np.uint8)
    K, phi = oracle.transfer_ambiguity(psi, valid, psi_f, K_f)
    v = valid.astype(bool)
    target = psi_f.astype(np.float64) + 2 * np.pi * K_f
    # brute force over nearby integers
    cands = K_f[..., None] + np.arange(-3, 4)[None, None, :]
    dist = np.abs(psi.astype(np.float64)[..., None] + 2 * np.pi * cands - target[..., None])
    best = cands[np.arange(m)[:, None], np.arange(n)[None, :], np.argmin(dist, axis=2)]
    assert np.array_equal(K[v], best[v])
    assert np.array_equal(K[~v], K_f[~v])
    assert np.all(np.abs(phi[v] - target[v]) <= np.pi + 1e-5)
    cyc = (phi.astype(np.float64) - psi) / (2 * np.pi)
    assert np.abs(cyc[v] - K[v]).max() < 1e-5
    assert np.all(np.isnan(phi[~v]))


def test_transfer_of_an_unfiltered_phase_is_the_identity():
    rng = np.random.default_rng(4)
    psi = rng.uniform(-np.pi, np.pi, (20, 30)).astype(np.float32)
    K_f = rng.integers(-9, 9, (20, 30)).astype(np.int32)
    K, _ = oracle.transfer_ambiguity(psi, None, psi, K_f)
    assert np.array_equal(K, K_f)


def test_unwrap_filtered_keeps_the_original_phase():
    """Whole path on the filtered phase: the output is congruent to the
    original phase at every valid pixel, and far fewer residues are solved."""
    psi, clean = noisy_ramp(11, 96, 128, sigma=0.9)
    coh = np.full(psi.shape, 0.5, np.float32)
    valid = np.ones(psi.shape, np.uint8)
    out = oracle.unwrap_filtered(psi, coh, valid, 9, want=True)
    cyc = (out["phi"].astype(np.float64) - psi) / (2 * np.pi)
    assert np.abs(cyc - np.round(cyc)).max() < 1e-4
    assert np.abs(out["res"]).sum() * 5 < np.abs(oracle.residues(psi)[0]).sum()


def test_transfer_reference_shift_is_a_constant():
    rng = np.random.default_rng(6)
    m, n = 25, 31
    psi = rng.uniform(-np.pi, np.pi, (m, n)).astype(np.float32)
    psi_f = np.angle(np.exp(1j * (psi + rng.normal(0, 2.0, (m, n))))).astype(np.float32)
    K_f = rng.integers(-4, 5, (m, n)).astype(np.int32)
    K0, _ = oracle.transfer_ambiguity(psi, None, psi_f, K_f)
    for ref in ((0, 0), (7, 19), (24, 30)):
        K, phi = oracle.transfer_ambiguity(psi, None, psi_f, K_f, ref=ref)
        assert K[ref] == 0
        d = K.astype(np.int64) - K0
        assert np.all(d == d[0, 0])
