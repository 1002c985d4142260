"""The input generators: shapes, ranges, seeding, and agreement of the
device-drawn recipe with the host one in distribution."""
import numpy as np
import pytest

from paper_2609_36267_amd import synth


def test_host_recipe_is_seeded():
    a = synth.make(40, 56, looks=9, seed=11, disks=2, disk_radius=(5, 10), mask_frac=0.05,
                   keep_truth=False, workers=1)
    b = synth.make(40, 56, looks=9, seed=11, disks=2, disk_radius=(5, 10), mask_frac=0.05,
                   keep_truth=False, workers=1)
    assert np.array_equal(a.psi, b.psi) and np.array_equal(a.coh, b.coh)
    assert np.array_equal(a.valid, b.valid)


@pytest.fixture(scope="module")
def drawn():
    torch = pytest.importorskip("torch")
    torch.set_num_threads(4)
    return synth.make_device(48, 40, looks=9, seed=5, disks=2, disk_radius=(4, 8), mask_frac=0.05,
                             device="cpu", rows_per_draw=16)


def test_device_recipe_shapes_and_ranges(drawn):
    import torch
    psi, coh, valid = drawn
    assert psi.shape == coh.shape == valid.shape == (48, 40)
    assert psi.dtype == torch.float32 and coh.dtype == torch.float32 and valid.dtype == torch.uint8
    pi32 = float(np.float32(np.pi))
    assert float(psi.abs().max()) <= pi32
    assert float(coh.min()) >= 0.0 and float(coh.max()) <= 1.0 + 1e-6
    assert set(valid.unique().tolist()) <= {0, 1}


def test_device_recipe_is_seeded(drawn):
    psi2, coh2, valid2 = synth.make_device(48, 40, looks=9, seed=5, disks=2, disk_radius=(4, 8),
                                           mask_frac=0.05, device="cpu", rows_per_draw=16)
    assert bool((drawn[0] == psi2).all()) and bool((drawn[1] == coh2).all())
    assert bool((drawn[2] == valid2).all())


def test_device_recipe_matches_host_recipe_in_distribution():
    """Same recipe, other random numbers: the mask is the same draw, and
    at one coherence (the smooth field is then constant) the wrapped-phase
    gradients and the sample coherence agree in distribution."""
    import torch
    torch.set_num_threads(4)
    m, n = 96, 80
    kw = dict(looks=9, seed=3, coh_lo=0.6, coh_hi=0.6, mask_frac=0.05)
    h = synth.make(m, n, keep_truth=False, workers=1, **kw)
    d = synth.make_device(m, n, device="cpu", rows_per_draw=32, **kw)
    assert np.array_equal(h.valid, d[2].numpy())

    def grad_ms(psi):
        g = np.diff(psi.astype(np.float64), axis=1)
        g = (g + np.pi) % (2 * np.pi) - np.pi
        return float((g ** 2).mean())

    a, b = grad_ms(h.psi), grad_ms(d[0].numpy())
    assert abs(a - b) < 0.1 * a
    assert abs(float(h.coh.mean()) - float(d[1].mean())) < 0.02
