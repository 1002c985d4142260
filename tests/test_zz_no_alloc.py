"""ww_integrate_noalloc against ww_integrate, through the C ABI: two calls in
a row on the same device, the second on a smaller image, and the limit."""
import ctypes as C
import math

import numpy as np
import pytest

import oracle
from paper_2609_36267_amd import binding as ww
from paper_2609_36267_amd import synth

pytestmark = pytest.mark.gpu


def _case(m, n, seed):
    sc = synth.make(m, n, looks=9, seed=seed, mask_frac=0.05, disks=1, disk_radius=(10, 20),
                    keep_truth=False, workers=1)
    T = oracle.build_lut(9)
    out = oracle.unwrap(sc.psi, sc.coh, sc.valid, 9, lut=T, want=True)
    return sc, out


def test_noalloc_matches_integrate_twice():
    import torch
    assert torch.cuda.is_available()
    lib = ww.load()
    for (m, n, seed, ref) in ((300, 517, 3, None), (97, 130, 4, (5, 7))):
        sc, out = _case(m, n, seed)
        psi = torch.from_numpy(sc.psi).cuda()
        valid = torch.from_numpy(sc.valid).cuda()
        dkx = torch.from_numpy(out["dkx"]).cuda()
        dky = torch.from_numpy(out["dky"]).cuda()
        K_ref, phi_ref = ww.integrate(psi, valid, dkx, dky, ref=ref)
        K = torch.full((m, n), -7, dtype=torch.int32, device="cuda")
        phi = torch.full((m, n), 1.5, dtype=torch.float32, device="cuda")
        cp = ww.default_cost_params()
        if ref is not None:
            cp.ref_i, cp.ref_j = ref
        torch.cuda.synchronize()
        rc = lib.ww_integrate_noalloc(ww._ptr(psi), ww._ptr(valid), ww._ptr(dkx), ww._ptr(dky),
                                      m, n, C.byref(cp), ww._ptr(K), ww._ptr(phi), ww._stream())
        assert rc == 0, lib.ww_last_error()
        torch.cuda.synchronize()
        assert np.array_equal(K.cpu().numpy(), K_ref.cpu().numpy())
        assert phi.cpu().numpy().tobytes() == phi_ref.cpu().numpy().tobytes()
        if ref is None:  # the oracle's integration of the same cycle differences
            assert np.array_equal(K.cpu().numpy(), out["K"])


def test_noalloc_rejects_rows_above_limit():
    import torch
    lib = ww.load()
    m, n = 65537, 2
    t = torch.zeros(1, dtype=torch.float32, device="cuda")
    rc = lib.ww_integrate_noalloc(ww._ptr(t), None, ww._ptr(t), ww._ptr(t), m, n, None,
                                  ww._ptr(t), ww._ptr(t), ww._stream())
    assert rc == ww.E_INVALID_ARG
    assert b"65536" in lib.ww_last_error()
