"""The C-ABI library loads on a machine without a GPU and exports every entry
point that include/ww.h declares (no compute call is made here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ww.h")
LIB = os.path.join(ROOT, "paper_2609_36267_amd", "libww.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ww_[a-z_]+)\s*\(", text)))


def test_header_declares_the_six_calls():
    names = declared_functions()
    for f in ["ww_residues", "ww_build_cost_lut", "ww_edge_costs", "ww_mcf_solve",
              "ww_integrate", "ww_unwrap", "ww_last_error"]:
        assert f in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libww.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (ww_[a-z_]+)\b", out))
    for f in declared_functions():
        assert f in exported, f
        assert hasattr(lib, f)
    from paper_2609_36267_amd import binding
    assert set(binding.EXPORTS) <= exported


@pytest.mark.skipif(not os.path.exists(LIB), reason="libww.so not built")
def test_defaults_and_version_without_gpu():
    from paper_2609_36267_amd import binding
    lp = binding.default_lut_params()
    assert (lp.n_alpha, lp.n_gamma, lp.n_eta, lp.n_aquad) == (128, 64, 2048, 513)
    cp = binding.default_cost_params()
    assert cp.box_half == 2 and cp.steep_cap_pct == 3 and cp.ref_i == -1
    assert cp.lut_interp == 0  # nearest table bin unless asked
    assert binding.load().ww_version().startswith(b"ww-gfx950")


@pytest.mark.skipif(not os.path.exists(LIB), reason="libww.so not built")
def test_argument_errors_are_reported_without_touching_the_gpu():
    from paper_2609_36267_amd import binding
    L = binding.load()
    assert L.ww_residues(None, None, 0, 5, None, None, None, None) == binding.E_INVALID_ARG
    assert b"shape" in L.ww_last_error()
    assert L.ww_build_cost_lut(1, None, None) == binding.E_INVALID_ARG
    assert L.ww_unwrap(None, None, None, 4, 4, 9, None, None, None, None, None) == binding.E_INVALID_ARG
    bad = binding.default_cost_params(lut_interp=2)
    assert L.ww_edge_costs(None, None, None, 4, 4, None, None, ctypes.byref(bad),
                           None, None, None, None, None) == binding.E_INVALID_ARG
    assert b"lut_interp" in L.ww_last_error()


def test_product_path_has_no_oracle_dependency():
    """Nothing under the package imports or loads the oracle."""
    pkg = os.path.join(ROOT, "paper_2609_36267_amd")
    for dp, _, fs in os.walk(pkg):
        for f in fs:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dp, f)).read()
                assert "oracle" not in txt.lower() or f == "synth.py", f


def test_mcf_schedule_round_trip_and_range():
    """The solve schedule is host state: settable without a GPU."""
    from paper_2609_36267_amd import binding as ww
    old = ww.get_mcf_params()
    try:
        ww.set_mcf_params(16, 4096)
        p = ww.get_mcf_params()
        assert (p.first_hop_window, p.first_distance_step) == (16, 4096)
        ww.set_mcf_params(full_passes=8, first_deficit_after=1)
        assert ww.get_mcf_params().as_tuple() == (16, 4096, 8, 1, 0, 2, 32)
        ww.set_mcf_params(hop_growth=8)
        assert ww.get_mcf_params().as_tuple() == (16, 4096, 8, 1, 0, 8, 32)
        for bad in ((0, 256), (64, 0), (64, (1 << 30) + 1), (1 << 29, 256), (64, 256, -1, 0),
                    (64, 256, (1 << 20) + 1, 0), (64, 256, 0, 2), (64, 256, 0, 0, -1),
                    (64, 256, 0, 0, 0, 1), (64, 256, 0, 0, 0, (1 << 20) + 1),
                    (64, 256, 0, 0, 0, 2, 48), (64, 256, 0, 0, 0, 2, 128), (64, 256, 0, 0, 0, 2, 0)):
            with pytest.raises(ww.WWError):
                ww.set_mcf_params(*bad)
        assert ww.get_mcf_params().as_tuple() == (16, 4096, 8, 1, 0, 8, 32)
        ww.set_mcf_params(tile_cols=64)
        assert ww.get_mcf_params().tile_cols == 64
        ww.set_mcf_params(tile_cols=16)
        assert ww.get_mcf_params().as_tuple() == (16, 4096, 8, 1, 0, 8, 16)
        d = ww.McfParams()
        ww.load().ww_default_mcf_params(ctypes.byref(d))
        assert d.as_tuple() == (64, 256, 0, 0, 0, 2, 32)
    finally:
        ww.set_mcf_params(*old.as_tuple())
