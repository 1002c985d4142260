"""Thin ctypes binding over ``libww.so`` (the C ABI declared in include/ww.h).

PyTorch only supplies device memory and the current HIP stream; every step of
the computation runs in the library's HIP kernels.  There is no fallback: if
the library is missing or no GPU is present the calls raise.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import threading
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libww.so")
_lock = threading.Lock()
_lib = None

OK, E_INVALID_ARG, E_OOM, E_INFEASIBLE, E_DEVICE, E_OVERFLOW = 0, -1, -2, -3, -4, -5
_NAMES = {E_INVALID_ARG: "WW_E_INVALID_ARG", E_OOM: "WW_E_OOM", E_INFEASIBLE: "WW_E_INFEASIBLE",
          E_DEVICE: "WW_E_DEVICE", E_OVERFLOW: "WW_E_OVERFLOW"}

EXPORTS = ["ww_last_error", "ww_version", "ww_last_mcf_stats", "ww_default_lut_params", "ww_default_cost_params",
           "ww_residues", "ww_build_cost_lut", "ww_edge_costs", "ww_mcf_solve", "ww_integrate",
           "ww_unwrap"]


class WWError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class LutParams(C.Structure):
    _fields_ = [("n_alpha", C.c_int32), ("n_gamma", C.c_int32), ("n_eta", C.c_int32),
                ("n_gpanel", C.c_int32), ("n_gnode", C.c_int32), ("n_aquad", C.c_int32),
                ("sigma_span", C.c_double)]


class CostParams(C.Structure):
    _fields_ = [("box_half", C.c_int32), ("steep_rule", C.c_int32),
                ("steep_thresh_rad", C.c_double), ("steep_cap_pct", C.c_int32),
                ("ref_i", C.c_int32), ("ref_j", C.c_int32), ("nodata", C.c_float)]


class McfStats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("passes", "windows", "rounds", "tile_visits",
                                         "augmentations", "path_arcs", "supplies",
                                         "max_potential")] + [("relax_ms", C.c_double),
                                                              ("solve_ms", C.c_double)]

    def as_dict(self):
        return {k: (float(getattr(self, k)) if t is C.c_double else int(getattr(self, k)))
                for k, t in self._fields_}


def last_mcf_stats() -> dict:
    st = McfStats()
    load().ww_last_mcf_stats(C.byref(st))
    return st.as_dict()


def load(path: str = LIB_PATH):
    """Load the library (raises if it was not built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(path):
                raise ImportError(f"HIP library {path} is missing: run "
                                  "`python -m paper_2609_36267_amd.build` first")
            lib = C.CDLL(path)
            _declare(lib)
            _lib = lib
    return _lib


def _declare(L):
    P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
    L.ww_last_error.restype = C.c_char_p
    L.ww_version.restype = C.c_char_p
    L.ww_last_mcf_stats.argtypes = [P]
    L.ww_default_lut_params.argtypes = [P]
    L.ww_default_cost_params.argtypes = [P]
    L.ww_residues.argtypes = [P, P, I32, I32, P, P, P, P]
    L.ww_build_cost_lut.argtypes = [I32, P, P]
    L.ww_edge_costs.argtypes = [P, P, P, I32, I32, P, P, P, P, P, P, P, P]
    L.ww_mcf_solve.argtypes = [P, I32, I32, P, P, P, P, P, P, P, P, P, P]
    L.ww_integrate.argtypes = [P, P, P, P, I32, I32, P, P, P, P]
    L.ww_unwrap.argtypes = [P, P, P, I32, I32, I32, P, P, P, P, P]
    for f in ("ww_residues", "ww_build_cost_lut", "ww_edge_costs", "ww_mcf_solve",
              "ww_integrate", "ww_unwrap"):
        getattr(L, f).restype = C.c_int32


def _check(rc):
    if rc != OK:
        raise WWError(rc, load().ww_last_error().decode())


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the HIP unwrapper needs a GPU (torch.cuda.is_available() is False)")
    return torch


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("arrays must be contiguous device tensors")
    return C.c_void_p(t.data_ptr())


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def default_lut_params() -> LutParams:
    p = LutParams()
    load().ww_default_lut_params(C.byref(p))
    return p


def default_cost_params(**kw) -> CostParams:
    p = CostParams()
    load().ww_default_cost_params(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _dev(a, dtype):
    """Move a numpy array / tensor to the current device with the given dtype."""
    torch = _torch()
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        a = torch.from_numpy(np.ascontiguousarray(a))
    return a.to(device="cuda", dtype=dtype).contiguous()


# ------------------------------------------------------------- the calls ---

def residues(psi, valid=None):
    """(res int8 [m-1, n-1], perim int8 [2(n-1)+2(m-1)], ground charge)."""
    torch = _torch()
    psi = _dev(psi, torch.float32)
    valid = _dev(valid, torch.uint8)
    m, n = psi.shape
    res = torch.empty((max(m - 1, 0), max(n - 1, 0)), dtype=torch.int8, device="cuda")
    perim = torch.empty((max(2 * (n - 1) + 2 * (m - 1), 0),), dtype=torch.int8, device="cuda")
    g = C.c_int64(0)
    _check(load().ww_residues(_ptr(psi), _ptr(valid), m, n, _ptr(res) if res.numel() else None,
                              _ptr(perim) if perim.numel() else None, C.byref(g), _stream()))
    return res, perim, int(g.value)


def build_cost_lut(looks, params: LutParams | None = None) -> np.ndarray:
    p = params or default_lut_params()
    out = np.zeros((p.n_gamma, p.n_alpha), np.int16)
    _check(load().ww_build_cost_lut(int(looks), C.byref(p), out.ctypes.data_as(C.c_void_p)))
    return out


def edge_costs(psi, coh, valid, lut, params: CostParams | None = None,
               lut_params: LutParams | None = None):
    """Four int16 planes (cx_pos, cx_neg [m, n-1], cy_pos, cy_neg [m-1, n])."""
    torch = _torch()
    psi = _dev(psi, torch.float32)
    coh = _dev(coh, torch.float32)
    valid = _dev(valid, torch.uint8)
    lut = _dev(lut, torch.int16)
    m, n = psi.shape
    cp = params or default_cost_params()
    lp = lut_params or default_lut_params()
    cxp = torch.empty((m, max(n - 1, 0)), dtype=torch.int16, device="cuda")
    cxn = torch.empty_like(cxp)
    cyp = torch.empty((max(m - 1, 0), n), dtype=torch.int16, device="cuda")
    cyn = torch.empty_like(cyp)
    nz = lambda t: _ptr(t) if t.numel() else None  # noqa: E731
    _check(load().ww_edge_costs(_ptr(psi), _ptr(coh), _ptr(valid), m, n, _ptr(lut), C.byref(lp),
                                C.byref(cp), nz(cxp), nz(cxn), nz(cyp), nz(cyn), _stream()))
    return cxp, cxn, cyp, cyn


@dataclass
class McfResult:
    dk_x: object
    dk_y: object
    total_cost: int
    potentials: object
    stats: dict


def mcf_solve(res, costs, m, n, want_potentials=False) -> McfResult:
    torch = _torch()
    res = _dev(res, torch.int8)
    cxp, cxn, cyp, cyn = [_dev(c, torch.int16) for c in costs]
    dkx = torch.empty((m, max(n - 1, 0)), dtype=torch.int8, device="cuda")
    dky = torch.empty((max(m - 1, 0), n), dtype=torch.int8, device="cuda")
    pot = (torch.empty((max(m - 1, 0) * max(n - 1, 0) + 1,), dtype=torch.int64, device="cuda")
           if want_potentials else None)
    tot = C.c_int64(0)
    st = McfStats()
    nz = lambda t: _ptr(t) if (t is not None and t.numel()) else None  # noqa: E731
    _check(load().ww_mcf_solve(nz(res), m, n, nz(cxp), nz(cxn), nz(cyp), nz(cyn), nz(dkx),
                               nz(dky), nz(pot), C.byref(tot), C.byref(st), _stream()))
    return McfResult(dkx, dky, int(tot.value), pot, st.as_dict())


def integrate(psi, valid, dkx, dky, ref=None, nodata=math.nan):
    torch = _torch()
    psi = _dev(psi, torch.float32)
    valid = _dev(valid, torch.uint8)
    dkx = _dev(dkx, torch.int8)
    dky = _dev(dky, torch.int8)
    m, n = psi.shape
    cp = default_cost_params(nodata=nodata)
    if ref is not None:
        cp.ref_i, cp.ref_j = ref
    K = torch.empty((m, n), dtype=torch.int32, device="cuda")
    phi = torch.empty((m, n), dtype=torch.float32, device="cuda")
    nz = lambda t: _ptr(t) if t.numel() else None  # noqa: E731
    _check(load().ww_integrate(_ptr(psi), _ptr(valid), nz(dkx), nz(dky), m, n, C.byref(cp),
                               _ptr(K), _ptr(phi), _stream()))
    return K, phi


def unwrap(psi, coh, valid, looks, params: CostParams | None = None, out=None):
    """Whole path on the device.  Returns (K, phi, total_cost)."""
    torch = _torch()
    psi = _dev(psi, torch.float32)
    coh = _dev(coh, torch.float32)
    valid = _dev(valid, torch.uint8)
    m, n = psi.shape
    if out is None:
        K = torch.empty((m, n), dtype=torch.int32, device="cuda")
        phi = torch.empty((m, n), dtype=torch.float32, device="cuda")
    else:
        K, phi = out
    tot = C.c_int64(0)
    cp = params or default_cost_params()
    _check(load().ww_unwrap(_ptr(psi), _ptr(coh), _ptr(valid), m, n, int(looks), C.byref(cp),
                            _ptr(K), _ptr(phi), C.byref(tot), _stream()))
    return K, phi, int(tot.value)
