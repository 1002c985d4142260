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
           "ww_unwrap", "ww_clock", "ww_server_create", "ww_server_submit", "ww_server_poll",
           "ww_server_in_flight", "ww_server_destroy", "ww_unwrap_batch", "ww_default_mcf_params",
           "ww_set_mcf_params", "ww_get_mcf_params", "ww_default_cc_params",
           "ww_connected_components", "ww_default_filter_params", "ww_goldstein_filter",
           "ww_transfer_ambiguity", "ww_unwrap_filtered", "ww_default_bridge_params",
           "ww_bridge"]


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
                ("ref_i", C.c_int32), ("ref_j", C.c_int32), ("nodata", C.c_float),
                ("lut_interp", C.c_int32), ("looks_frac16", C.c_int32)]


class McfStats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("passes", "windows", "rounds", "tile_visits",
                                         "augmentations", "path_arcs", "supplies",
                                         "max_potential")] + [("relax_ms", C.c_double),
                                                              ("solve_ms", C.c_double),
                                                              ("settled_nodes", C.c_int64),
                                                              ("arcs_scanned", C.c_int64)]

    def as_dict(self):
        return {k: (float(getattr(self, k)) if t is C.c_double else int(getattr(self, k)))
                for k, t in self._fields_}


class CcParams(C.Structure):
    """Reliability threshold and minimum component size (ww_cc_params)."""
    _fields_ = [("threshold", C.c_int32), ("min_size_frac", C.c_double)]


def default_cc_params(**kw) -> CcParams:
    p = CcParams()
    load().ww_default_cc_params(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def connected_components(dkx, dky, costs, valid, params: CcParams | None = None):
    """(labels uint32 [m, n] device tensor, number of labelled components)."""
    torch = _torch()
    dkx = _dev(dkx, torch.int8)
    dky = _dev(dky, torch.int8)
    cxp, cxn, cyp, cyn = [_dev(c, torch.int16) for c in costs]
    valid = _dev(valid, torch.uint8)
    m, n = dkx.shape[0], dky.shape[1]
    labels = torch.empty((m, n), dtype=torch.int32, device="cuda")  # uint32 bits
    nc = C.c_int64(0)
    p = params or default_cc_params()
    nz = lambda t: _ptr(t) if (t is not None and t.numel()) else None  # noqa: E731
    _check(load().ww_connected_components(nz(dkx), nz(dky), nz(cxp), nz(cxn), nz(cyp), nz(cyn),
                                          _ptr(valid), m, n, C.byref(p), _ptr(labels),
                                          C.byref(nc), _stream()))
    return labels, int(nc.value)


class FilterParams(C.Structure):
    """Goldstein filter parameters (ww_filter_params)."""
    _fields_ = [("patch", C.c_int32), ("smooth", C.c_int32), ("alpha", C.c_float)]


def default_filter_params(**kw) -> FilterParams:
    p = FilterParams()
    load().ww_default_filter_params(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def goldstein_filter(psi, valid, params: FilterParams | None = None, out=None):
    """Filtered wrapped phase (float32 [m, n] device tensor)."""
    torch = _torch()
    psi = _dev(psi, torch.float32)
    valid = _dev(valid, torch.uint8)
    m, n = psi.shape
    if out is None:
        out = torch.empty((m, n), dtype=torch.float32, device="cuda")
    p = params or default_filter_params()
    _check(load().ww_goldstein_filter(_ptr(psi), _ptr(valid), m, n, C.byref(p), _ptr(out),
                                      _stream()))
    return out


def transfer_ambiguity(psi, valid, psi_f, K_f, ref=None, nodata=math.nan):
    """(K, phi): cycle counts of a filtered phase moved onto psi."""
    torch = _torch()
    psi = _dev(psi, torch.float32)
    valid = _dev(valid, torch.uint8)
    psi_f = _dev(psi_f, torch.float32)
    K_f = _dev(K_f, torch.int32)
    m, n = psi.shape
    K = torch.empty((m, n), dtype=torch.int32, device="cuda")
    phi = torch.empty((m, n), dtype=torch.float32, device="cuda")
    ri, rj = ref if ref is not None else (-1, -1)
    _check(load().ww_transfer_ambiguity(_ptr(psi), _ptr(valid), _ptr(psi_f), _ptr(K_f), m, n,
                                        int(ri), int(rj), float(nodata), _ptr(K), _ptr(phi),
                                        _stream()))
    return K, phi


def unwrap_filtered(psi, coh, valid, looks, params: CostParams | None = None,
                    filter_params: FilterParams | None = None, out=None):
    """The whole path on the Goldstein-filtered phase, cycle counts moved
    back onto psi.  Returns (K, phi, total_cost of the filtered problem)."""
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
    fp = filter_params or default_filter_params()
    _check(load().ww_unwrap_filtered(_ptr(psi), _ptr(coh), _ptr(valid), m, n, int(looks),
                                     C.byref(cp), C.byref(fp), _ptr(K), _ptr(phi), C.byref(tot),
                                     _stream()))
    return K, phi, int(tot.value)


class BridgeParams(C.Structure):
    """Bridging parameters (ww_bridge_params)."""
    _fields_ = [("half_window", C.c_int32)]


def default_bridge_params(**kw) -> BridgeParams:
    p = BridgeParams()
    load().ww_default_bridge_params(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def bridge(psi, valid, K, params: BridgeParams | None = None, nodata=math.nan, out=None,
           want_regions=False):
    """Bridging of mask-separated regions.  Returns (K_out, phi, nregions)
    and the region numbers (uint32 bits in an int32 tensor) when asked."""
    torch = _torch()
    psi = _dev(psi, torch.float32)
    valid = _dev(valid, torch.uint8)
    K = _dev(K, torch.int32)
    m, n = psi.shape
    if out is None:
        K_out = torch.empty((m, n), dtype=torch.int32, device="cuda")
        phi = torch.empty((m, n), dtype=torch.float32, device="cuda")
    else:
        K_out, phi = out
    reg = torch.empty((m, n), dtype=torch.int32, device="cuda") if want_regions else None
    nr = C.c_int64(0)
    p = params or default_bridge_params()
    _check(load().ww_bridge(_ptr(psi), _ptr(valid), _ptr(K), m, n, C.byref(p), float(nodata),
                            _ptr(K_out), _ptr(phi), _ptr(reg), C.byref(nr), _stream()))
    if want_regions:
        return K_out, phi, int(nr.value), reg
    return K_out, phi, int(nr.value)


class McfParams(C.Structure):
    """Schedule of the min-cost-flow passes (ww_mcf_params)."""
    _fields_ = [("first_hop_window", C.c_int32), ("first_distance_step", C.c_int32),
                ("full_passes", C.c_int32), ("first_deficit_after", C.c_int32),
                ("reverse_below", C.c_int32), ("hop_growth", C.c_int32), ("tile_cols", C.c_int32)]

    def as_tuple(self):
        return (self.first_hop_window, self.first_distance_step, self.full_passes,
                self.first_deficit_after, self.reverse_below, self.hop_growth, self.tile_cols)


def get_mcf_params() -> McfParams:
    p = McfParams()
    load().ww_get_mcf_params(C.byref(p))
    return p


def set_mcf_params(first_hop_window=None, first_distance_step=None, full_passes=None,
                   first_deficit_after=None, reverse_below=None, hop_growth=None,
                   tile_cols=None) -> McfParams:
    """Set the process-wide solve schedule (None keeps a field); returns the
    previous schedule."""
    old = get_mcf_params()
    p = McfParams(*old.as_tuple())
    for k, v in (("first_hop_window", first_hop_window), ("first_distance_step", first_distance_step),
                 ("full_passes", full_passes), ("first_deficit_after", first_deficit_after),
                 ("reverse_below", reverse_below), ("hop_growth", hop_growth),
                 ("tile_cols", tile_cols)):
        if v is not None:
            setattr(p, k, int(v))
    _check(load().ww_set_mcf_params(C.byref(p)))
    return old


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
    L.ww_build_cost_lut_q16.argtypes = [I32, P, P]
    L.ww_edge_costs.argtypes = [P, P, P, I32, I32, P, P, P, P, P, P, P, P]
    L.ww_mcf_solve.argtypes = [P, I32, I32, P, P, P, P, P, P, P, P, P, P]
    L.ww_integrate.argtypes = [P, P, P, P, I32, I32, P, P, P, P]
    L.ww_integrate_noalloc.argtypes = [P, P, P, P, I32, I32, P, P, P, P]
    L.ww_unwrap.argtypes = [P, P, P, I32, I32, I32, P, P, P, P, P]
    for f in ("ww_residues", "ww_build_cost_lut", "ww_build_cost_lut_q16", "ww_edge_costs", "ww_mcf_solve",
              "ww_integrate", "ww_integrate_noalloc", "ww_unwrap"):
        getattr(L, f).restype = C.c_int32
    L.ww_clock.restype = C.c_double
    L.ww_clock.argtypes = []
    L.ww_server_create.argtypes = [I32, I64, P]
    L.ww_server_create.restype = C.c_int32
    L.ww_server_submit.argtypes = [P, P]
    L.ww_server_submit.restype = C.c_int32
    L.ww_server_poll.argtypes = [P, P, I32, I32]
    L.ww_server_poll.restype = C.c_int32
    L.ww_server_in_flight.argtypes = [P]
    L.ww_server_in_flight.restype = C.c_int64
    L.ww_server_destroy.argtypes = [P]
    L.ww_server_destroy.restype = C.c_int32
    L.ww_unwrap_batch.argtypes = [P, I32, I32, P]
    L.ww_unwrap_batch.restype = C.c_int32
    L.ww_default_mcf_params.argtypes = [P]
    L.ww_get_mcf_params.argtypes = [P]
    L.ww_set_mcf_params.argtypes = [P]
    L.ww_set_mcf_params.restype = C.c_int32
    L.ww_default_cc_params.argtypes = [P]
    L.ww_connected_components.argtypes = [P, P, P, P, P, P, P, I32, I32, P, P, P, P]
    L.ww_connected_components.restype = C.c_int32
    L.ww_default_filter_params.argtypes = [P]
    L.ww_goldstein_filter.argtypes = [P, P, I32, I32, P, P, P]
    L.ww_transfer_ambiguity.argtypes = [P, P, P, P, I32, I32, I32, I32, C.c_float, P, P, P]
    L.ww_unwrap_filtered.argtypes = [P, P, P, I32, I32, I32, P, P, P, P, P, P]
    for f in ("ww_goldstein_filter", "ww_transfer_ambiguity", "ww_unwrap_filtered"):
        getattr(L, f).restype = C.c_int32
    L.ww_stream_probe.argtypes = [P, P, I64, I32, I32, P, P]
    L.ww_stream_probe.restype = C.c_int32
    L.ww_default_bridge_params.argtypes = [P]
    L.ww_bridge.argtypes = [P, P, P, I32, I32, P, C.c_float, P, P, P, P, P]
    L.ww_bridge.restype = C.c_int32


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


def build_cost_lut_q16(looks_q16, params: LutParams | None = None) -> np.ndarray:
    """The table at looks_q16 / 2^16 looks (ww_build_cost_lut_q16)."""
    p = params or default_lut_params()
    out = np.zeros((p.n_gamma, p.n_alpha), np.int16)
    _check(load().ww_build_cost_lut_q16(int(looks_q16), C.byref(p), out.ctypes.data_as(C.c_void_p)))
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


def integrate_noalloc(psi, valid, dkx, dky, K, phi, ref=None, nodata=math.nan):
    """ww_integrate_noalloc: the integration into caller-provided device
    tensors K (int32) and phi (float32); the library allocates nothing."""
    torch = _torch()
    m, n = psi.shape
    cp = default_cost_params(nodata=nodata)
    if ref is not None:
        cp.ref_i, cp.ref_j = ref
    nz = lambda t: _ptr(t) if t.numel() else None  # noqa: E731
    _check(load().ww_integrate_noalloc(_ptr(psi), _ptr(valid), nz(dkx), nz(dky), m, n,
                                       C.byref(cp), _ptr(K), _ptr(phi), _stream()))
    del torch
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


# ------------------------------------------------- many interferograms ---

class Job(C.Structure):
    """Mirror of ww_job (include/ww.h)."""
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("looks", C.c_int32), ("host_io", C.c_int32),
                ("psi", C.c_void_p), ("coh", C.c_void_p), ("valid", C.c_void_p),
                ("K", C.c_void_p), ("phi", C.c_void_p), ("tag", C.c_int64),
                ("status", C.c_int32), ("total_cost", C.c_int64), ("t_submit", C.c_double),
                ("t_start", C.c_double), ("t_end", C.c_double), ("footprint_bytes", C.c_int64),
                ("error", C.c_char * 160), ("use_sched", C.c_int32), ("sched", McfParams)]


def stream_probe(src, dst, mode: int = 0, reps: int = 5) -> float:
    """ww_stream_probe: average milliseconds of one hand-written streaming
    sweep over src's bytes (mode 0 copy, 1 read only, 2 non-temporal
    copy)."""
    ms = C.c_float(0.0)
    _check(load().ww_stream_probe(_ptr(src), _ptr(dst), src.numel() * src.element_size(), int(mode),
                                  int(reps), C.byref(ms), _stream()))
    return float(ms.value)


def clock() -> float:
    """Seconds on the monotonic clock the job server stamps jobs with."""
    return float(load().ww_clock())


def _host_ptr(a, dtype):
    if a is None:
        return None, None
    if isinstance(a, np.ndarray):
        if a.dtype != dtype or not a.flags.c_contiguous:
            raise ValueError(f"host arrays must be C-contiguous {np.dtype(dtype).name}")
        return C.c_void_p(a.ctypes.data), a
    # a (pinned) host torch tensor
    if a.is_cuda or not a.is_contiguous():
        raise ValueError("host tensors must be contiguous CPU tensors")
    return C.c_void_p(a.data_ptr()), a


def make_job(psi, coh, valid, looks, K=None, phi=None, tag=0, sched=None):
    """A Job over device tensors (host_io = 0) or host arrays / pinned CPU
    tensors (host_io = 1; the worker copies in and out).  Outputs are
    allocated beside the inputs when not given.  Returns (job, keep) where
    keep holds every array the job points to."""
    on_device = not isinstance(psi, np.ndarray) and psi.is_cuda
    m, n = psi.shape
    j = Job()
    j.m, j.n, j.looks, j.tag = m, n, int(looks), int(tag)
    if sched is not None:
        from .autotune import pad
        j.use_sched = 1
        j.sched = McfParams(*pad(sched))
    if on_device:
        torch = _torch()
        if K is None:
            K = torch.empty((m, n), dtype=torch.int32, device=psi.device)
        if phi is None:
            phi = torch.empty((m, n), dtype=torch.float32, device=psi.device)
        j.host_io = 0
        j.psi, j.coh, j.valid, j.K, j.phi = (_ptr(psi), _ptr(coh), _ptr(valid), _ptr(K), _ptr(phi))
        keep = (psi, coh, valid, K, phi)
    else:
        if K is None:
            K = np.empty((m, n), np.int32)
        if phi is None:
            phi = np.empty((m, n), np.float32)
        ptrs = [_host_ptr(psi, np.float32), _host_ptr(coh, np.float32), _host_ptr(valid, np.uint8),
                _host_ptr(K, np.int32), _host_ptr(phi, np.float32)]
        j.host_io = 1
        j.psi, j.coh, j.valid, j.K, j.phi = [p for p, _ in ptrs]
        keep = tuple(a for _, a in ptrs)
    return j, keep


class Server:
    """Continuous-batching unwrap server (ww_server_*): `slots` workers, each
    with its own stream and workspace, admitting queued jobs as slots and the
    HBM budget free up.  Results come back through poll() in completion
    order as (job, K, phi)."""

    def __init__(self, slots: int = 4, hbm_budget_bytes: int = 0):
        _torch()
        self._h = C.c_void_p()
        _check(load().ww_server_create(int(slots), int(hbm_budget_bytes), C.byref(self._h)))
        self._live = {}

    def submit(self, psi, coh, valid, looks, K=None, phi=None, tag=0, sched=None) -> Job:
        """sched: this job's own solve schedule (None: the process-wide one)."""
        j, keep = make_job(psi, coh, valid, looks, K, phi, tag, sched)
        self._live[C.addressof(j)] = (j, keep)
        rc = load().ww_server_submit(self._h, C.byref(j))
        if rc != OK:
            del self._live[C.addressof(j)]
            _check(rc)
        return j

    def poll(self, wait_ms: int = 0, max_done: int = 256):
        buf = (C.c_void_p * max_done)()
        k = load().ww_server_poll(self._h, buf, max_done, int(wait_ms))
        out = []
        for a in buf[:k]:
            j, keep = self._live.pop(a)
            out.append((j, keep[3], keep[4]))
        return out

    def in_flight(self) -> int:
        return int(load().ww_server_in_flight(self._h))

    def drain(self):
        out = []
        while self.in_flight():
            out += self.poll(wait_ms=-1)
        return out

    def close(self):
        if self._h:
            _check(load().ww_server_destroy(self._h))
            self._h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def unwrap_batch(jobs, group: int = 0, sched=None):
    """jobs: list of (psi, coh, valid, looks) device tensors.  ww_unwrap_batch:
    the jobs' min-cost-flow problems solved together, `group` jobs per solve
    at most (0: up to 256), with the schedule `sched` (a tuple as for
    set_mcf_params; None: the process-wide one).  Returns
    ([(K, phi, total_cost)] in the input order, the Job array)."""
    arr = (Job * len(jobs))()
    keep = []
    for k, (psi, coh, valid, looks) in enumerate(jobs):
        j, kp = make_job(psi, coh, valid, looks, tag=k)
        arr[k] = j
        keep.append(kp)
    sp = None
    if sched is not None:
        from .autotune import pad
        sp = McfParams(*pad(sched))
    rc = load().ww_unwrap_batch(arr, len(jobs), int(group), C.byref(sp) if sp is not None else None)
    if rc != OK:
        bad = [a for a in arr if a.status != OK]
        raise WWError(rc, bad[0].error.decode() if bad else load().ww_last_error().decode())
    return [(kp[3], kp[4], int(a.total_cost)) for a, kp in zip(arr, keep)], arr
