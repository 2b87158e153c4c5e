"""MI355X (gfx950) folded-data SGWB radiometer map-making (arXiv:1803.08285).

Thin ctypes binding over ``libsgwb.so`` (C ABI in ``include/sgwb.h``).  Every
step of the computation runs in the library's HIP kernels; this module only
checks shapes, allocates outputs as torch tensors on the current device and
passes raw device pointers plus the current HIP stream.  There is no CPU
fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsgwb.so")

SGWB_MAPS_ANTIPODAL = 1
SGWB_MAPS_VALU_X = 2
SGWB_BB_TABLE = 4
SGWB_BB_STRIPS = 8
SGWB_NOALLOC_SCRATCH_BYTES = 256 << 20


class SgwbError(RuntimeError):
    pass


class _Detector(ctypes.Structure):
    _fields_ = [("lat_deg", ctypes.c_double), ("lon_deg", ctypes.c_double), ("xarm_az_deg", ctypes.c_double)]


class _Baseline(ctypes.Structure):
    _fields_ = [("a", _Detector), ("b", _Detector)]


class _TGrid(ctypes.Structure):
    _fields_ = [("nt", ctypes.c_int32), ("t0_s", ctypes.c_double), ("stride_s", ctypes.c_double),
                ("seg_dur_s", ctypes.c_double)]


class _FGrid(ctypes.Structure):
    _fields_ = [("f0_hz", ctypes.c_double), ("df_hz", ctypes.c_double)]


class _Job(ctypes.Structure):
    _fields_ = [("C", ctypes.c_void_p), ("w", ctypes.c_void_p), ("ldc", ctypes.c_int64), ("nt", ctypes.c_int32),
                ("nf", ctypes.c_int32), ("fg", _FGrid), ("k0", ctypes.c_int64), ("gamma", ctypes.c_void_p),
                ("tau", ctypes.c_void_p), ("npix", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("X", ctypes.c_void_p), ("Gam", ctypes.c_void_p), ("H", ctypes.c_void_p),
                ("band_lo", ctypes.c_int32), ("band_hi", ctypes.c_int32), ("Xbb", ctypes.c_void_p),
                ("Gbb", ctypes.c_void_p)]


class _Dataset(ctypes.Structure):
    _fields_ = [("C", ctypes.c_void_p), ("w", ctypes.c_void_p), ("ldc", ctypes.c_int64), ("nf", ctypes.c_int32),
                ("fg", _FGrid), ("k0", ctypes.c_int64), ("H", ctypes.c_void_p), ("bl", _Baseline), ("tg", _TGrid)]


class _ServerCfg(ctypes.Structure):
    _fields_ = [("datasets", ctypes.c_void_p), ("ndatasets", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_size_t),
                ("slots", ctypes.c_int32), ("queue_capacity", ctypes.c_int32)]


class _Query(ctypes.Structure):
    _fields_ = [("dataset", ctypes.c_int32), ("nside", ctypes.c_int32), ("k_lo", ctypes.c_int32),
                ("k_hi", ctypes.c_int32)]


class _Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("npix", ctypes.c_int32), ("Xbb", ctypes.c_void_p),
                ("Gbb", ctypes.c_void_p), ("t_submit_s", ctypes.c_double), ("t_start_s", ctypes.c_double),
                ("t_done_s", ctypes.c_double)]


_lib = None

_VP = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64

_SIGNATURES = {
    "sgwb_build_geometry": ([ctypes.POINTER(_Baseline), _I32, ctypes.POINTER(_TGrid), _VP, _VP, _VP], ctypes.c_int),
    "sgwb_build_geometry_f64": ([ctypes.POINTER(_Baseline), _I32, ctypes.POINTER(_TGrid), _VP, _VP, _VP],
                                ctypes.c_int),
    "sgwb_make_maps_workspace_size": ([_I32, _I32, _I32, ctypes.c_uint32], ctypes.c_size_t),
    "sgwb_make_maps": ([_VP, _VP, _I64, _I32, _I32, ctypes.POINTER(_FGrid), _I64, _VP, _VP, _I32,
                        ctypes.c_uint32, _VP, _VP, _VP, ctypes.c_size_t, _VP], ctypes.c_int),
    "sgwb_make_maps_f64": ([_VP, _VP, _I64, _I32, _I32, ctypes.POINTER(_FGrid), _I64, _VP, _VP, _I32,
                            ctypes.c_uint32, _VP, _VP, _VP], ctypes.c_int),
    "sgwb_network_sum": ([ctypes.POINTER(ctypes.c_void_p), _I32, _I64, _VP, _VP], ctypes.c_int),
    "sgwb_contract_pixels": ([_VP, _I32, _I32, _VP, _I32, _VP, _VP], ctypes.c_int),
    "sgwb_fold": ([_VP, _VP, _VP, _I64, _I32, _I32, _I32, ctypes.c_double, _VP, _VP, _VP, _VP, _VP], ctypes.c_int),
    "sgwb_fisher_overlap_workspace_size": ([_I32, _I32, _I32, ctypes.c_uint32], ctypes.c_size_t),
    "sgwb_fisher_overlap": ([_VP, _VP, _VP, _I64, _I32, _I32, ctypes.POINTER(_FGrid), _I64, _VP, _VP, _I32,
                             ctypes.c_uint32, _VP, _VP, ctypes.c_size_t, _VP], ctypes.c_int),
    "sgwb_fisher_full_workspace_size": ([ctypes.POINTER(_FGrid), _I64, _I32, _I32, _I32], ctypes.c_size_t),
    "sgwb_fisher_full": ([_VP, _VP, _I32, _VP, _I32, ctypes.POINTER(_FGrid), _I64, _I32, _I32, _VP, _VP, _I32, _I32,
                          ctypes.c_uint32, _VP, _VP, ctypes.c_size_t, _VP], ctypes.c_int),
    "sgwb_fisher_full_general_workspace_size": ([ctypes.POINTER(_FGrid), _I64, _I32, _I32, _I32, _I32,
                                                 ctypes.c_uint32], ctypes.c_size_t),
    "sgwb_fisher_full_general": ([_VP, _I64, _VP, _I32, ctypes.POINTER(_FGrid), _I64, _I32, _I32, _VP, _VP, _I32,
                                  _I32, ctypes.c_uint32, _VP, _VP, ctypes.c_size_t, _VP], ctypes.c_int),
    "sgwb_clean_map_workspace_size": ([_I32], ctypes.c_size_t),
    "sgwb_clean_map_cg": ([_VP, _VP, _I32, _I32, _VP, _VP, ctypes.c_size_t, _VP], ctypes.c_int),
    "sgwb_make_maps_band_workspace_size": ([_I32, _I32, _I32, ctypes.c_uint32], ctypes.c_size_t),
    "sgwb_make_maps_band": ([_VP, _VP, _I64, _I32, _I32, ctypes.POINTER(_FGrid), _I64, _VP, _VP, _I32,
                             ctypes.c_uint32, _VP, _I32, _I32, _VP, _VP, _VP, _VP, _VP, ctypes.c_size_t, _VP],
                            ctypes.c_int),
    "sgwb_baseline_delay_bound": ([ctypes.POINTER(_Baseline)], ctypes.c_double),
    "sgwb_broadband_maps_workspace_size": ([_I32, _I32, _I32, ctypes.c_uint32, ctypes.POINTER(_FGrid), _I32, _I32,
                                            ctypes.c_double], ctypes.c_size_t),
    "sgwb_broadband_maps": ([_VP, _VP, _I64, _I32, _I32, ctypes.POINTER(_FGrid), _I64, _VP, _VP, _I32,
                             ctypes.c_uint32, ctypes.c_double, _VP, _I32, _I32, _VP, _VP, _VP, ctypes.c_size_t, _VP],
                            ctypes.c_int),
    "sgwb_make_maps_band_noalloc": ([_VP, _VP, _I64, _I32, _I32, ctypes.POINTER(_FGrid), _I64, _VP, _VP, _I32,
                                     ctypes.c_uint32, _VP, _I32, _I32, _VP, _VP, _VP, _VP, _VP], ctypes.c_int),
    "sgwb_reduce_band_workspace_size": ([_I32, _I32, _I32], ctypes.c_size_t),
    "sgwb_reduce_band": ([_VP, _VP, _VP, _I32, _I32, _I32, _I32, _VP, _VP, _VP, ctypes.c_size_t, _VP], ctypes.c_int),
    "sgwb_reduce_band_f64": ([_VP, _VP, _VP, _I32, _I32, _I32, _I32, _VP, _VP, _VP], ctypes.c_int),
    "sgwb_healpix_centres": ([_I32, _VP, _VP, _VP], ctypes.c_int),
    "sgwb_server_create": ([ctypes.POINTER(_ServerCfg), ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "sgwb_server_submit": ([_VP, ctypes.POINTER(_Query), ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "sgwb_server_poll": ([_VP, ctypes.c_uint64, ctypes.POINTER(_Result)], ctypes.c_int),
    "sgwb_server_fetch": ([_VP, ctypes.c_uint64, _VP, _VP, _VP], ctypes.c_int),
    "sgwb_server_release": ([_VP, ctypes.c_uint64], ctypes.c_int),
    "sgwb_server_stats": ([_VP, ctypes.c_char_p, ctypes.c_size_t], ctypes.c_int),
    "sgwb_server_destroy": ([_VP], None),
    "sgwb_plan_create": ([ctypes.POINTER(_Job), _I32, ctypes.c_uint32, ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "sgwb_plan_launch": ([_VP, _VP], ctypes.c_int),
    "sgwb_plan_destroy": ([_VP], None),
    "sgwb_plan_describe": ([_VP, ctypes.c_char_p, ctypes.c_size_t], ctypes.c_int),
    "sgwb_last_x_form": ([ctypes.POINTER(_I32)], ctypes.c_int),
    "sgwb_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "sgwb_last_error": ([], ctypes.c_char_p),
    "sgwb_device_supported": ([], ctypes.c_int),
}


def exported_symbols():
    """Names of the C entry points this binding expects the library to export."""
    return sorted(_SIGNATURES)


def lib():
    """Load libsgwb.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SgwbError(f"{LIB_PATH} is missing: build it with paper_1803_08285_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        L = lib()
        raise SgwbError(f"{what}: {L.sgwb_status_string(rc).decode()} ({rc}): {L.sgwb_last_error().decode()}")


def _stream(device=None) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _require(t: torch.Tensor, name: str, dtype, shape=None, cols_contig=True):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise SgwbError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise SgwbError(f"{name} must be {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise SgwbError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if cols_contig and t.dim() == 2 and t.stride(1) != 1:
        raise SgwbError(f"{name} must have unit stride along its last axis")


def _require_contig(t: torch.Tensor, name: str):
    if not t.is_contiguous():
        raise SgwbError(f"{name} must be contiguous")


# ---------------------------------------------------------------------------
# Geometry descriptions
# ---------------------------------------------------------------------------
@dataclass(frozen=True)
class TGrid:
    nt: int
    t0: float
    stride: float
    dur: float


@dataclass(frozen=True)
class FGrid:
    """Absolute bin grid f_k = f0 + k df."""
    f0: float
    df: float


def _baseline(sites) -> _Baseline:
    s = [float(x) for x in sites]
    if len(s) != 6:
        raise SgwbError("baseline needs (latA, lonA, azA, latB, lonB, azB)")
    return _Baseline(_Detector(*s[:3]), _Detector(*s[3:]))


def npix_of(nside: int) -> int:
    return 12 * nside * nside


# ---------------------------------------------------------------------------
# Calls
# ---------------------------------------------------------------------------
def build_geometry(sites, nside: int, tgrid: TGrid, dtype=torch.float32, device=None, out=None):
    """ORF seed matrices (gamma, tau) of shape [nt][12 nside^2]; gamma float32
    (or float64 with dtype=torch.float64), tau float64 seconds."""
    device = torch.device("cuda") if device is None else torch.device(device)
    npix = npix_of(nside)
    if out is None:
        gamma = torch.empty((tgrid.nt, npix), dtype=dtype, device=device)
        tau = torch.empty((tgrid.nt, npix), dtype=torch.float64, device=device)
    else:
        gamma, tau = out
    _require(gamma, "gamma", dtype, (tgrid.nt, npix))
    _require(tau, "tau", torch.float64, (tgrid.nt, npix))
    _require_contig(gamma, "gamma")
    _require_contig(tau, "tau")
    bl = _baseline(sites)
    tg = _TGrid(int(tgrid.nt), float(tgrid.t0), float(tgrid.stride), float(tgrid.dur))
    fn = lib().sgwb_build_geometry if dtype == torch.float32 else lib().sgwb_build_geometry_f64
    with torch.cuda.device(gamma.device):
        _check(fn(ctypes.byref(bl), int(nside), ctypes.byref(tg), _ptr(gamma), _ptr(tau), _stream()),
               "build_geometry")
    return gamma, tau


X_FORMS = {0: "none", 1: "valu", 2: "mfma4", 3: "mfma5", 4: "mfma5_split", 5: "table"}


def last_x_form() -> str:
    """Form of the dirty map that the last make_maps / make_maps_band /
    fisher_overlap call of this thread took: "none", "valu", "mfma4", "mfma5" or
    "mfma5_split", or "table" after a broadband_maps call that took the delay-table
    route (synchronises that call's stream for the matrix-core forms;
    raises if its seeds failed the antipodal check)."""
    f = _I32(0)
    _check(lib().sgwb_last_x_form(ctypes.byref(f)), "last_x_form")
    return X_FORMS[int(f.value)]


def workspace_bytes(nt: int, nf: int, npix: int, antipodal: bool = True) -> int:
    return int(lib().sgwb_make_maps_workspace_size(nt, nf, npix, SGWB_MAPS_ANTIPODAL if antipodal else 0))


def make_workspace(nt: int, nf: int, npix: int, antipodal: bool = True, device=None) -> torch.Tensor:
    n = workspace_bytes(nt, nf, npix, antipodal)
    return torch.empty(max(n, 256), dtype=torch.uint8, device=device or "cuda")


def make_maps(C: torch.Tensor, w: torch.Tensor, fgrid: FGrid, k0: int, gamma: torch.Tensor,
              tau: torch.Tensor, antipodal: bool = True, want_x: bool = True, want_gamma: bool = True,
              out=None, workspace: torch.Tensor | None = None, x_kernel: str = "auto"):
    """Narrowband dirty map X and Fisher diagonal Gam, both [nf][npix].

    C: complex64 [nt][>= nf] (columns = bins k0 ..), or complex128 for the
    float64 path; w: float32/float64 [nt][same columns]; gamma [nt][npix] of the
    working precision; tau float64 [nt][npix].  Column slices of a wider array
    are accepted (rows may be strided, columns must be unit-stride).
    x_kernel: "auto" (matrix cores where they apply) or "valu" (vector-unit recurrence).
    """
    f64 = C.dtype == torch.complex128
    rdt = torch.float64 if f64 else torch.float32
    cdt = torch.complex128 if f64 else torch.complex64
    if C.dim() != 2 or w.dim() != 2:
        raise SgwbError("C and w must be 2-D")
    nt, nf = w.shape
    npix = gamma.shape[1]
    _require(C, "C", cdt, (nt, nf))
    _require(w, "w", rdt, (nt, nf))
    if C.stride(0) != w.stride(0):
        raise SgwbError("C and w must share their row stride")
    _require(gamma, "gamma", rdt, (nt, npix))
    _require(tau, "tau", torch.float64, (nt, npix))
    _require_contig(gamma, "gamma")
    _require_contig(tau, "tau")
    dev = C.device
    X = G = None
    if out is not None:
        X, G = out
    if want_x and X is None:
        X = torch.empty((nf, npix), dtype=rdt, device=dev)
    if want_gamma and G is None:
        G = torch.empty((nf, npix), dtype=rdt, device=dev)
    for name, t in (("X", X), ("Gam", G)):
        if t is not None:
            _require(t, name, rdt, (nf, npix))
            _require_contig(t, name)
    if x_kernel not in ("auto", "valu"):
        raise SgwbError("x_kernel must be 'auto' or 'valu'")
    flags = (SGWB_MAPS_ANTIPODAL if antipodal else 0) | (SGWB_MAPS_VALU_X if x_kernel == "valu" else 0)
    fg = _FGrid(float(fgrid.f0), float(fgrid.df))
    Cr = torch.view_as_real(C)
    with torch.cuda.device(dev):
        if f64:
            rc = lib().sgwb_make_maps_f64(_ptr(Cr), _ptr(w), int(w.stride(0)), nt, nf, ctypes.byref(fg), int(k0),
                                          _ptr(gamma), _ptr(tau), npix, flags, _ptr(X), _ptr(G), _stream())
        else:
            need = workspace_bytes(nt, nf, npix, antipodal)
            if workspace is None:
                workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
            ws = workspace
            wsz = workspace.numel() * workspace.element_size()
            rc = lib().sgwb_make_maps(_ptr(Cr), _ptr(w), int(w.stride(0)), nt, nf, ctypes.byref(fg), int(k0),
                                      _ptr(gamma), _ptr(tau), npix, flags, _ptr(X), _ptr(G), _ptr(ws), wsz,
                                      _stream())
    _check(rc, "make_maps")
    return X, G


def band_maps_workspace_bytes(nt: int, nf: int, npix: int, antipodal: bool = True) -> int:
    return int(lib().sgwb_make_maps_band_workspace_size(nt, nf, npix, SGWB_MAPS_ANTIPODAL if antipodal else 0))


def make_maps_band(C: torch.Tensor, w: torch.Tensor, fgrid: FGrid, k0: int, gamma: torch.Tensor,
                   tau: torch.Tensor, H: torch.Tensor | None, k_lo: int, k_hi: int, antipodal: bool = True,
                   want_x: bool = True, want_gamma: bool = True, out=None, workspace: torch.Tensor | None = None,
                   x_kernel: str = "auto", noalloc: bool = False, narrowband: bool = True):
    """make_maps and reduce_band over columns [k_lo, k_hi) in one call (float32):
    returns X, Gam [nf][npix] and Xbb, Gbb [npix] (None where not asked for).
    narrowband=False computes the broadband maps alone (X and Gam None: no
    narrowband row is written and no beam GEMM runs; the broadband bits are
    those of the full call).  noalloc=True calls sgwb_make_maps_band_noalloc
    (the library's fixed scratch array instead of a workspace; pass
    preallocated outputs in ``out`` for a call that allocates nothing at all)."""
    if C.dim() != 2 or w.dim() != 2:
        raise SgwbError("C and w must be 2-D")
    nt, nf = w.shape
    npix = gamma.shape[1]
    _require(C, "C", torch.complex64, (nt, nf))
    _require(w, "w", torch.float32, (nt, nf))
    if C.stride(0) != w.stride(0):
        raise SgwbError("C and w must share their row stride")
    _require(gamma, "gamma", torch.float32, (nt, npix))
    _require(tau, "tau", torch.float64, (nt, npix))
    _require_contig(gamma, "gamma")
    _require_contig(tau, "tau")
    if want_gamma:
        if H is None:
            raise SgwbError("H is needed for Gbb")
        _require(H, "H", torch.float32, (nf,))
        _require_contig(H, "H")
    dev = C.device
    if out is None:
        X = torch.empty((nf, npix), dtype=torch.float32, device=dev) if want_x and narrowband else None
        G = torch.empty((nf, npix), dtype=torch.float32, device=dev) if want_gamma and narrowband else None
        Xbb = torch.empty(npix, dtype=torch.float32, device=dev) if want_x else None
        Gbb = torch.empty(npix, dtype=torch.float32, device=dev) if want_gamma else None
    else:
        X, G, Xbb, Gbb = out
    for name, t, shape in (("X", X, (nf, npix)), ("Gam", G, (nf, npix)), ("Xbb", Xbb, (npix,)),
                           ("Gbb", Gbb, (npix,))):
        if t is not None:
            _require(t, name, torch.float32, shape)
            _require_contig(t, name)
    if x_kernel not in ("auto", "valu"):
        raise SgwbError("x_kernel must be 'auto' or 'valu'")
    flags = (SGWB_MAPS_ANTIPODAL if antipodal else 0) | (SGWB_MAPS_VALU_X if x_kernel == "valu" else 0)
    fg = _FGrid(float(fgrid.f0), float(fgrid.df))
    with torch.cuda.device(dev):
        if noalloc:
            if workspace is not None:
                raise SgwbError("make_maps_band: noalloc takes no workspace")
            rc = lib().sgwb_make_maps_band_noalloc(_ptr(torch.view_as_real(C)), _ptr(w), int(w.stride(0)), nt, nf,
                                                   ctypes.byref(fg), int(k0), _ptr(gamma), _ptr(tau), npix, flags,
                                                   _ptr(H) if H is not None else None, int(k_lo), int(k_hi), _ptr(X),
                                                   _ptr(G), _ptr(Xbb), _ptr(Gbb), _stream())
        else:
            if workspace is None:
                workspace = torch.empty(max(band_maps_workspace_bytes(nt, nf, npix, antipodal), 256),
                                        dtype=torch.uint8, device=dev)
            wsz = workspace.numel() * workspace.element_size()
            rc = lib().sgwb_make_maps_band(_ptr(torch.view_as_real(C)), _ptr(w), int(w.stride(0)), nt, nf,
                                           ctypes.byref(fg), int(k0), _ptr(gamma), _ptr(tau), npix, flags,
                                           _ptr(H) if H is not None else None, int(k_lo), int(k_hi), _ptr(X), _ptr(G),
                                           _ptr(Xbb), _ptr(Gbb), _ptr(workspace), wsz, _stream())
    _check(rc, "make_maps_band_noalloc" if noalloc else "make_maps_band")
    return X, G, Xbb, Gbb


def baseline_delay_bound(sites) -> float:
    """|x_a - x_b| / c (s) of a baseline's two sites: the bound its seeds' delays meet."""
    bl = _baseline(sites)
    return float(lib().sgwb_baseline_delay_bound(ctypes.byref(bl)))


_BB_ROUTES = {"auto": 0, "table": SGWB_BB_TABLE, "strips": SGWB_BB_STRIPS}


def broadband_maps_workspace_bytes(nt: int, nf: int, npix: int, fgrid: FGrid, k_lo: int, k_hi: int,
                                   tau_bound: float = 0.0, antipodal: bool = True, route: str = "auto") -> int:
    if route not in _BB_ROUTES:
        raise SgwbError("route must be 'auto', 'table' or 'strips'")
    fg = _FGrid(float(fgrid.f0), float(fgrid.df))
    flags = (SGWB_MAPS_ANTIPODAL if antipodal else 0) | _BB_ROUTES[route]
    return int(lib().sgwb_broadband_maps_workspace_size(nt, nf, npix, flags, ctypes.byref(fg), int(k_lo), int(k_hi),
                                                        float(tau_bound)))


def broadband_maps(C: torch.Tensor, w: torch.Tensor, fgrid: FGrid, k0: int, gamma: torch.Tensor,
                   tau: torch.Tensor, H: torch.Tensor | None, k_lo: int, k_hi: int, tau_bound: float = 0.0,
                   antipodal: bool = True, want_x: bool = True, want_gamma: bool = True, out=None,
                   workspace: torch.Tensor | None = None, route: str = "auto"):
    """Broadband maps Xbb, Gbb [npix] over columns [k_lo, k_hi), no narrowband
    map (float32): the library takes the strips route (the matrix-core dirty
    map's strip sums) or sums the band first through per-segment delay tables,
    as ``route`` forces or its cost estimate picks.  tau_bound: a bound on the
    seeds' |tau| (s), e.g. baseline_delay_bound(sites); 0 takes 2R/c."""
    if C.dim() != 2 or w.dim() != 2:
        raise SgwbError("C and w must be 2-D")
    nt, nf = w.shape
    npix = gamma.shape[1]
    _require(C, "C", torch.complex64, (nt, nf))
    _require(w, "w", torch.float32, (nt, nf))
    if C.stride(0) != w.stride(0):
        raise SgwbError("C and w must share their row stride")
    _require(gamma, "gamma", torch.float32, (nt, npix))
    _require(tau, "tau", torch.float64, (nt, npix))
    _require_contig(gamma, "gamma")
    _require_contig(tau, "tau")
    if want_gamma:
        if H is None:
            raise SgwbError("H is needed for Gbb")
        _require(H, "H", torch.float32, (nf,))
        _require_contig(H, "H")
    if route not in _BB_ROUTES:
        raise SgwbError("route must be 'auto', 'table' or 'strips'")
    dev = C.device
    if out is None:
        Xbb = torch.empty(npix, dtype=torch.float32, device=dev) if want_x else None
        Gbb = torch.empty(npix, dtype=torch.float32, device=dev) if want_gamma else None
    else:
        Xbb, Gbb = out
    for name, t in (("Xbb", Xbb), ("Gbb", Gbb)):
        if t is not None:
            _require(t, name, torch.float32, (npix,))
            _require_contig(t, name)
    flags = (SGWB_MAPS_ANTIPODAL if antipodal else 0) | _BB_ROUTES[route]
    fg = _FGrid(float(fgrid.f0), float(fgrid.df))
    with torch.cuda.device(dev):
        if workspace is None:
            need = broadband_maps_workspace_bytes(nt, nf, npix, fgrid, k_lo, k_hi, tau_bound, antipodal, route)
            workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
        wsz = workspace.numel() * workspace.element_size()
        rc = lib().sgwb_broadband_maps(_ptr(torch.view_as_real(C)), _ptr(w), int(w.stride(0)), nt, nf,
                                       ctypes.byref(fg), int(k0), _ptr(gamma), _ptr(tau), npix, flags,
                                       float(tau_bound), _ptr(H) if H is not None else None, int(k_lo), int(k_hi),
                                       _ptr(Xbb), _ptr(Gbb), _ptr(workspace), wsz, _stream())
    _check(rc, "broadband_maps")
    return Xbb, Gbb


def network_sum(maps, out=None):
    """Element-wise sum of float32 maps of several baselines (same shape), in order."""
    maps = list(maps)
    if not maps:
        raise SgwbError("network_sum: no maps")
    shape, dev = tuple(maps[0].shape), maps[0].device
    for i, m in enumerate(maps):
        _require(m, f"maps[{i}]", torch.float32, shape)
        _require_contig(m, f"maps[{i}]")
    out = torch.empty(shape, dtype=torch.float32, device=dev) if out is None else out
    _require(out, "out", torch.float32, shape)
    _require_contig(out, "out")
    arr = (ctypes.c_void_p * len(maps))(*[m.data_ptr() for m in maps])
    with torch.cuda.device(dev):
        rc = lib().sgwb_network_sum(arr, len(maps), int(out.numel()), _ptr(out), _stream())
    _check(rc, "network_sum")
    return out


def contract_pixels(M: torch.Tensor, pix: torch.Tensor | None = None, out=None):
    """Per-row sum of M [nf][npix] (or a broadband map [npix]) over the pixel set
    pix (int tensor of RING indices on the device; None = all pixels: isotropic)."""
    M2 = M if M.dim() == 2 else M.reshape(1, -1)
    nf, npix = M2.shape
    _require(M2, "M", torch.float32, (nf, npix))
    _require_contig(M2, "M")
    p = None
    nsel = 0
    if pix is not None:
        p = pix.to(device=M.device, dtype=torch.int32).contiguous()
        nsel = int(p.numel())
        if nsel and (int(p.min()) < 0 or int(p.max()) >= npix):
            raise SgwbError("contract_pixels: pixel index out of range")
    out = torch.empty(nf, dtype=torch.float32, device=M.device) if out is None else out
    with torch.cuda.device(M.device):
        rc = lib().sgwb_contract_pixels(_ptr(M2), nf, npix, _ptr(p) if p is not None else None, nsel, _ptr(out),
                                        _stream())
    _check(rc, "contract_pixels")
    return out


def fold(C: torch.Tensor, sinv: torch.Tensor, present: torch.Tensor, W: float, out=None):
    """Fold ndays sidereal days into one (Sec. II.B): C complex64 [ndays][nt][>= nf],
    sinv float32 [ndays][nt][same columns], present bool/uint8 [ndays][nt].
    Returns v, u, w float32 [nt][nf] and x complex64 [nt][nf]."""
    if C.dim() != 3 or sinv.dim() != 3:
        raise SgwbError("C and sinv must be 3-D [ndays][nt][bins]")
    ndays, nt, nf = sinv.shape
    if C.dtype != torch.complex64 or tuple(C.shape) != (ndays, nt, nf):
        raise SgwbError("C must be complex64 with the shape of sinv")
    if sinv.dtype != torch.float32:
        raise SgwbError("sinv must be float32")
    for name, t in (("C", C), ("sinv", sinv)):
        if t.stride(2) != 1 or t.stride(0) != nt * t.stride(1):
            raise SgwbError(f"{name}: rows must be contiguous segments with unit-stride bins")
    if C.stride(1) != sinv.stride(1):
        raise SgwbError("C and sinv must share their row stride")
    if tuple(present.shape) != (ndays, nt):
        raise SgwbError("present must be [ndays][nt]")
    dev = sinv.device
    if C.device != dev or present.device != dev:
        raise SgwbError("all tensors must be on the same device")
    pres = present.to(torch.uint8).contiguous()
    if out is None:
        v = torch.empty((nt, nf), dtype=torch.float32, device=dev)
        u = torch.empty_like(v)
        w = torch.empty_like(v)
        x = torch.empty((nt, nf), dtype=torch.complex64, device=dev)
    else:
        v, u, w, x = out
    for name, t, dt in (("v", v, torch.float32), ("u", u, torch.float32), ("w", w, torch.float32),
                        ("x", x, torch.complex64)):
        _require(t, name, dt, (nt, nf))
        _require_contig(t, name)
    with torch.cuda.device(dev):
        rc = lib().sgwb_fold(_ptr(torch.view_as_real(C)), _ptr(sinv), _ptr(pres), int(sinv.stride(1)), ndays, nt, nf,
                             float(W), _ptr(v), _ptr(u), _ptr(w), _ptr(torch.view_as_real(x)), _stream())
    _check(rc, "fold")
    return v, u, w, x


def fisher_overlap_workspace_bytes(nt: int, nf: int, npix: int, antipodal: bool = True) -> int:
    return int(lib().sgwb_fisher_overlap_workspace_size(nt, nf, npix, SGWB_MAPS_ANTIPODAL if antipodal else 0))


def fisher_overlap(v: torch.Tensor, u: torch.Tensor, wn: torch.Tensor, fgrid: FGrid, k0: int,
                   gamma: torch.Tensor, tau: torch.Tensor, antipodal: bool = True, out=None,
                   workspace: torch.Tensor | None = None, x_kernel: str = "auto"):
    """Overlap-corrected Fisher diagonal Gam [nf][npix] (Sec. II.B, Eq. fwGamma with
    p = p'): v, u, wn float32 [nt][>= nf] folded series sharing one row stride."""
    nt, nf = v.shape
    npix = gamma.shape[1]
    for name, t in (("v", v), ("u", u), ("w", wn)):
        _require(t, name, torch.float32, (nt, nf))
        if t.stride(0) != v.stride(0):
            raise SgwbError("v, u and w must share their row stride")
    _require(gamma, "gamma", torch.float32, (nt, npix))
    _require(tau, "tau", torch.float64, (nt, npix))
    _require_contig(gamma, "gamma")
    _require_contig(tau, "tau")
    if x_kernel not in ("auto", "valu"):
        raise SgwbError("x_kernel must be 'auto' or 'valu'")
    dev = v.device
    G = out if out is not None else torch.empty((nf, npix), dtype=torch.float32, device=dev)
    _require(G, "Gam", torch.float32, (nf, npix))
    _require_contig(G, "Gam")
    flags = (SGWB_MAPS_ANTIPODAL if antipodal else 0) | (SGWB_MAPS_VALU_X if x_kernel == "valu" else 0)
    fg = _FGrid(float(fgrid.f0), float(fgrid.df))
    with torch.cuda.device(dev):
        if workspace is None:
            need = fisher_overlap_workspace_bytes(nt, nf, npix, antipodal)
            workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
        wsz = workspace.numel() * workspace.element_size()
        rc = lib().sgwb_fisher_overlap(_ptr(v), _ptr(u), _ptr(wn), int(v.stride(0)), nt, nf, ctypes.byref(fg),
                                       int(k0), _ptr(gamma), _ptr(tau), npix, flags, _ptr(G), _ptr(workspace),
                                       wsz, _stream())
    _check(rc, "fisher_overlap")
    return G


def fisher_full_workspace_bytes(fgrid: FGrid, k0: int, khi: int, nt: int, npix: int) -> int:
    fg = _FGrid(float(fgrid.f0), float(fgrid.df))
    return int(lib().sgwb_fisher_full_workspace_size(ctypes.byref(fg), int(k0), int(khi), int(nt), int(npix)))


def fisher_full(a: torch.Tensor, b: torch.Tensor, H: torch.Tensor, fgrid: FGrid, k0: int, klo: int, khi: int,
                gamma: torch.Tensor, tau: torch.Tensor, out=None, workspace: torch.Tensor | None = None,
                antipodal: bool = False):
    """Full Fisher matrix G [npix][npix] of the bins [klo, khi) (Eq. eq_fisher,
    broadband H weighting of Sec. V) for weights w(t,c) = sum_r a[r][t] b[r][c]:
    a float32 [nt] or [rank][nt], b float32 [nf] or [rank][nf], H float32 [nf]
    (column c = bin k0 + c).  antipodal=True: seeds from build_geometry (all
    12 nside^2 pixels), half the work."""
    nt, npix = gamma.shape
    a2 = a.reshape(1, -1) if a.dim() == 1 else a
    b2 = b.reshape(1, -1) if b.dim() == 1 else b
    rank, nf = b2.shape
    _require(a2, "a", torch.float32, (rank, nt))
    _require(b2, "b", torch.float32, (rank, nf))
    _require(H, "H", torch.float32, (nf,))
    _require(gamma, "gamma", torch.float32, (nt, npix))
    _require(tau, "tau", torch.float64, (nt, npix))
    for name, t in (("a", a2), ("b", b2), ("H", H), ("gamma", gamma), ("tau", tau)):
        _require_contig(t, name)
    dev = gamma.device
    G = out if out is not None else torch.empty((npix, npix), dtype=torch.float32, device=dev)
    _require(G, "G", torch.float32, (npix, npix))
    _require_contig(G, "G")
    fg = _FGrid(float(fgrid.f0), float(fgrid.df))
    with torch.cuda.device(dev):
        if workspace is None:
            need = fisher_full_workspace_bytes(fgrid, k0, khi, nt, npix)
            workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
        wsz = workspace.numel() * workspace.element_size()
        rc = lib().sgwb_fisher_full(_ptr(a2), _ptr(b2), rank, _ptr(H), nf, ctypes.byref(fg), int(k0), int(klo),
                                    int(khi), _ptr(gamma), _ptr(tau), nt, npix,
                                    SGWB_MAPS_ANTIPODAL if antipodal else 0, _ptr(G), _ptr(workspace), wsz,
                                    _stream())
    _check(rc, "fisher_full")
    return G


def fisher_full_general_workspace_bytes(fgrid: FGrid, k0: int, klo: int, khi: int, nt: int, npix: int,
                                       antipodal: bool = False) -> int:
    fg = _FGrid(float(fgrid.f0), float(fgrid.df))
    return int(lib().sgwb_fisher_full_general_workspace_size(ctypes.byref(fg), int(k0), int(klo), int(khi), int(nt),
                                                             int(npix), SGWB_MAPS_ANTIPODAL if antipodal else 0))


def fisher_full_general(w: torch.Tensor, H: torch.Tensor, fgrid: FGrid, k0: int, klo: int, khi: int,
                        gamma: torch.Tensor, tau: torch.Tensor, out=None, workspace: torch.Tensor | None = None,
                        antipodal: bool = False):
    """Full Fisher matrix G [npix][npix] of the bins [klo, khi) (Eq. eq_fisher,
    broadband H weighting of Sec. V) for general weights: w float32 [nt][nf]
    (rows may be padded: w.stride(0) >= nf), H float32 [nf] (column c = bin
    k0 + c).  antipodal=True: seeds from build_geometry, half the work."""
    nt, npix = gamma.shape
    if w.dim() != 2 or w.shape[0] != nt:
        raise SgwbError(f"w must be [nt={nt}][nf], got {tuple(w.shape)}")
    nf = w.shape[1]
    _require(w, "w", torch.float32, (nt, nf))
    if w.stride(1) != 1 or w.stride(0) < nf:
        raise SgwbError("w must have unit column stride and row stride >= nf")
    _require(H, "H", torch.float32, (nf,))
    _require(gamma, "gamma", torch.float32, (nt, npix))
    _require(tau, "tau", torch.float64, (nt, npix))
    for name, t in (("H", H), ("gamma", gamma), ("tau", tau)):
        _require_contig(t, name)
    dev = gamma.device
    G = out if out is not None else torch.empty((npix, npix), dtype=torch.float32, device=dev)
    _require(G, "G", torch.float32, (npix, npix))
    _require_contig(G, "G")
    fg = _FGrid(float(fgrid.f0), float(fgrid.df))
    with torch.cuda.device(dev):
        if workspace is None:
            need = fisher_full_general_workspace_bytes(fgrid, k0, klo, khi, nt, npix, antipodal)
            workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
        wsz = workspace.numel() * workspace.element_size()
        rc = lib().sgwb_fisher_full_general(_ptr(w), int(w.stride(0)), _ptr(H), nf, ctypes.byref(fg), int(k0),
                                            int(klo), int(khi), _ptr(gamma), _ptr(tau), nt, npix,
                                            SGWB_MAPS_ANTIPODAL if antipodal else 0, _ptr(G), _ptr(workspace), wsz,
                                            _stream())
    _check(rc, "fisher_full_general")
    return G


def clean_map_cg(G: torch.Tensor, X: torch.Tensor, niter: int, out=None, workspace: torch.Tensor | None = None):
    """Clean map (Eq. eq_ML_linear and its footnote): niter conjugate-gradient
    steps on G P = X from P = 0; G float32 [n][n], X float32 [n]."""
    n = X.shape[0]
    _require(G, "G", torch.float32, (n, n))
    _require(X, "X", torch.float32, (n,))
    _require_contig(G, "G")
    _require_contig(X, "X")
    dev = X.device
    P = out if out is not None else torch.empty(n, dtype=torch.float32, device=dev)
    _require(P, "P", torch.float32, (n,))
    _require_contig(P, "P")
    with torch.cuda.device(dev):
        if workspace is None:
            workspace = torch.empty(max(int(lib().sgwb_clean_map_workspace_size(n)), 256), dtype=torch.uint8,
                                    device=dev)
        wsz = workspace.numel() * workspace.element_size()
        rc = lib().sgwb_clean_map_cg(_ptr(G), _ptr(X), n, int(niter), _ptr(P), _ptr(workspace), wsz, _stream())
    _check(rc, "clean_map_cg")
    return P


def band_workspace_bytes(npix: int, k_lo: int, k_hi: int) -> int:
    return int(lib().sgwb_reduce_band_workspace_size(npix, k_lo, k_hi))


def reduce_band(X: torch.Tensor | None, G: torch.Tensor | None, H: torch.Tensor | None, k_lo: int, k_hi: int,
                out=None, workspace: torch.Tensor | None | bool = True):
    """Broadband Xbb = sum_k X[k], Gbb = sum_k H[k] G[k] over rows [k_lo, k_hi).

    workspace: a uint8 device tensor, True to allocate one (parallel slab
    reduction), or None for the single-pass kernel.
    """
    ref = X if X is not None else G
    if ref is None:
        raise SgwbError("reduce_band: X or G needed")
    nf, npix = ref.shape
    rdt = ref.dtype
    for name, t in (("X", X), ("G", G)):
        if t is not None:
            _require(t, name, rdt, (nf, npix))
            _require_contig(t, name)
    if G is not None:
        _require(H, "H", rdt, (nf,))
        _require_contig(H, "H")
    Xbb = Gbb = None
    if out is not None:
        Xbb, Gbb = out
    if X is not None and Xbb is None:
        Xbb = torch.empty(npix, dtype=rdt, device=ref.device)
    if G is not None and Gbb is None:
        Gbb = torch.empty(npix, dtype=rdt, device=ref.device)
    with torch.cuda.device(ref.device):
        if rdt == torch.float64:
            rc = lib().sgwb_reduce_band_f64(_ptr(X), _ptr(G), _ptr(H) if G is not None else None, nf, npix,
                                            int(k_lo), int(k_hi), _ptr(Xbb), _ptr(Gbb), _stream())
        else:
            ws = None
            if workspace is True:
                n = band_workspace_bytes(npix, k_lo, k_hi)
                ws = torch.empty(max(n, 256), dtype=torch.uint8, device=ref.device) if n else None
            elif isinstance(workspace, torch.Tensor):
                ws = workspace
            wsz = ws.numel() if ws is not None else 0
            rc = lib().sgwb_reduce_band(_ptr(X), _ptr(G), _ptr(H) if G is not None else None, nf, npix,
                                        int(k_lo), int(k_hi), _ptr(Xbb), _ptr(Gbb), _ptr(ws), wsz, _stream())
    _check(rc, "reduce_band")
    return Xbb, Gbb


SGWB_PLAN_AUTOTUNE = 1
SGWB_PLAN_NO_GRAPH = 2


@dataclass
class Job:
    """One map job of a batched plan (float32 path).  Outputs X/G/Xbb/Gbb may be None."""
    C: torch.Tensor
    w: torch.Tensor
    fgrid: FGrid
    k0: int
    gamma: torch.Tensor
    tau: torch.Tensor
    X: torch.Tensor | None = None
    G: torch.Tensor | None = None
    H: torch.Tensor | None = None
    band: tuple | None = None
    Xbb: torch.Tensor | None = None
    Gbb: torch.Tensor | None = None
    antipodal: bool = True
    x_kernel: str = "auto"


class Plan:
    """A batched plan: all jobs' maps in one persistent launch per kernel, replayed from a HIP graph.

    The plan holds references to every tensor of its jobs; their storage must
    not be resized while the plan lives.
    """

    def __init__(self, jobs, autotune: bool = True, graph: bool = True):
        self.jobs = list(jobs)
        arr = (_Job * len(self.jobs))()
        for i, j in enumerate(self.jobs):
            nt, nf = j.w.shape
            npix = j.gamma.shape[1]
            _require(j.C, "C", torch.complex64, (nt, nf))
            _require(j.w, "w", torch.float32, (nt, nf))
            _require(j.gamma, "gamma", torch.float32, (nt, npix))
            _require(j.tau, "tau", torch.float64, (nt, npix))
            for name, t in (("X", j.X), ("G", j.G)):
                if t is not None:
                    _require(t, name, torch.float32, (nf, npix))
                    _require_contig(t, name)
            lo, hi = j.band if j.band is not None else (0, 0)
            arr[i] = _Job(j.C.data_ptr(), j.w.data_ptr(), j.w.stride(0), nt, nf, _FGrid(j.fgrid.f0, j.fgrid.df),
                          int(j.k0), j.gamma.data_ptr(), j.tau.data_ptr(), npix,
                          (SGWB_MAPS_ANTIPODAL if j.antipodal else 0) | (SGWB_MAPS_VALU_X if j.x_kernel == "valu" else 0),
                          j.X.data_ptr() if j.X is not None else None, j.G.data_ptr() if j.G is not None else None,
                          j.H.data_ptr() if j.H is not None else None, int(lo), int(hi),
                          j.Xbb.data_ptr() if j.Xbb is not None else None,
                          j.Gbb.data_ptr() if j.Gbb is not None else None)
        flags = (SGWB_PLAN_AUTOTUNE if autotune else 0) | (0 if graph else SGWB_PLAN_NO_GRAPH)
        self._h = ctypes.c_void_p()
        self.device = self.jobs[0].C.device
        with torch.cuda.device(self.device):
            torch.cuda.synchronize()
            _check(lib().sgwb_plan_create(arr, len(self.jobs), flags, ctypes.byref(self._h)), "plan_create")

    def launch(self):
        with torch.cuda.device(self.device):
            _check(lib().sgwb_plan_launch(self._h, _stream()), "plan_launch")

    def describe(self) -> dict:
        import json

        buf = ctypes.create_string_buffer(8192)
        _check(lib().sgwb_plan_describe(self._h, buf, len(buf)), "plan_describe")
        return json.loads(buf.value.decode())

    def close(self):
        if self._h:
            lib().sgwb_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


SGWB_EAGAIN = 1
SGWB_EBUSY = -4


@dataclass
class Dataset:
    """One baseline's resident folded day: C complex64 [nt][nf], w float32 [nt][nf],
    H float32 [nf] covering absolute bins [k0, k0 + nf) of fgrid."""
    C: torch.Tensor
    w: torch.Tensor
    H: torch.Tensor
    fgrid: FGrid
    k0: int
    sites: tuple
    tgrid: TGrid


class Server:
    """Continuous-batching query server (C++ worker thread inside libsgwb)."""

    def __init__(self, datasets, slots: int = 4, hbm_budget_bytes: int = 0, queue_capacity: int = 0):
        self.datasets = list(datasets)
        arr = (_Dataset * len(self.datasets))()
        for i, d in enumerate(self.datasets):
            nt, nf = d.w.shape
            _require(d.C, "C", torch.complex64, (nt, nf))
            _require(d.w, "w", torch.float32, (nt, nf))
            _require(d.H, "H", torch.float32, (nf,))
            if d.C.stride(0) != d.w.stride(0):
                raise SgwbError("C and w must share their row stride")
            tg = _TGrid(int(d.tgrid.nt), float(d.tgrid.t0), float(d.tgrid.stride), float(d.tgrid.dur))
            if d.tgrid.nt != nt:
                raise SgwbError("tgrid.nt must match the rows of C")
            arr[i] = _Dataset(d.C.data_ptr(), d.w.data_ptr(), d.w.stride(0), nf, _FGrid(d.fgrid.f0, d.fgrid.df),
                              int(d.k0), d.H.data_ptr(), _baseline(d.sites), tg)
        self._arr = arr
        cfg = _ServerCfg(ctypes.cast(arr, ctypes.c_void_p), len(self.datasets), int(hbm_budget_bytes), int(slots),
                         int(queue_capacity))
        self.device = self.datasets[0].C.device
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            torch.cuda.synchronize()
            _check(lib().sgwb_server_create(ctypes.byref(cfg), ctypes.byref(self._h)), "server_create")

    def submit(self, dataset: int, nside: int, k_lo: int, k_hi: int) -> int:
        """Queue a query; returns its ticket (raises on a bad query, returns -1 if the queue is full)."""
        t = ctypes.c_uint64()
        rc = lib().sgwb_server_submit(self._h, ctypes.byref(_Query(dataset, nside, k_lo, k_hi)), ctypes.byref(t))
        if rc == SGWB_EBUSY:
            return -1
        _check(rc, "server_submit")
        return int(t.value)

    def poll(self, ticket: int):
        """None while running; else a dict with status, npix and timestamps (seconds)."""
        r = _Result()
        rc = lib().sgwb_server_poll(self._h, ticket, ctypes.byref(r))
        if rc == SGWB_EAGAIN:
            return None
        _check(rc, "server_poll")
        return {"status": r.status, "npix": r.npix, "t_submit": r.t_submit_s, "t_start": r.t_start_s,
                "t_done": r.t_done_s}

    def fetch(self, ticket: int, npix: int):
        """Copy a finished query's (Xbb, Gbb) into new device tensors."""
        Xbb = torch.empty(npix, dtype=torch.float32, device=self.device)
        Gbb = torch.empty_like(Xbb)
        with torch.cuda.device(self.device):
            _check(lib().sgwb_server_fetch(self._h, ticket, _ptr(Xbb), _ptr(Gbb), _stream()), "server_fetch")
        return Xbb, Gbb

    def release(self, ticket: int):
        _check(lib().sgwb_server_release(self._h, ticket), "server_release")

    def stats(self) -> dict:
        import json

        buf = ctypes.create_string_buffer(4096)
        _check(lib().sgwb_server_stats(self._h, buf, len(buf)), "server_stats")
        return json.loads(buf.value.decode())

    def close(self):
        if self._h:
            lib().sgwb_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def healpix_centres(nside: int, device=None):
    """(xyz float64 [npix][3], antipode int32 [npix]) computed on the device."""
    device = torch.device("cuda") if device is None else torch.device(device)
    npix = npix_of(nside)
    xyz = torch.empty((npix, 3), dtype=torch.float64, device=device)
    anti = torch.empty(npix, dtype=torch.int32, device=device)
    with torch.cuda.device(device):
        _check(lib().sgwb_healpix_centres(int(nside), _ptr(xyz), _ptr(anti), _stream()), "healpix_centres")
    return xyz, anti


def device_supported() -> bool:
    return lib().sgwb_device_supported() == 1
