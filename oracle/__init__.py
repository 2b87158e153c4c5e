"""FP64 CPU oracle for folded-data SGWB radiometer map-making (arXiv:1803.08285).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use it; the library never does.  It shares no code with the
HIP path and never imports it.

The heavy loops live in ``sgwb_oracle.c`` (plain C, double precision, libm
``cos``/``sin`` per term).  This module compiles it with gcc on first use and
wraps it with ctypes.  ``paper_form`` holds a second, independent route: the
paper's own per-bin formulation (materialised ORF, complex matrix product).

Definitions (constant prefactors dropped, real part kept):
  * seeds, Sec. III.D / Fig. 3: gamma(t,p) = sum_A F^A_1 F^A_2,
    tau(t,p) = Omega_p . dx(t) / c
  * dirty map, Eq. eq_dirtymap split per bin as in Eq. eq:narrowband:
    X(k,p) = sum_t w(t,k) gamma(t,p) Re[C(t,k) exp(2 pi i f_k tau(t,p))]
  * Fisher diagonal per bin, Eq. eq_fisher with p = p':
    G(k,p) = sum_t w(t,k) gamma(t,p)^2
  * broadband, Sec. V: Xbb = sum_k X(k,.), Gbb = sum_k H(f_k) G(k,.)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sgwb_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

T_SIDEREAL = 86164.0905
C_LIGHT = 299792458.0
EARTH_R = 6.371e6


def build(force: bool = False) -> str:
    """Compile the C oracle (gcc -O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.orc_healpix_centres.argtypes = [ctypes.c_int, dp]
        lib.orc_healpix_centres.restype = ctypes.c_int
        lib.orc_detector.argtypes = [ctypes.c_double] * 3 + [dp, dp]
        lib.orc_detector.restype = None
        lib.orc_antenna.argtypes = [dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp]
        lib.orc_antenna.restype = None
        lib.orc_geometry.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, dp, dp]
        lib.orc_geometry.restype = ctypes.c_int
        lib.orc_geometry_at.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_long, i64p, dp, dp]
        lib.orc_geometry_at.restype = ctypes.c_int
        lib.orc_maps.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_long, ctypes.c_long, dp, dp,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_long, dp, dp, dp, dp, dp,
                                 ctypes.c_int]
        lib.orc_maps.restype = None
        lib.orc_maps_at.argtypes = [ctypes.c_int, ctypes.c_long, ctypes.c_long, dp, dp, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_long, dp, dp, ctypes.c_long, i64p, i64p,
                                    dp, dp, dp, ctypes.c_int]
        lib.orc_maps_at.restype = None
        lib.orc_band.argtypes = [ctypes.c_int, ctypes.c_long, dp, dp, dp, ctypes.c_int, ctypes.c_int,
                                 dp, dp]
        lib.orc_band.restype = None
        lib.orc_fisher_overlap_at.argtypes = [ctypes.c_int, ctypes.c_long, ctypes.c_long, dp, dp, dp,
                                              ctypes.c_double, ctypes.c_double, ctypes.c_long, dp, dp,
                                              ctypes.c_long, i64p, i64p, dp, dp, dp, ctypes.c_int]
        lib.orc_fisher_overlap_at.restype = None
        lib.orc_fold.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_long, dp, dp,
                                 ctypes.POINTER(ctypes.c_ubyte), ctypes.c_double, dp, dp, dp, dp]
        lib.orc_fold.restype = None
        lib.orc_network_sum.argtypes = [ctypes.c_int, ctypes.c_long, dp, dp]
        lib.orc_network_sum.restype = None
        lib.orc_contract.argtypes = [ctypes.c_int, ctypes.c_long, dp, ctypes.c_int, i64p, dp]
        lib.orc_contract.restype = None
        lib.orc_fisher_full.argtypes = [ctypes.c_int, ctypes.c_long, ctypes.c_long, dp, dp, ctypes.c_double,
                                        ctypes.c_double, ctypes.c_long, ctypes.c_int, ctypes.c_int, dp, dp, dp,
                                        ctypes.c_int]
        lib.orc_fisher_full.restype = None
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _cplx(C) -> np.ndarray:
    """Complex array -> contiguous interleaved float64 view [..., 2]."""
    C = np.ascontiguousarray(C, dtype=np.complex128)
    return C.view(np.float64)


def default_threads() -> int:
    return len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)


def healpix_centres(nside: int) -> np.ndarray:
    """Unit vectors of the HEALPix RING pixel centres, shape [12 nside^2, 3]."""
    out = np.empty((12 * nside * nside, 3), dtype=np.float64)
    rc = _load().orc_healpix_centres(int(nside), _dp(out))
    if rc != 0:
        raise ValueError(f"healpix_centres failed ({rc})")
    return out


def detector(lat_deg: float, lon_deg: float, az_deg: float):
    """Return (position [3] in metres, response tensor [3,3]) of an L-shaped detector."""
    r = np.empty(3)
    D = np.empty(9)
    _load().orc_detector(lat_deg, lon_deg, az_deg, _dp(r), _dp(D))
    return r, D.reshape(3, 3)


def antenna(D: np.ndarray, theta: float, phi: float):
    """(F+, Fx) of response tensor D for the direction (theta, phi)."""
    D = _f64(D).reshape(9)
    fp = np.empty(1)
    fx = np.empty(1)
    _load().orc_antenna(_dp(D), float(np.cos(theta)), float(np.sin(theta)), float(phi), _dp(fp), _dp(fx))
    return float(fp[0]), float(fx[0])


def geometry(det, nside: int, nt: int, t0: float, stride: float, dur: float):
    """Seed matrices gamma[nt][npix], tau[nt][npix] (seconds), both float64.

    ``det`` = (latA, lonA, azA, latB, lonB, azB) in degrees.
    """
    det = _f64(det).reshape(6)
    npix = 12 * nside * nside
    gamma = np.empty((nt, npix))
    tau = np.empty((nt, npix))
    rc = _load().orc_geometry(_dp(det), int(nside), int(nt), float(t0), float(stride), float(dur),
                              _dp(gamma), _dp(tau))
    if rc != 0:
        raise ValueError(f"geometry failed ({rc})")
    return gamma, tau


def geometry_at(det, nside: int, nt: int, t0: float, stride: float, dur: float, pix):
    """Seed columns gamma[nt][len(pix)], tau[nt][len(pix)] for selected pixels."""
    det = _f64(det).reshape(6)
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    gamma = np.empty((nt, pix.size))
    tau = np.empty((nt, pix.size))
    rc = _load().orc_geometry_at(_dp(det), int(nside), int(nt), float(t0), float(stride), float(dur), pix.size,
                                 pix.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(gamma), _dp(tau))
    if rc != 0:
        raise ValueError(f"geometry_at failed ({rc})")
    return gamma, tau


def maps(C, w, f0: float, df: float, k0: int, gamma, tau, with_scale: bool = False,
         nthreads: int | None = None):
    """Full X[nf][npix] and G[nf][npix] (and S = sum_t |w gamma||C| if asked)."""
    Cv = _cplx(C)
    w = _f64(w)
    gamma = _f64(gamma)
    tau = _f64(tau)
    nt, nf = w.shape
    npix = gamma.shape[1]
    assert C.shape == (nt, nf) and gamma.shape == (nt, npix) and tau.shape == (nt, npix)
    X = np.empty((nf, npix))
    G = np.empty((nf, npix))
    S = np.empty((nf, npix)) if with_scale else None
    _load().orc_maps(nt, nf, nf, npix, _dp(Cv), _dp(w), float(f0), float(df), int(k0), _dp(gamma),
                     _dp(tau), _dp(X), _dp(G), _dp(S) if S is not None else None,
                     int(nthreads or default_threads()))
    return (X, G, S) if with_scale else (X, G)


def maps_at(C, w, f0: float, df: float, k0: int, gamma, tau, cols, pix, nthreads: int | None = None):
    """X, G, S at the selected (column, pixel) pairs (1-D arrays of equal length)."""
    Cv = _cplx(C)
    w = _f64(w)
    gamma = _f64(gamma)
    tau = _f64(tau)
    nt, nf = w.shape
    npix = gamma.shape[1]
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    assert cols.shape == pix.shape
    if cols.size and (cols.min() < 0 or cols.max() >= nf or pix.min() < 0 or pix.max() >= npix):
        raise IndexError("selection out of range")
    n = cols.size
    X = np.empty(n)
    G = np.empty(n)
    S = np.empty(n)
    i64p = ctypes.POINTER(ctypes.c_int64)
    _load().orc_maps_at(nt, nf, npix, _dp(Cv), _dp(w), float(f0), float(df), int(k0), _dp(gamma),
                        _dp(tau), n, cols.ctypes.data_as(i64p), pix.ctypes.data_as(i64p), _dp(X),
                        _dp(G), _dp(S), int(nthreads or default_threads()))
    return X, G, S


def fisher_overlap_at(v, u, wn, f0: float, df: float, k0: int, gamma, tau, cols, pix,
                      nthreads: int | None = None):
    """Overlap-corrected Fisher diagonal (Sec. II.B, Eq. fwGamma with p = p') at the
    selected (column, pixel) pairs: real part G, imaginary part Gi, scale S.  The
    folded day is periodic: segment 0's predecessor is segment nt - 1."""
    v, u, wn = _f64(v), _f64(u), _f64(wn)
    gamma = _f64(gamma)
    tau = _f64(tau)
    nt, nf = v.shape
    assert u.shape == v.shape and wn.shape == v.shape
    npix = gamma.shape[1]
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    assert cols.shape == pix.shape
    if cols.size and (cols.min() < 0 or cols.max() >= nf or pix.min() < 0 or pix.max() >= npix):
        raise IndexError("selection out of range")
    n = cols.size
    G = np.empty(n)
    Gi = np.empty(n)
    S = np.empty(n)
    i64p = ctypes.POINTER(ctypes.c_int64)
    _load().orc_fisher_overlap_at(nt, nf, npix, _dp(v), _dp(u), _dp(wn), float(f0), float(df), int(k0),
                                  _dp(gamma), _dp(tau), n, cols.ctypes.data_as(i64p),
                                  pix.ctypes.data_as(i64p), _dp(G), _dp(Gi), _dp(S),
                                  int(nthreads or default_threads()))
    return G, Gi, S


def fisher_overlap(v, u, wn, f0: float, df: float, k0: int, gamma, tau, nthreads: int | None = None):
    """Full overlap-corrected Fisher diagonal G[nf][npix] (and Gi, S)."""
    nf = np.asarray(v).shape[1]
    npix = np.asarray(gamma).shape[1]
    cols = np.repeat(np.arange(nf, dtype=np.int64), npix)
    pix = np.tile(np.arange(npix, dtype=np.int64), nf)
    G, Gi, S = fisher_overlap_at(v, u, wn, f0, df, k0, gamma, tau, cols, pix, nthreads)
    return G.reshape(nf, npix), Gi.reshape(nf, npix), S.reshape(nf, npix)


def fold(C, s, present, W: float):
    """Folded series (Sec. II.B) from per-day data: C complex [ndays][nt][nf],
    s = sigma^-2 [ndays][nt][nf], present bool [ndays][nt].  Returns v, u, w
    [nt][nf] and complex x [nt][nf]."""
    s = _f64(s)
    ndays, nt, nf = s.shape
    Cv = np.ascontiguousarray(np.asarray(C, dtype=np.complex128)).reshape(ndays * nt, nf)
    Cv = np.ascontiguousarray(Cv.view(np.float64))
    pres = np.ascontiguousarray(np.asarray(present, dtype=np.uint8))
    assert pres.shape == (ndays, nt)
    v = np.empty((nt, nf))
    u = np.empty((nt, nf))
    w = np.empty((nt, nf))
    x = np.empty((nt, nf), dtype=np.complex128)
    xv = x.view(np.float64)
    _load().orc_fold(ndays, nt, nf, nf, _dp(Cv), _dp(s), pres.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)),
                     float(W), _dp(v), _dp(u), _dp(w), _dp(xv))
    return v, u, w, x


def network_sum(maps):
    """Element-wise sum over baselines of equally shaped maps (sequence of arrays)."""
    arr = np.ascontiguousarray(np.stack([_f64(m) for m in maps]))
    nmaps = arr.shape[0]
    out = np.empty(arr.shape[1:])
    _load().orc_network_sum(nmaps, int(out.size), _dp(arr), _dp(out))
    return out


def contract(M, pix=None):
    """Per-row sum of M[nf][npix] over the pixel set pix (all pixels if None)."""
    M = _f64(M)
    if M.ndim == 1:
        M = M[None, :]
    nf, npix = M.shape
    out = np.empty(nf)
    if pix is None:
        _load().orc_contract(nf, npix, _dp(M), -1, None, _dp(out))
    else:
        pix = np.ascontiguousarray(pix, dtype=np.int64)
        if pix.size and (pix.min() < 0 or pix.max() >= npix):
            raise IndexError("pixel out of range")
        _load().orc_contract(nf, npix, _dp(M), int(pix.size), pix.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                             _dp(out))
    return out


def fisher_full(w, H, f0: float, df: float, k0: int, klo: int, khi: int, gamma, tau, nthreads: int | None = None):
    """Full Fisher matrix of the bins [klo, khi) (Eq. eq_fisher, broadband H
    weighting of Sec. V): G[npix][npix]."""
    w, H, gamma, tau = _f64(w), _f64(H), _f64(gamma), _f64(tau)
    nt, nf = w.shape
    npix = gamma.shape[1]
    if not (0 <= klo <= khi <= nf):
        raise IndexError("band out of range")
    G = np.empty((npix, npix))
    _load().orc_fisher_full(nt, nf, npix, _dp(w), _dp(H), float(f0), float(df), int(k0), int(klo), int(khi),
                            _dp(gamma), _dp(tau), _dp(G), int(nthreads or default_threads()))
    return G


def cg(A, b, niter: int):
    """Conjugate gradient for A x = b from x = 0, exactly niter iterations (the
    clean-map solver of the footnote to Eq. eq_ML_linear); float64 NumPy."""
    A = np.asarray(A, dtype=np.float64)
    x = np.zeros_like(np.asarray(b, dtype=np.float64))
    r = np.array(b, dtype=np.float64)
    p = r.copy()
    rr = r @ r
    for _ in range(niter):
        if rr == 0.0:
            break
        Ap = A @ p
        alpha = rr / (p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        rr_new = r @ r
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x


def band(X, G, H, klo: int, khi: int):
    """Broadband Xbb[npix] = sum_k X, Gbb[npix] = sum_k H G over rows [klo, khi)."""
    X = _f64(X)
    G = _f64(G)
    H = _f64(H)
    nf, npix = X.shape
    if not (0 <= klo <= khi <= nf):
        raise IndexError("band out of range")
    Xbb = np.empty(npix)
    Gbb = np.empty(npix)
    _load().orc_band(nf, npix, _dp(X), _dp(G), _dp(H), int(klo), int(khi), _dp(Xbb), _dp(Gbb))
    return Xbb, Gbb
