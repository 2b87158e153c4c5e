"""Seeded synthetic inputs for folded-data radiometer map-making.

Shared by the tests, the benchmark and the smoke check; used for BOTH the
oracle and the HIP library.  It holds no map-making arithmetic: it only draws
noise, builds the noise weights and spectral shape of the stated noise model,
describes the detector sites and grids, and adds point sources whose seed
columns (gamma, tau at the source pixel) the caller passes in.

Noise model of the workloads (a stand-in for the LIGO O1 folded data, which
are not available): one-sided PSD P(f) = (f/100)^-2 + 1 + (f/500)^2, spectral
shape H(f) = (f/100)^-3, weights w = a_t H / P^2 (a_t = 1 for a stationary
day), CSD C circular complex normal with E|C|^2 = P^2 (real and imaginary
parts i.i.d. N(0, P^2/2)).  A point source of amplitude A at pixel p0 adds
A gamma(t,p0) H(f) exp(-2 pi i f tau(t,p0)) to C (Sec. IV injections).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# Detector sites: (latitude deg N, longitude deg E, x-arm azimuth deg CCW from East).
DETECTORS = {
    "A": (46.5, -119.4, 126.0),
    "B": (30.6, -90.8, 198.0),
    "C": (43.6, 10.5, 71.0),
    # a fourth site, far from the others (chord to A 11.8 Mm): long-baseline test cases
    "D": (-31.5, 115.7, 45.0),
}
BASELINES = {"AB": ("A", "B"), "AC": ("A", "C"), "BC": ("B", "C"), "AD": ("A", "D")}


def baseline_sites(name: str):
    """(latA, lonA, azA, latB, lonB, azB) for a baseline name such as 'AB'."""
    a, b = BASELINES[name]
    return DETECTORS[a] + DETECTORS[b]


@dataclass
class TGrid:
    nt: int
    t0: float
    stride: float
    dur: float


@dataclass
class FGrid:
    """Absolute bin grid f_k = f0 + k df; a workload uses bins [k0, k0 + nf)."""
    f0: float
    df: float
    nf: int
    k0: int = 0

    def freqs(self) -> np.ndarray:
        return self.f0 + (self.k0 + np.arange(self.nf, dtype=np.float64)) * self.df


@dataclass
class Workload:
    name: str
    baseline: str
    nside: int
    tgrid: TGrid
    fgrid: FGrid
    noise_seed: int
    src_pix: list = field(default_factory=list)
    src_amp: list = field(default_factory=list)
    nonstationary_seed: int | None = None


# One folded sidereal day of 240 x 360 s segments (no overlap), 0.25 Hz bins.
TGRID_TINY = TGrid(nt=240, t0=0.0, stride=360.0, dur=360.0)
# One folded sidereal day of 192 s segments at 50% overlap (896 x 96 s + 192 s ~ T_s).
TGRID_FULL = TGrid(nt=898, t0=0.0, stride=96.0, dur=192.0)
# 20 Hz to 1726 Hz at 1/32 Hz.
FGRID_FULL = FGrid(f0=20.0, df=1.0 / 32.0, nf=54592)


def _sources(seed: int, npix: int, n: int = 3):
    rng = np.random.default_rng(seed)
    pix = [int(p) for p in rng.choice(npix, n, replace=False)]
    amp = [float(a) for a in rng.uniform(0.05, 0.2, n)]
    return pix, amp


def workload(cfg: int, baseline: str = "AB") -> Workload:
    """The named workloads: 1 tiny, 2 full band nside 32, 3 full band nside 64,
    4 the batched jobs (use ``batched_jobs``)."""
    if cfg == 1:
        return Workload("tiny", baseline, 8, TGRID_TINY, FGrid(20.0, 0.25, 1024), 1, [100], [0.1])
    if cfg == 2:
        pix, amp = _sources(2, 12 * 32 * 32)
        return Workload("full_band_nside32", baseline, 32, TGRID_FULL, FGrid(20.0, 1 / 32, 54592), 2, pix, amp)
    if cfg == 3:
        # Same data as workload 2: the source directions are the nside-32 pixel
        # centres; at nside 64 the caller injects them at the nearest nside-64
        # centre.
        pix, amp = _sources(2, 12 * 32 * 32)
        return Workload("full_band_nside64", baseline, 64, TGRID_FULL, FGrid(20.0, 1 / 32, 54592), 2, pix, amp)
    raise ValueError(cfg)


def batched_jobs():
    """Uneven batch: AB nside 64 full band, AC nside 32 20-500 Hz, BC nside 16 100-300 Hz."""
    pix, amp = _sources(2, 12 * 32 * 32)
    df = 1 / 32
    return [
        Workload("AB", "AB", 64, TGRID_FULL, FGrid(20.0, df, 54592, 0), 4, pix, amp),
        Workload("AC", "AC", 32, TGRID_FULL, FGrid(20.0, df, 15360, 0), 5, pix, amp),
        Workload("BC", "BC", 16, TGRID_FULL, FGrid(20.0, df, 6400, 2560), 6, pix, amp),
    ]


def noise_psd(f):
    f = np.asarray(f, dtype=np.float64)
    return (f / 100.0) ** -2 + 1.0 + (f / 500.0) ** 2


def spectrum_H(f):
    f = np.asarray(f, dtype=np.float64)
    return (f / 100.0) ** -3


def segment_scale(nt: int, seed: int | None):
    """Per-segment weight factor a_t: ones, or U[0.5, 1.5] (non-stationary day)."""
    if seed is None:
        return np.ones(nt)
    return np.random.default_rng(seed).uniform(0.5, 1.5, nt)


def weights(f, a_t):
    """w(t,f) = a_t H(f) / P(f)^2, float64 [nt][nf]."""
    return np.outer(a_t, spectrum_H(f) / noise_psd(f) ** 2)


def nonstationary_weights(f, nt: int, seed: int):
    """Folded weights of a day whose noise changes shape, not only level, from
    segment to segment: w(t,f) = H(f) / (P_t(f) Q_t(f)) with per-detector
    spectra P_t = s_t P(f) (f / 100 Hz)^(e_t) g_t(f) and Q_t likewise: seeded
    level s_t in U[0.5, 1.5], tilt e_t in U[-0.3, 0.3], the scatter g_t(f) of a
    16-average spectral estimate (Gamma(16, 1/16) per bin), and a few narrow
    lines (a bin-wide power excess of 10-100x) switching on and off across the
    day.  float64 [nt][nf], of full rank (min(nt, nf)): no sum of a few
    products a(t) b(f) equals it."""
    f = np.asarray(f, dtype=np.float64)
    rng = np.random.default_rng(seed)
    P0 = noise_psd(f)
    out = np.empty((nt, f.size))
    nlines = max(1, f.size // 200)
    lines = rng.choice(f.size, size=min(nlines, f.size), replace=False)
    for t in range(nt):
        psd = []
        for _ in range(2):
            level = rng.uniform(0.5, 1.5)
            tilt = rng.uniform(-0.3, 0.3)
            P = level * P0 * (f / 100.0) ** tilt * rng.gamma(16.0, 1.0 / 16.0, f.size)
            on = lines[rng.random(lines.size) < 0.5]
            P[on] *= rng.uniform(10.0, 100.0, on.size)
            psd.append(P)
        out[t] = spectrum_H(f) / (psd[0] * psd[1])
    return out


# Neighbour weight of 50%-overlapping Hann windows (Sec. II.B).
HANN_OVERLAP_W = 3.0 / 70.0


def overlap_series(v, W: float = HANN_OVERLAP_W):
    """Neighbour series u, w of a single day in which every segment exists, from
    the inverse variances v[nt][nf] (Sec. II.B): u_t = W (v_t + v_{t-1}) / 2 for
    t >= 1 and w_t = W (v_t + v_{t+1}) / 2 for t <= nt - 2; zero where the neighbour
    is missing (u row 0, w row nt - 1: no previous or next day).  Then u_t = w_{t-1}."""
    v = np.asarray(v, dtype=np.float64)
    u = np.zeros_like(v)
    w = np.zeros_like(v)
    u[1:] = 0.5 * W * (v[1:] + v[:-1])
    w[:-1] = 0.5 * W * (v[:-1] + v[1:])
    return u, w


def day_presence(seed: int, ndays: int, nt: int, p_missing: float = 0.05):
    """Segments with data [ndays][nt] (True), a seeded fraction missing at random."""
    return np.random.default_rng(seed).random((ndays, nt)) >= p_missing


def noise_csd(seed: int, nt: int, f, dtype=np.complex128):
    """Circular complex normal C(t,f) with E|C|^2 = P(f)^2."""
    rng = np.random.default_rng(seed)
    nf = len(f)
    scale = (noise_psd(f) / np.sqrt(2.0)).astype(np.float64)
    out = np.empty((nt, nf), dtype=dtype)
    # Draw row by row to bound the float64 temporaries.
    for t in range(nt):
        z = rng.standard_normal((nf, 2))
        out[t] = (z[:, 0] + 1j * z[:, 1]) * scale
    return out


def add_point_source(C, f, amp: float, gamma_col, tau_col):
    """C += amp * gamma(t) H(f) exp(-2 pi i f tau(t)) for one source (in place)."""
    f = np.asarray(f, dtype=np.float64)
    Hf = spectrum_H(f)
    g = np.asarray(gamma_col, dtype=np.float64)
    tau = np.asarray(tau_col, dtype=np.float64)
    for t in range(C.shape[0]):
        ph = -2.0 * np.pi * f * tau[t]
        C[t] += (amp * g[t] * Hf * (np.cos(ph) + 1j * np.sin(ph))).astype(C.dtype)
    return C


def random_selection(seed: int, nrows: int, ncols: int, n_rows_sel: int, n_cols_sel: int):
    """Deterministic (row, col) sample: n_rows_sel evenly spaced rows x all cols,
    plus n_cols_sel seeded cols x all rows.  Returns two int64 arrays."""
    rows = np.unique(np.linspace(0, nrows - 1, n_rows_sel).round().astype(np.int64))
    rng = np.random.default_rng(seed)
    cols = np.sort(rng.choice(ncols, min(n_cols_sel, ncols), replace=False)).astype(np.int64)
    r1 = np.repeat(rows, ncols)
    c1 = np.tile(np.arange(ncols, dtype=np.int64), rows.size)
    r2 = np.tile(np.arange(nrows, dtype=np.int64), cols.size)
    c2 = np.repeat(cols, nrows)
    return np.concatenate([r1, r2]), np.concatenate([c1, c2])


NSIDES_SERVED = (8, 16, 32, 64, 128)


def serving_queries(rate_hz: float, duration_s: float, seed: int = 5, nf: int = 54592, max_band: int = 4096,
                    ndatasets: int = 3):
    """Poisson stream of map queries: arrival time (s), dataset index, nside,
    band [k_lo, k_hi) with length uniform on 1..max_band and a uniform start."""
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        ds = int(rng.integers(0, ndatasets))
        nside = int(NSIDES_SERVED[rng.integers(0, len(NSIDES_SERVED))])
        length = int(rng.integers(1, max_band + 1))
        lo = int(rng.integers(0, nf - length + 1))
        out.append((t, ds, nside, lo, lo + length))
    return out
