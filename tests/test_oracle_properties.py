"""Property tests of the oracle (hypothesis): invariants that hold for any
detector pair, time grid, frequency grid and data, drawn at random, so that a
mistake the fixed pins happen not to exercise still fails one of them.

  * seeds (Sec. III.D): the combined antenna pattern equals the projector form
    2 tr(P D_a P D_b) - tr(P D_a) tr(P D_b) (P the transverse projector of the
    direction; independent of the polarisation basis the oracle uses), it is
    even and the delay odd under Omega -> -Omega, |tau| <= |x_a - x_b| / c, and
    swapping the detectors keeps gamma and flips tau;
  * dirty map and Fisher diagonal (Eq. eq_dirtymap split per bin, Eq.
    eq_fisher with p = p'): X is linear in C and Gam linear in w; (C, tau) ->
    (conj C, -tau) leaves X unchanged; reordering the segments changes nothing
    (the sum over t commutes); |X| <= S; Gam >= 0; a shift of the absolute bin
    grid by one bin equals the same maps of the shifted frequencies;
  * band sums (Sec. V): adjacent bands add, and X_bb is linear;
  * folding (Sec. II.B): one day without overlapping windows (W = 0) gives
    v = s, u = w = 0, x = s C; folding two halves of the days and adding gives
    the fold of all days, for v always and for u, w, x when no neighbour pair
    with data crosses the split;
  * full Fisher matrix for general weights (Eq. eq_fisher, Sec. V): symmetric,
    positive semi-definite for w >= 0, linear in w, segment-order invariant,
    diagonal = band-summed per-bin diagonal.  Planted in a copy of the oracle,
    tau_p + tau_q for tau_p - tau_q, a dropped H and gamma_p^2 for
    gamma_p gamma_q each fail it.
"""
import numpy as np
import pytest

hypothesis = pytest.importorskip("hypothesis")
from hypothesis import given, settings, strategies as st  # noqa: E402

C_LIGHT = 299792458.0
SETTINGS = settings(max_examples=25, deadline=None, derandomize=True)

lat = st.floats(-89.0, 89.0)
lon = st.floats(-180.0, 180.0)
az = st.floats(0.0, 360.0)
detector = st.tuples(lat, lon, az)


def _rotz(th):
    c, s = np.cos(th), np.sin(th)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])


def _projector_gamma(DA, DB, om):
    out = np.empty(om.shape[0])
    for i, n in enumerate(om):
        P = np.eye(3) - np.outer(n, n)
        A, B = P @ DA @ P, P @ DB @ P
        out[i] = 2.0 * np.trace(A @ B) - np.trace(P @ DA) * np.trace(P @ DB)
    return out


@SETTINGS
@given(a=detector, b=detector, t0=st.floats(0.0, 86164.0), nt=st.integers(1, 4), nside=st.sampled_from([1, 2, 4]))
def test_seeds_for_any_baseline(oracle_mod, a, b, t0, nt, nside):
    det = a + b
    stride = 86164.0905 / 7.0
    g, tau = oracle_mod.geometry(det, nside, nt, t0, stride, stride)
    om = oracle_mod.healpix_centres(nside)
    rA, DA = oracle_mod.detector(*a)
    rB, DB = oracle_mod.detector(*b)
    anti = np.array([int(np.argmin(np.linalg.norm(om + v, axis=1))) for v in om])
    bound = np.linalg.norm(rA - rB) / C_LIGHT
    for k in range(nt):
        R = _rotz(2 * np.pi * (t0 + k * stride + stride / 2) / 86164.0905)
        np.testing.assert_allclose(g[k], _projector_gamma(R @ DA @ R.T, R @ DB @ R.T, om), atol=1e-13)
        np.testing.assert_allclose(g[k][anti], g[k], atol=1e-13)
        np.testing.assert_allclose(tau[k][anti], -tau[k], atol=1e-17)
        assert np.all(np.abs(tau[k]) <= bound * (1 + 1e-12) + 1e-18)
    g2, tau2 = oracle_mod.geometry(b + a, nside, nt, t0, stride, stride)
    np.testing.assert_allclose(g2, g, atol=1e-13)
    np.testing.assert_allclose(tau2, -tau, atol=1e-17)


def _inputs(seed, nt, nf, npix):
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((nt, nf)) + 1j * rng.standard_normal((nt, nf))
    w = rng.uniform(0.1, 2.0, (nt, nf))
    gamma = rng.uniform(-1.0, 1.0, (nt, npix))
    tau = rng.uniform(-0.04, 0.04, (nt, npix))
    return C, w, gamma, tau


grid = st.tuples(st.floats(1.0, 500.0), st.sampled_from([0.25, 1 / 32, 1.0, 0.1]), st.integers(0, 5000))


@SETTINGS
@given(seed=st.integers(0, 2**31), nt=st.integers(1, 9), nf=st.integers(1, 12), npix=st.integers(1, 10), g=grid,
       a=st.floats(-3.0, 3.0), b=st.floats(-3.0, 3.0))
def test_maps_invariants(oracle_mod, seed, nt, nf, npix, g, a, b):
    f0, df, k0 = g
    C1, w, gamma, tau = _inputs(seed, nt, nf, npix)
    C2, w2, _, _ = _inputs(seed + 1, nt, nf, npix)
    X1, G, S = oracle_mod.maps(C1, w, f0, df, k0, gamma, tau, with_scale=True)
    X2, _ = oracle_mod.maps(C2, w, f0, df, k0, gamma, tau)
    X12, _ = oracle_mod.maps(a * C1 + b * C2, w, f0, df, k0, gamma, tau)
    scale = np.abs(a) * S + np.abs(b) * oracle_mod.maps(C2, w, f0, df, k0, gamma, tau, with_scale=True)[2] + 1e-300
    assert np.all(np.abs(X12 - (a * X1 + b * X2)) <= 1e-12 * scale)
    # Gam linear in w, and >= 0 for w >= 0
    _, G2 = oracle_mod.maps(C1, w2, f0, df, k0, gamma, tau)
    _, Gab = oracle_mod.maps(C1, abs(a) * w + abs(b) * w2, f0, df, k0, gamma, tau)
    np.testing.assert_allclose(Gab, abs(a) * G + abs(b) * G2, rtol=1e-12, atol=1e-300)
    assert np.all(G >= 0)
    # conjugation symmetry and |X| <= S
    Xc, _ = oracle_mod.maps(np.conj(C1), w, f0, df, k0, gamma, -tau)
    assert np.all(np.abs(Xc - X1) <= 1e-12 * S + 1e-300)
    assert np.all(np.abs(X1) <= S * (1 + 1e-12))
    # the sum over segments commutes
    perm = np.random.default_rng(seed).permutation(nt)
    Xp, Gp = oracle_mod.maps(C1[perm], w[perm], f0, df, k0, gamma[perm], tau[perm])
    assert np.all(np.abs(Xp - X1) <= 1e-12 * S + 1e-300)
    np.testing.assert_allclose(Gp, G, rtol=1e-12, atol=1e-300)
    # the absolute grid: bins [k0 + 1, ..) of grid f0 are bins [k0, ..) of grid f0 + df
    Xs, _ = oracle_mod.maps(C1, w, f0 + df, df, k0, gamma, tau)
    Xt, _ = oracle_mod.maps(C1, w, f0, df, k0 + 1, gamma, tau)
    assert np.all(np.abs(Xs - Xt) <= 1e-9 * S + 1e-300)


@SETTINGS
@given(seed=st.integers(0, 2**31), nf=st.integers(1, 20), npix=st.integers(1, 8), data=st.data())
def test_band_sums_add(oracle_mod, seed, nf, npix, data):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((nf, npix))
    G = rng.uniform(0.0, 1.0, (nf, npix))
    H = rng.uniform(0.0, 2.0, nf)
    lo = data.draw(st.integers(0, nf))
    mid = data.draw(st.integers(lo, nf))
    hi = data.draw(st.integers(mid, nf))
    Xa, Ga = oracle_mod.band(X, G, H, lo, mid)
    Xb, Gb = oracle_mod.band(X, G, H, mid, hi)
    Xt, Gt = oracle_mod.band(X, G, H, lo, hi)
    sx = np.abs(X).sum(axis=0) + 1e-300
    assert np.all(np.abs(Xa + Xb - Xt) <= 1e-12 * sx)
    np.testing.assert_allclose(Ga + Gb, Gt, rtol=1e-12, atol=1e-300)
    X2 = rng.standard_normal((nf, npix))
    Xc, _ = oracle_mod.band(2.0 * X - X2, G, H, lo, hi)
    X2b, _ = oracle_mod.band(X2, G, H, lo, hi)
    assert np.all(np.abs(Xc - (2.0 * Xt - X2b)) <= 1e-12 * (2.0 * sx + np.abs(X2).sum(axis=0)))


@SETTINGS
@given(seed=st.integers(0, 2**31), ndays=st.integers(2, 5), nt=st.integers(2, 7), nf=st.integers(1, 4),
       W=st.floats(0.0, 0.2))
def test_fold_properties(oracle_mod, seed, ndays, nt, nf, W):
    rng = np.random.default_rng(seed)
    C = rng.standard_normal((ndays, nt, nf)) + 1j * rng.standard_normal((ndays, nt, nf))
    s = rng.uniform(0.1, 2.0, (ndays, nt, nf))
    present = rng.random((ndays, nt)) > 0.2
    # one day, no overlapping windows
    v, u, w, x = oracle_mod.fold(C[:1], s[:1], present[:1], 0.0)
    m = present[0][:, None]
    np.testing.assert_allclose(v, np.where(m, s[0], 0.0), rtol=1e-14)
    assert np.all(u == 0) and np.all(w == 0)
    np.testing.assert_allclose(x, np.where(m, s[0] * C[0], 0.0), rtol=1e-14, atol=1e-300)
    # v is additive over days whatever W; u, w and x add over day ranges whose
    # boundary days have no data in the last or first segment of the day (so
    # no neighbour pair crosses the split)
    half = ndays // 2
    v1 = oracle_mod.fold(C[:half], s[:half], present[:half], W)[0]
    v2 = oracle_mod.fold(C[half:], s[half:], present[half:], W)[0]
    vt = oracle_mod.fold(C, s, present, W)[0]
    np.testing.assert_allclose(v1 + v2, vt, rtol=1e-13)
    pr = present.copy()
    pr[half - 1, -1] = False
    pr[half, 0] = False
    pr[0, 0] = False
    pr[-1, -1] = False
    a = oracle_mod.fold(C[:half], s[:half], pr[:half], W)
    b = oracle_mod.fold(C[half:], s[half:], pr[half:], W)
    t = oracle_mod.fold(C, s, pr, W)
    for ai, bi, ti in zip(a, b, t):
        np.testing.assert_allclose(ai + bi, ti, rtol=1e-12, atol=1e-12)


@SETTINGS
@given(seed=st.integers(0, 2**31), nt=st.integers(1, 7), nf=st.integers(1, 10), npix=st.integers(1, 9), g=grid,
       a=st.floats(0.0, 3.0), b=st.floats(0.0, 3.0), data=st.data())
def test_full_fisher_properties(oracle_mod, seed, nt, nf, npix, g, a, b, data):
    """Full Fisher matrix for general weights (Eq. eq_fisher with the band's H,
    Sec. V), any w(t,c) >= 0: symmetric; positive semi-definite (a sum over
    segments and bins of H w k k^T with k = gamma cos / sin of the phases);
    linear in w; unchanged by reordering the segments; its diagonal is the
    band sum of the per-bin Fisher diagonal (Eq. eq_fisher at p = p')."""
    f0, df, k0 = g
    rng = np.random.default_rng(seed)
    w1 = rng.uniform(0.0, 2.0, (nt, nf))
    w2 = rng.uniform(0.0, 2.0, (nt, nf))
    H = rng.uniform(0.1, 2.0, nf)
    gamma = rng.uniform(-1.0, 1.0, (nt, npix))
    tau = rng.uniform(-0.04, 0.04, (nt, npix))
    klo = data.draw(st.integers(0, nf - 1))
    khi = data.draw(st.integers(klo + 1, nf))
    G1 = oracle_mod.fisher_full(w1, H, f0, df, k0, klo, khi, gamma, tau)
    G2 = oracle_mod.fisher_full(w2, H, f0, df, k0, klo, khi, gamma, tau)
    scale = np.abs(H[klo:khi]).sum() * (np.abs(w1).sum(axis=1) @ (gamma ** 2).sum(axis=1)) + 1e-300
    np.testing.assert_allclose(G1, G1.T, rtol=0, atol=1e-13 * scale)
    assert np.linalg.eigvalsh(0.5 * (G1 + G1.T)).min() >= -1e-12 * scale
    G12 = oracle_mod.fisher_full(a * w1 + b * w2, H, f0, df, k0, klo, khi, gamma, tau)
    np.testing.assert_allclose(G12, a * G1 + b * G2, rtol=0, atol=1e-12 * (1 + a + b) * scale)
    perm = rng.permutation(nt)
    Gp = oracle_mod.fisher_full(w1[perm], H, f0, df, k0, klo, khi, gamma[perm], tau[perm])
    np.testing.assert_allclose(Gp, G1, rtol=0, atol=1e-12 * scale)
    C = np.zeros((nt, nf), dtype=np.complex128)
    _, Gk = oracle_mod.maps(C, w1, f0, df, k0, gamma, tau)
    _, Gbb = oracle_mod.band(np.zeros_like(Gk), Gk, H, klo, khi)
    np.testing.assert_allclose(np.diag(G1), Gbb, rtol=1e-12, atol=1e-300)
