"""Pins for the oracle's narrowband dirty map X, Fisher diagonal G and band sums.

Each check is fixed by something other than the oracle's own loop:
  * tau = 0 reduces X to a plain matrix-vector product gamma^T (w Re C) (NumPy);
  * a noise-free point source at a pixel centre, C = A gamma(t,p0) H e^{-2 pi i f tau(t,p0)},
    gives X(k,p0) = A H(f_k) G(k,p0) exactly (Eq. eq_dirtymap with the injected
    CSD of Eq. eq_expCSD; every phase cancels at p0);
  * linearity in C: X(noise + source) - X(noise) = A H G at p0;
  * brute force on nside 2 by the paper's own per-bin route (materialised ORF,
    complex matrix product, Secs. III.C-III.E);
  * G is a plain matrix product W^T gamma^2; G >= 0; rank-one closed form
    w(f) sum_t gamma^2 for a stationary day; antipodal symmetry of G;
  * S = sum_t |w gamma| |C| bounds |X|;
  * band sums are plain NumPy sums, and the point-source identity carries over;
  * the point-spread spot of a source shrinks as the frequency rises (Sec. IV,
    Fig. 4: the baseline resolves finer angles at shorter wavelengths).
"""
import numpy as np
import pytest

import synth
from oracle import paper_form


def _small_case(oracle_mod, nside=2, nt=24, nf=40, k0=7, bl="AB", seed=11, f0=20.0, df=0.25):
    det = synth.baseline_sites(bl)
    gamma, tau = oracle_mod.geometry(det, nside, nt, 0.0, 3600.0, 3600.0)
    f = f0 + (k0 + np.arange(nf)) * df
    C = synth.noise_csd(seed, nt, f)
    w = synth.weights(f, synth.segment_scale(nt, 100 + seed))
    return dict(gamma=gamma, tau=tau, f=f, C=C, w=w, f0=f0, df=df, k0=k0)


def test_zero_delay_is_matvec(oracle_mod):
    c = _small_case(oracle_mod)
    tau0 = np.zeros_like(c["tau"])
    X, G = oracle_mod.maps(c["C"], c["w"], c["f0"], c["df"], c["k0"], c["gamma"], tau0)
    want = (c["w"] * c["C"].real).T @ c["gamma"]
    np.testing.assert_allclose(X, want, rtol=1e-12, atol=1e-14 * np.abs(want).max())


@pytest.mark.parametrize("bl", ["AB", "BC"])
def test_point_source_identity(oracle_mod, bl):
    c = _small_case(oracle_mod, nside=4, bl=bl, k0=300, df=1.0)
    p0, A = 37, 0.3
    C = np.zeros_like(c["C"])
    synth.add_point_source(C, c["f"], A, c["gamma"][:, p0], c["tau"][:, p0])
    X, G = oracle_mod.maps(C, c["w"], c["f0"], c["df"], c["k0"], c["gamma"], c["tau"])
    H = synth.spectrum_H(c["f"])
    np.testing.assert_allclose(X[:, p0], A * H * G[:, p0], rtol=1e-12)


def test_linearity_with_noise(oracle_mod):
    c = _small_case(oracle_mod, nside=4)
    p0, A = 100, 0.05
    Cs = c["C"].copy()
    synth.add_point_source(Cs, c["f"], A, c["gamma"][:, p0], c["tau"][:, p0])
    Xn, G = oracle_mod.maps(c["C"], c["w"], c["f0"], c["df"], c["k0"], c["gamma"], c["tau"])
    Xs, _ = oracle_mod.maps(Cs, c["w"], c["f0"], c["df"], c["k0"], c["gamma"], c["tau"])
    H = synth.spectrum_H(c["f"])
    np.testing.assert_allclose(Xs[:, p0] - Xn[:, p0], A * H * G[:, p0], rtol=1e-9)


def test_conjugation_symmetry(oracle_mod):
    c = _small_case(oracle_mod)
    X1, _ = oracle_mod.maps(c["C"], c["w"], c["f0"], c["df"], c["k0"], c["gamma"], c["tau"])
    X2, _ = oracle_mod.maps(np.conj(c["C"]), c["w"], c["f0"], c["df"], c["k0"], c["gamma"], -c["tau"])
    np.testing.assert_allclose(X2, X1, rtol=1e-13, atol=1e-15 * np.abs(X1).max())


@pytest.mark.parametrize("bl", ["AB", "AC"])
def test_brute_force_paper_route_nside2(oracle_mod, bl):
    c = _small_case(oracle_mod, nside=2, bl=bl, nt=30, nf=33, k0=1000, df=0.25)
    X, G, S = oracle_mod.maps(c["C"], c["w"], c["f0"], c["df"], c["k0"], c["gamma"], c["tau"],
                              with_scale=True)
    Xp = paper_form.narrowband_maps(c["C"], c["w"], c["f"], c["gamma"], c["tau"])
    np.testing.assert_allclose(X, Xp, rtol=0, atol=1e-12 * S.max())
    np.testing.assert_allclose(G, paper_form.fisher_diagonal(c["w"], c["gamma"]), rtol=1e-12)
    assert np.all(np.abs(X) <= S * (1 + 1e-12))


def test_fisher_properties(oracle_mod):
    c = _small_case(oracle_mod, nside=4)
    _, G = oracle_mod.maps(c["C"], c["w"], c["f0"], c["df"], c["k0"], c["gamma"], c["tau"])
    assert np.all(G >= 0)
    om = oracle_mod.healpix_centres(4)
    q = np.argmax(om @ (-om).T, axis=1)
    np.testing.assert_allclose(G[:, q], G, rtol=1e-13)
    # stationary day: rank one, w(f) * sum_t gamma^2
    w1 = synth.weights(c["f"], np.ones(c["w"].shape[0]))
    _, G1 = oracle_mod.maps(c["C"], w1, c["f0"], c["df"], c["k0"], c["gamma"], c["tau"])
    np.testing.assert_allclose(G1, np.outer(w1[0], (c["gamma"] ** 2).sum(axis=0)), rtol=1e-13)


def test_maps_at_matches_full(oracle_mod):
    c = _small_case(oracle_mod, nside=2)
    X, G, S = oracle_mod.maps(c["C"], c["w"], c["f0"], c["df"], c["k0"], c["gamma"], c["tau"],
                              with_scale=True)
    rng = np.random.default_rng(3)
    cols = rng.integers(0, X.shape[0], 50)
    pix = rng.integers(0, X.shape[1], 50)
    Xa, Ga, Sa = oracle_mod.maps_at(c["C"], c["w"], c["f0"], c["df"], c["k0"], c["gamma"], c["tau"],
                                   cols, pix)
    np.testing.assert_array_equal(Xa, X[cols, pix])
    np.testing.assert_array_equal(Ga, G[cols, pix])
    np.testing.assert_array_equal(Sa, S[cols, pix])


def test_band_sums(oracle_mod):
    c = _small_case(oracle_mod, nside=4, nf=64)
    p0, A = 5, 0.2
    C = np.zeros_like(c["C"])
    synth.add_point_source(C, c["f"], A, c["gamma"][:, p0], c["tau"][:, p0])
    X, G = oracle_mod.maps(C, c["w"], c["f0"], c["df"], c["k0"], c["gamma"], c["tau"])
    H = synth.spectrum_H(c["f"])
    Xbb, Gbb = oracle_mod.band(X, G, H, 3, 50)
    np.testing.assert_allclose(Xbb, X[3:50].sum(axis=0), rtol=1e-13, atol=1e-300)
    np.testing.assert_allclose(Gbb, (H[3:50, None] * G[3:50]).sum(axis=0), rtol=1e-13)
    np.testing.assert_allclose(Xbb[p0], A * Gbb[p0], rtol=1e-12)
    e1, e2 = oracle_mod.band(X, G, H, 10, 10)
    assert np.all(e1 == 0) and np.all(e2 == 0)


@pytest.mark.parametrize("p0", [100, 1500, 2900])
def test_point_spread_narrows_with_frequency(oracle_mod, p0):
    """Sec. IV, Fig. 4: the dirty map of a noise-free point source over one
    sidereal day has a spot whose size falls with frequency (diffraction limit
    ~ c / (f |dx|)).  Spot = the pixels with X(f,p) >= X(f,p0) / 2, at 40, 200,
    360 and 520 Hz on nside 16; above 40 Hz the source pixel is the maximum."""
    det = synth.baseline_sites("AB")
    nside, nt = 16, 48
    gamma, tau = oracle_mod.geometry(det, nside, nt, 0.0, 86164.0905 / nt, 86164.0905 / nt)
    f0, df, k0, nf = 40.0, 160.0, 0, 4
    f = f0 + (k0 + np.arange(nf)) * df
    C = np.zeros((nt, nf), np.complex128)
    synth.add_point_source(C, f, 1.0, gamma[:, p0], tau[:, p0])
    X, _ = oracle_mod.maps(C, np.ones((nt, nf)), f0, df, k0, gamma, tau)
    spot = [int((X[k] >= 0.5 * X[k, p0]).sum()) for k in range(nf)]
    assert all(a > b for a, b in zip(spot, spot[1:]))
    assert spot[0] > 10 * spot[-1]
    assert all(int(X[k].argmax()) == p0 for k in range(1, nf))
