"""Pins of the oracle's network sum and pixel contractions (Sec. V and the sum
over baselines of Eq. eq:narrowband)."""
import numpy as np

import synth
from tests._cases import freqs, make_csd


def test_network_sum_is_the_elementwise_sum(oracle_mod):
    rng = np.random.default_rng(1)
    maps = [rng.standard_normal((7, 48)) for _ in range(3)]
    np.testing.assert_allclose(oracle_mod.network_sum(maps), maps[0] + maps[1] + maps[2], rtol=1e-15)


def test_contractions_are_pixel_sums(oracle_mod):
    rng = np.random.default_rng(2)
    M = rng.standard_normal((5, 192))
    sel = np.array([3, 17, 100, 191])
    np.testing.assert_allclose(oracle_mod.contract(M, sel), M[:, sel].sum(axis=1), rtol=1e-14)
    np.testing.assert_allclose(oracle_mod.contract(M), M.sum(axis=1), rtol=1e-13)
    assert np.all(oracle_mod.contract(M, np.array([], dtype=np.int64)) == 0.0)


def test_isotropic_contraction_is_the_matched_filter_with_the_summed_overlap(oracle_mod):
    """sum_p X(k,p) = sum_t w Re[C sum_p gamma e^{2 pi i f tau}]: the dirty map of the
    pixel-summed overlap (the isotropic ORF at the HEALPix quadrature), by NumPy."""
    nt, nf, nside, k0, df = 24, 6, 4, 300, 1 / 32
    g, t = oracle_mod.geometry(synth.baseline_sites("AB"), nside, nt, 0.0, 3600.0, 3600.0)
    f = freqs(20.0, df, k0, nf)
    C, w = make_csd(5, nt, f, dtype=np.complex128)
    X, _ = oracle_mod.maps(C, w, 20.0, df, k0, g, t)
    iso = oracle_mod.contract(X)
    orf = np.stack([(g * np.exp(2j * np.pi * fk * t)).sum(axis=1) for fk in f], axis=1)  # [nt][nf]
    ref = np.sum(w * np.real(C * orf), axis=0)
    np.testing.assert_allclose(iso, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


def test_directed_contraction_recovers_a_point_source(oracle_mod):
    """A noise-free source at p0: the directed statistic over {p0} is A H Gamma(k, p0)."""
    nt, nf, nside, df = 30, 4, 4, 0.25
    g, t = oracle_mod.geometry(synth.baseline_sites("AB"), nside, nt, 0.0, 2880.0, 2880.0)
    f = freqs(20.0, df, 0, nf)
    w = synth.weights(f, np.ones(nt))
    C = np.zeros((nt, nf), dtype=np.complex128)
    p0 = 37
    synth.add_point_source(C, f, 0.1, g[:, p0], t[:, p0])
    X, G = oracle_mod.maps(C, w, 20.0, df, 0, g, t)
    d = oracle_mod.contract(X, np.array([p0]))
    np.testing.assert_allclose(d, 0.1 * synth.spectrum_H(f) * G[:, p0], rtol=1e-12)
