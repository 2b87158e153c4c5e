"""Pins of the oracle's overlap-corrected Fisher diagonal (Sec. II.B, Eq. fwGamma
with p = p'): each check uses a different formulation or a closed form, so a
dropped neighbour term, a wrong sign, a swapped t-1/t+1 or a conjugation slip in
the oracle fails one of them."""
import numpy as np
import pytest

import synth
from tests._cases import freqs

F0, DF = 20.0, 0.25


def _geometry(oracle_mod, nside, nt, stride):
    g, t = oracle_mod.geometry(synth.baseline_sites("AB"), nside, nt, 0.0, stride, stride)
    return g, t


def _series(seed, nt, nf, symmetric=True):
    rng = np.random.default_rng(seed)
    v = rng.uniform(0.5, 2.0, (nt, nf))
    if symmetric:
        u, w = synth.overlap_series(v)
    else:  # unrelated series, nonzero wrap entries u[0], w[-1]
        u = rng.uniform(-0.1, 0.1, (nt, nf))
        w = rng.uniform(-0.1, 0.1, (nt, nf))
    return v, u, w


def test_no_neighbours_is_the_plain_diagonal(oracle_mod):
    nt, nf, nside = 30, 6, 2
    g, t = _geometry(oracle_mod, nside, nt, 86164.0905 / nt)
    v, _, _ = _series(1, nt, nf)
    z = np.zeros_like(v)
    G, Gi, S = oracle_mod.fisher_overlap(v, z, z, F0, DF, 3, g, t)
    ref = v.T @ (g ** 2)  # sum_t v(t,k) gamma(t,p)^2 as a matrix product
    np.testing.assert_allclose(G, ref, rtol=1e-13)
    assert np.max(np.abs(Gi) / S) < 1e-14


@pytest.mark.parametrize("symmetric", [True, False])
def test_matches_tridiagonal_quadratic_form(oracle_mod, symmetric):
    """Gamma_pp = K_p^H M K_p with the periodic tridiagonal M = diag(v) - sub(u) -
    super(w), corners -u_0 and -w_{nt-1} (the folded day repeats), by NumPy
    complex algebra."""
    nt, nf, nside, k0 = 17, 5, 2, 40
    g, t = _geometry(oracle_mod, nside, nt, 5000.0)
    v, u, w = _series(2, nt, nf, symmetric)
    G, Gi, _ = oracle_mod.fisher_overlap(v, u, w, F0, DF, k0, g, t)
    f = freqs(F0, DF, k0, nf)
    for k in range(nf):
        M = np.diag(v[:, k]) - np.diag(u[1:, k], -1) - np.diag(w[:-1, k], 1)
        M[0, -1] -= u[0, k]
        M[-1, 0] -= w[-1, k]
        K = g * np.exp(2j * np.pi * f[k] * t)  # [nt][npix]
        quad = np.einsum("tp,ts,sp->p", K.conj(), M, K)
        np.testing.assert_allclose(G[k], quad.real, rtol=1e-11, atol=1e-12 * np.abs(quad).max())
        np.testing.assert_allclose(Gi[k], quad.imag, rtol=1e-9, atol=1e-11 * np.abs(quad).max())


def test_folded_series_give_a_real_diagonal(oracle_mod):
    nt, nf, nside = 40, 4, 4
    g, t = _geometry(oracle_mod, nside, nt, 86164.0905 / nt)
    v, u, w = _series(3, nt, nf)
    assert np.array_equal(u[1:], w[:-1])
    G, Gi, S = oracle_mod.fisher_overlap(v, u, w, F0, DF, 100, g, t)
    assert np.max(np.abs(Gi) / S) < 1e-13


def test_static_delays_closed_form(oracle_mod):
    """tau constant in t: every neighbour phase difference vanishes."""
    nt, nf, nside = 25, 3, 2
    g, t = _geometry(oracle_mod, nside, nt, 3000.0)
    t_static = np.repeat(t[:1], nt, axis=0)
    v, u, w = _series(4, nt, nf, symmetric=False)
    G, _, _ = oracle_mod.fisher_overlap(v, u, w, F0, DF, 7, g, t_static)
    gp = np.roll(g, 1, axis=0)   # predecessor, periodic
    gn = np.roll(g, -1, axis=0)  # successor, periodic
    ref = v.T @ g ** 2 - u.T @ (g * gp) - w.T @ (g * gn)
    np.testing.assert_allclose(G, ref, rtol=1e-12)


def test_hann_weights_keep_the_diagonal_positive(oracle_mod):
    """With W = 3/70 the neighbour matrix is diagonally dominant, so Gamma_pp > 0,
    and the correction stays within 2W of the plain diagonal."""
    nt, nf, nside = 60, 8, 4
    g, t = _geometry(oracle_mod, nside, nt, 86164.0905 / nt)
    v, u, w = _series(5, nt, nf)
    G, _, _ = oracle_mod.fisher_overlap(v, u, w, F0, 1 / 32, 2000, g, t)
    G0 = v.T @ g ** 2
    assert np.all(G > 0)
    assert np.all(np.abs(G - G0) <= 2 * synth.HANN_OVERLAP_W * 2 * G0 + 1e-12)
