"""Pins of the oracle's full Fisher matrix and conjugate-gradient clean map
(Eqs. eq_CSD_conv, eq_ML_solution, eq_fisher, eq_ML_linear; Sec. V)."""
import numpy as np

import synth
from tests._cases import freqs

F0 = 20.0


def _setup(oracle_mod, nside=2, nt=20, nf=12, df=1.0, k0=10, seed=1):
    g, t = oracle_mod.geometry(synth.baseline_sites("AB"), nside, nt, 0.0, 86164.0905 / nt, 86164.0905 / nt)
    f = freqs(F0, df, k0, nf)
    a = np.random.default_rng(seed).uniform(0.5, 1.5, nt)
    w = synth.weights(f, a)
    H = synth.spectrum_H(f)
    return g, t, f, w, H


def test_diagonal_is_the_band_summed_fisher_diagonal(oracle_mod):
    g, t, f, w, H = _setup(oracle_mod)
    G = oracle_mod.fisher_full(w, H, F0, 1.0, 10, 2, 11, g, t)
    _, Gk = oracle_mod.maps(np.zeros(w.shape, complex), w, F0, 1.0, 10, g, t)
    _, Gbb = oracle_mod.band(np.zeros_like(Gk), Gk, H, 2, 11)
    np.testing.assert_allclose(np.diag(G), Gbb, rtol=1e-12)
    np.testing.assert_allclose(G, G.T, rtol=1e-12, atol=1e-15 * np.abs(G).max())
    assert np.linalg.eigvalsh(G).min() > -1e-10 * np.abs(G).max()


def test_noise_free_sky_satisfies_the_convolution_identity(oracle_mod):
    """C = K P (noise-free, Eq. eq_CSD_conv) gives the broadband dirty map X = Gamma P."""
    g, t, f, w, H = _setup(oracle_mod, nside=4, nt=24, nf=10, df=0.5, k0=40)
    npix = g.shape[1]
    rng = np.random.default_rng(7)
    P = np.zeros(npix)
    P[rng.choice(npix, 5, replace=False)] = rng.uniform(0.5, 2.0, 5)
    C = np.zeros(w.shape, dtype=np.complex128)
    for p in np.nonzero(P)[0]:
        synth.add_point_source(C, f, P[p], g[:, p], t[:, p])
    X, Gk = oracle_mod.maps(C, w, F0, 0.5, 40, g, t)
    Xbb, _ = oracle_mod.band(X, Gk, H, 0, 10)
    # the injected CSD carries H (Eq. eq_convolution, K = tau H gamma), w carries the other
    # H/P^2: the broadband sum of X is the H-weighted Fisher matrix times the sky
    G = oracle_mod.fisher_full(w, H, F0, 0.5, 40, 0, 10, g, t)
    np.testing.assert_allclose(Xbb, G @ P, rtol=1e-10, atol=1e-12 * np.abs(Xbb).max())
    # and conjugate gradient on (Gamma, X) moves towards the injected sky
    Pc = oracle_mod.cg(G, Xbb, 200)
    assert np.linalg.norm(G @ Pc - Xbb) < 1e-3 * np.linalg.norm(Xbb)


def test_separable_weights_reduce_to_a_delay_table(oracle_mod):
    """w(t,f) = a_t b_f: Gamma(p,p') = sum_t a_t gamma_p gamma_p' W(tau_p - tau_p'),
    W(D) = sum_f H b cos 2 pi f D (the route the GPU takes), by NumPy."""
    g, t, f, w, H = _setup(oracle_mod, nside=2, nt=15, nf=9, df=1 / 32, k0=3000)
    a = w[:, 0] / w[0, 0]
    b = w[0]
    G = oracle_mod.fisher_full(w, H, F0, 1 / 32, 3000, 0, 9, g, t)
    D = t[:, :, None] - t[:, None, :]  # [nt][p][p']
    W = np.tensordot(np.cos(2 * np.pi * D[..., None] * f), H * b, axes=([3], [0]))
    ref = np.einsum("t,tp,tq,tpq->pq", a, g, g, W)
    np.testing.assert_allclose(G, ref, rtol=1e-11, atol=1e-14 * np.abs(G).max())


def test_cg_solves_spd_systems(oracle_mod):
    rng = np.random.default_rng(3)
    B = rng.standard_normal((40, 40))
    A = B @ B.T + 40 * np.eye(40)
    x = rng.standard_normal(40)
    np.testing.assert_allclose(oracle_mod.cg(A, A @ x, 60), x, rtol=1e-9)
    assert np.all(oracle_mod.cg(A, A @ x, 0) == 0.0)
