"""Pins of the oracle's folding (Sec. II.B).  The strongest one compares the
folded route with the unfolded maximum-likelihood quantities over absolute time,
X = Re K^H N^-1 C and Gamma_pp = Re K^H N^-1 K with the tridiagonal inverse noise
covariance of overlapping windows, built as a dense matrix: the paper's point
that folding is exact because the geometry repeats every sidereal day."""
import numpy as np

import synth
from tests._cases import freqs

W = synth.HANN_OVERLAP_W
T_S = 86164.0905


def _days(seed, ndays, nt, nf, p_missing=0.1):
    rng = np.random.default_rng(seed)
    s = rng.uniform(0.5, 2.0, (ndays, nt, nf))
    C = rng.standard_normal((ndays, nt, nf)) + 1j * rng.standard_normal((ndays, nt, nf))
    present = synth.day_presence(seed + 1, ndays, nt, p_missing)
    s = s * present[:, :, None]
    C = C * present[:, :, None]
    return C, s, present


def test_single_day_without_overlap(oracle_mod):
    C, s, present = _days(1, 1, 20, 6, p_missing=0.0)
    v, u, w, x = oracle_mod.fold(C, s, present, 0.0)
    np.testing.assert_array_equal(v, s[0])
    np.testing.assert_allclose(x, s[0] * C[0], rtol=1e-15)
    assert not u.any() and not w.any()


def test_empty_days_change_nothing(oracle_mod):
    C, s, present = _days(2, 4, 15, 5)
    present[2] = False
    s[2] = 0.0
    C[2] = 0.0
    ref = oracle_mod.fold(C, s, present, W)
    # the same three days with the empty one removed (days 1 and 3 are then adjacent
    # in the data, but day 2's absence already broke their neighbour link)
    keep = [0, 1, 3]
    C2, s2, p2 = C[keep], s[keep], present[keep]
    # separate days 1 and 3 by one empty segment so no new neighbour link appears
    got = oracle_mod.fold(np.concatenate([C2[:2], np.zeros_like(C2[:1]), C2[2:]]),
                          np.concatenate([s2[:2], np.zeros_like(s2[:1]), s2[2:]]),
                          np.concatenate([p2[:2], np.zeros_like(p2[:1]), p2[2:]]), W)
    for a, b in zip(ref, got):
        np.testing.assert_array_equal(a, b)


def test_identical_days_cross_day_neighbours(oracle_mod):
    ndays, nt, nf = 5, 12, 3
    C1, s1, _ = _days(3, 1, nt, nf, p_missing=0.0)
    C = np.repeat(C1, ndays, axis=0)
    s = np.repeat(s1, ndays, axis=0)
    v, u, w, x = oracle_mod.fold(C, s, np.ones((ndays, nt), bool), W)
    np.testing.assert_allclose(v, ndays * s1[0], rtol=1e-14)
    # segment 0 has a predecessor on every day but the first; the last segment a
    # successor on every day but the last
    np.testing.assert_allclose(u[0], (ndays - 1) * 0.5 * W * (s1[0, 0] + s1[0, -1]), rtol=1e-14)
    np.testing.assert_allclose(w[-1], (ndays - 1) * 0.5 * W * (s1[0, -1] + s1[0, 0]), rtol=1e-14)
    np.testing.assert_allclose(u[1:], ndays * 0.5 * W * (s1[0, 1:] + s1[0, :-1]), rtol=1e-14)


def test_folding_equals_the_unfolded_likelihood(oracle_mod):
    ndays, nt, nf, nside, k0 = 4, 10, 3, 2, 200
    df = 1 / 32
    stride = T_S / nt  # segments tile the sidereal day exactly: the geometry repeats
    g, t = oracle_mod.geometry(synth.baseline_sites("AB"), nside, nt, 0.0, stride, 2 * stride)
    C, s, present = _days(4, ndays, nt, nf)
    v, u, w, x = oracle_mod.fold(C, s, present, W)
    f = freqs(20.0, df, k0, nf)
    # folded route: dirty map of x with unit weights; overlap-corrected Fisher diagonal
    Xf, _ = oracle_mod.maps(x, np.ones((nt, nf)), 20.0, df, k0, g, t)
    Gf, Gi, _ = oracle_mod.fisher_overlap(v, u, w, 20.0, df, k0, g, t)
    # unfolded route over absolute time a = d nt + tau
    nseg = ndays * nt
    pa = present.reshape(nseg)
    for k in range(nf):
        sa = s.reshape(nseg, nf)[:, k]
        Ninv = np.diag(sa)
        for a in range(1, nseg):
            if pa[a] and pa[a - 1]:
                Ninv[a, a - 1] = Ninv[a - 1, a] = -0.5 * W * (sa[a] + sa[a - 1])
        Ca = C.reshape(nseg, nf)[:, k]
        Kx = np.tile(g * np.exp(-2j * np.pi * f[k] * t), (ndays, 1))  # dirty-map convention
        X = np.real(np.einsum("ap,ab,b->p", Kx.conj(), Ninv, Ca))
        Kg = np.tile(g * np.exp(2j * np.pi * f[k] * t), (ndays, 1))
        G = np.real(np.einsum("ap,ab,bp->p", Kg.conj(), Ninv, Kg))
        np.testing.assert_allclose(Xf[k], X, rtol=1e-10, atol=1e-11 * np.abs(X).max())
        np.testing.assert_allclose(Gf[k], G, rtol=1e-10)
        assert np.max(np.abs(Gi[k])) < 1e-10 * np.abs(G).max()
