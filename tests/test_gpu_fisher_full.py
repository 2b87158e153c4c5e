"""Full Fisher matrix of a band (Eq. eq_fisher, broadband H weighting of Sec. V)
and the conjugate-gradient clean map (Eq. eq_ML_linear and its footnote) on the
GPU against the FP64 oracle, through the C ABI.

Tolerance of G: max |G_gpu - G_oracle| / S <= 1e-5 with
S(p,q) = sum_c |H b| sum_t a |gamma_p gamma_q| (the same scale as the dirty
map's bound: each term of the band sum is bounded by it).  Budget: cubic Hermite
interpolation of the delay table (< 2.4e-7 S), float32 table entries and
interpolation arithmetic (a few 1e-7 S), float32 accumulation over the
segments (~ sqrt(nt) 6e-8 S).  The oracle entry G(p,q) depends only on pixels
p and q, so at sizes where the whole oracle matrix is slow it is evaluated on a
sampled pixel subset.
"""
import numpy as np
import pytest

import synth
from tests._cases import freqs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F0 = 20.0
CASES = [  # baseline, nside, npix used (None: all), nt, k0, nf, band, df
    ("AB", 2, None, 24, 10, 40, (0, 40), 0.25),         # one ragged tile (48 pixels)
    ("AC", 4, None, 40, 100, 64, (5, 60), 0.25),        # 3 x 3 tiles, sub-band
    ("BC", 4, 150, 33, 0, 30, (0, 30), 1.0),            # ragged multi-tile (150 = 2 x 64 + 22)
    ("AB", 8, None, 60, 53000, 64, (0, 64), 1 / 32),    # top of the band (1.68 kHz), 12 x 12 tiles
    ("AC", 2, None, 7, 63, 2, (1, 2), 0.25),            # single bin, tiny day
    ("AB", 4, 100, 30, 79000, 40, (0, 40), 1 / 32),     # 2.49 kHz: table above the LDS size, global-memory form
    ("BC", 2, None, 20, 39000, 50, (3, 47), 0.125),     # 4.9 kHz: 16 fraction bits
]


@pytest.fixture(scope="module")
def sg():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1803_08285_amd as sg

    return sg


def _inputs(sg, bl, nside, npix_used, nt, k0, nf, df, seed):
    tg = sg.TGrid(nt, 0.0, 86164.0905 / nt, 86164.0905 / nt)
    g, t = sg.build_geometry(synth.baseline_sites(bl), nside, tg)
    if npix_used is not None:
        g, t = g[:, :npix_used].contiguous(), t[:, :npix_used].contiguous()
    f = freqs(F0, df, k0, nf)
    a = synth.segment_scale(nt, seed).astype(np.float32)
    b = (synth.spectrum_H(f) / synth.noise_psd(f) ** 2).astype(np.float32)
    H = synth.spectrum_H(f).astype(np.float32)
    return g, t, a, b, H


def _scale(a, b, H, klo, khi, gh):
    """S(p,q) = sum_c |H b| sum_t a |gamma_p gamma_q|."""
    hb = np.abs(H[klo:khi].astype(np.float64) * b[klo:khi].astype(np.float64)).sum()
    ag = np.abs(gh) * a.astype(np.float64)[:, None]
    return hb * (ag.T @ np.abs(gh))


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{c[1]}-{c[2]}-{c[4]}-{c[7]}" for c in CASES])
def test_fisher_full_vs_oracle(sg, oracle_mod, case):
    bl, nside, npix_used, nt, k0, nf, (klo, khi), df = case
    g, t, a, b, H = _inputs(sg, bl, nside, npix_used, nt, k0, nf, df, 21)
    ad, bd, Hd = (torch.from_numpy(x).cuda() for x in (a, b, H))
    G = sg.fisher_full(ad, bd, Hd, sg.FGrid(F0, df), k0, klo, khi, g, t)
    torch.cuda.synchronize()
    Gg = G.cpu().numpy().astype(np.float64)
    gh, th = g.cpu().numpy().astype(np.float64), t.cpu().numpy()
    npix = gh.shape[1]
    sel = np.arange(npix) if npix <= 200 else np.sort(np.random.default_rng(4).choice(npix, 40, replace=False))
    w = np.outer(a.astype(np.float64), b.astype(np.float64))
    Go = oracle_mod.fisher_full(w, H.astype(np.float64), F0, df, k0, klo, khi, gh[:, sel], th[:, sel])
    S = _scale(a, b, H, klo, khi, gh[:, sel])
    err = np.abs(Gg[np.ix_(sel, sel)] - Go) / S
    assert np.max(err) <= 1e-5
    assert np.array_equal(Gg, Gg.T)  # both triangles written from one value


def test_fisher_full_diagonal_is_the_band_summed_diagonal(sg):
    """diag G = Gbb of the per-bin diagonal (same separable w) reduced over the band."""
    nt, nside, k0, nf, df, klo, khi = 48, 8, 200, 96, 1 / 32, 7, 90
    g, t, a, b, H = _inputs(sg, "AB", nside, None, nt, k0, nf, df, 22)
    ad, bd, Hd = (torch.from_numpy(x).cuda() for x in (a, b, H))
    G = sg.fisher_full(ad, bd, Hd, sg.FGrid(F0, df), k0, klo, khi, g, t)
    w = (ad[:, None] * bd[None, :]).contiguous()
    C = torch.zeros((nt, nf), dtype=torch.complex64, device="cuda")
    _, Gk = sg.make_maps(C, w, sg.FGrid(F0, df), k0, g, t, antipodal=False)
    _, Gbb = sg.reduce_band(None, Gk, Hd, klo, khi)
    torch.cuda.synchronize()
    d = torch.diagonal(G).double().cpu().numpy()
    ref = Gbb.double().cpu().numpy()
    assert np.max(np.abs(d - ref) / ref) <= 1e-4  # split-bf16 beam bound on the per-bin diagonal


def test_noise_free_sky_gives_x_equal_g_p(sg):
    """C = K P without noise (Eq. eq_CSD_conv): the broadband dirty map of the GPU
    path equals the GPU's full Fisher matrix times the injected sky."""
    nt, nside, k0, nf, df = 40, 4, 100, 64, 0.25
    g, t, a, b, H = _inputs(sg, "AC", nside, None, nt, k0, nf, df, 23)
    npix = g.shape[1]
    f = freqs(F0, df, k0, nf)
    gh, th = g.cpu().numpy().astype(np.float64), t.cpu().numpy()
    rng = np.random.default_rng(8)
    P = np.zeros(npix)
    P[rng.choice(npix, 4, replace=False)] = rng.uniform(0.5, 2.0, 4)
    C = np.zeros((nt, nf), dtype=np.complex128)
    for p in np.nonzero(P)[0]:
        synth.add_point_source(C, f, P[p], gh[:, p], th[:, p])
    ad, bd, Hd = (torch.from_numpy(x).cuda() for x in (a, b, H))
    w = (ad[:, None] * bd[None, :]).contiguous()
    Cd = torch.from_numpy(C.astype(np.complex64)).cuda()
    X, Gk = sg.make_maps(Cd, w, sg.FGrid(F0, df), k0, g, t, antipodal=False)
    Xbb, _ = sg.reduce_band(X, Gk, Hd, 0, nf)
    G = sg.fisher_full(ad, bd, Hd, sg.FGrid(F0, df), k0, 0, nf, g, t)
    torch.cuda.synchronize()
    lhs = Xbb.double().cpu().numpy()
    rhs = G.double().cpu().numpy() @ P
    assert np.max(np.abs(lhs - rhs)) <= 1e-4 * np.max(np.abs(lhs))


@pytest.mark.parametrize("n,niter", [(48, 10), (300, 25), (1000, 12), (333, 10), (7, 5), (5, 0)])
def test_clean_map_cg_vs_oracle(sg, oracle_mod, n, niter):
    rng = np.random.default_rng(n)
    M = rng.standard_normal((n, n + 7))
    A = (M @ M.T / n + 0.05 * np.eye(n)).astype(np.float32)
    A = np.triu(A) + np.triu(A, 1).T  # exactly symmetric in float32
    X = rng.standard_normal(n).astype(np.float32)
    P = sg.clean_map_cg(torch.from_numpy(A).cuda(), torch.from_numpy(X).cuda(), niter)
    torch.cuda.synchronize()
    Pg = P.double().cpu().numpy()
    Po = oracle_mod.cg(A.astype(np.float64), X.astype(np.float64), niter)
    if niter == 0:
        assert np.all(Pg == 0.0)
        return
    assert np.linalg.norm(Pg - Po) <= 1e-6 * np.linalg.norm(Po)


def test_clean_map_cg_on_the_fisher_matrix(sg, oracle_mod):
    """CG on the GPU's own (singular, semi-definite) full Fisher matrix with a
    dirty map in its range, X = G P for a few point sources: same iterate as the
    oracle's CG on the same matrix (15 steps: rounding differences between two
    float64 CGs stay near 1e-13 there and grow past 20 steps on this matrix), and
    the residual falls."""
    nt, nside, k0, nf, df = 40, 4, 100, 64, 0.25
    g, t, a, b, H = _inputs(sg, "AB", nside, None, nt, k0, nf, df, 24)
    ad, bd, Hd = (torch.from_numpy(x).cuda() for x in (a, b, H))
    G = sg.fisher_full(ad, bd, Hd, sg.FGrid(F0, df), k0, 0, nf, g, t)
    torch.cuda.synchronize()
    Gh = G.double().cpu().numpy()
    rng = np.random.default_rng(8)
    Pin = np.zeros(Gh.shape[0])
    Pin[rng.choice(Gh.shape[0], 4, replace=False)] = rng.uniform(0.5, 2.0, 4)
    Xh = (Gh @ Pin).astype(np.float32)
    P = sg.clean_map_cg(G, torch.from_numpy(Xh).cuda(), 15)
    torch.cuda.synchronize()
    Pg = P.double().cpu().numpy()
    Po = oracle_mod.cg(Gh, Xh.astype(np.float64), 15)
    assert np.linalg.norm(Pg - Po) <= 1e-6 * np.linalg.norm(Po)
    assert np.linalg.norm(Gh @ Pg - Xh) <= 0.05 * np.linalg.norm(Xh)


def test_fisher_full_and_clean_map_are_deterministic(sg):
    """Fixed summation orders: a second call gives the same bits (the table's chunk
    sums, the persistent tile walk and the CG reductions are order-fixed)."""
    nt, nside, k0, nf, df = 36, 8, 500, 300, 1 / 32
    g, t, a, b, H = _inputs(sg, "AC", nside, None, nt, k0, nf, df, 25)
    ad, bd, Hd = (torch.from_numpy(x).cuda() for x in (a, b, H))
    G1 = sg.fisher_full(ad, bd, Hd, sg.FGrid(F0, df), k0, 0, nf, g, t)
    G2 = sg.fisher_full(ad, bd, Hd, sg.FGrid(F0, df), k0, 0, nf, g, t)
    X = torch.diagonal(G1).contiguous()
    P1 = sg.clean_map_cg(G1, X, 20)
    P2 = sg.clean_map_cg(G2, X, 20)
    torch.cuda.synchronize()
    assert torch.equal(G1, G2)
    assert torch.equal(P1, P2)


@pytest.mark.parametrize("rank,nside,k0,nf,df", [(3, 4, 100, 64, 0.25), (2, 8, 53000, 64, 1 / 32)])
def test_fisher_full_rank_r_weights_vs_oracle(sg, oracle_mod, rank, nside, k0, nf, df):
    """w(t,c) = sum_r a_r(t) b_r(c) with unrelated factors (a noise level that drifts
    across the day with a spectral shape of its own per rank): one delay table and
    one pass per rank, against the oracle on the summed, non-separable w."""
    nt = 40
    g, t, _, _, H = _inputs(sg, "AC", nside, None, nt, k0, nf, df, 26)
    rng = np.random.default_rng(27)
    f = freqs(F0, df, k0, nf)
    a = rng.uniform(0.2, 1.0, (rank, nt)).astype(np.float32)
    b = np.stack([(synth.spectrum_H(f) / synth.noise_psd(f) ** 2) * rng.uniform(0.5, 1.5, nf)
                  for _ in range(rank)]).astype(np.float32)
    klo, khi = 2, nf - 3
    G = sg.fisher_full(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), torch.from_numpy(H).cuda(),
                       sg.FGrid(F0, df), k0, klo, khi, g, t)
    torch.cuda.synchronize()
    Gg = G.cpu().numpy().astype(np.float64)
    gh, th = g.cpu().numpy().astype(np.float64), t.cpu().numpy()
    npix = gh.shape[1]
    sel = np.arange(npix) if npix <= 200 else np.sort(np.random.default_rng(5).choice(npix, 40, replace=False))
    w = sum(np.outer(a[r].astype(np.float64), b[r].astype(np.float64)) for r in range(rank))
    Go = oracle_mod.fisher_full(w, H.astype(np.float64), F0, df, k0, klo, khi, gh[:, sel], th[:, sel])
    S = sum(_scale(a[r], b[r], H, klo, khi, gh[:, sel]) for r in range(rank))
    assert np.max(np.abs(Gg[np.ix_(sel, sel)] - Go) / S) <= 1e-5
    assert np.array_equal(Gg, Gg.T)


ANTI_CASES = [  # baseline, nside, nt, k0, nf, band, df, rank
    ("AB", 2, 24, 10, 40, (0, 40), 0.25, 1),          # one ragged tile per block (24 northern pixels)
    ("AC", 4, 40, 100, 64, (5, 60), 0.25, 1),         # 2 x 2 tiles per block, sub-band
    ("AB", 8, 60, 53000, 64, (0, 64), 1 / 32, 1),     # 1.68 kHz, 6 x 6 tiles per block
    ("BC", 2, 20, 39000, 50, (3, 47), 0.125, 1),      # 4.9 kHz: global-memory table
    ("AC", 4, 40, 100, 64, (2, 61), 0.25, 3),         # three ranks: the later passes add
]


@pytest.mark.parametrize("case", ANTI_CASES, ids=[f"{c[0]}-{c[1]}-{c[3]}-r{c[7]}" for c in ANTI_CASES])
def test_fisher_full_antipodal_vs_oracle_and_plain(sg, oracle_mod, case):
    """Antipodal seeds: only the northern blocks' triangles are computed.  Against
    the oracle at the usual bound, against the flag-free matrix within float32
    rounding of the weight products (1e-6 of S), exactly symmetric, and with the
    block structure G(a(p),a(q)) = G(p,q), G(p,a(q)) = G(q,a(p)) bit for bit."""
    bl, nside, nt, k0, nf, (klo, khi), df, rank = case
    g, t, _, _, H = _inputs(sg, bl, nside, None, nt, k0, nf, df, 31)
    rng = np.random.default_rng(32)
    f = freqs(F0, df, k0, nf)
    a = rng.uniform(0.2, 1.0, (rank, nt)).astype(np.float32)
    b = np.stack([(synth.spectrum_H(f) / synth.noise_psd(f) ** 2) * rng.uniform(0.5, 1.5, nf)
                  for _ in range(rank)]).astype(np.float32)
    ad, bd, Hd = (torch.from_numpy(x).cuda() for x in (a, b, H))
    Ga = sg.fisher_full(ad, bd, Hd, sg.FGrid(F0, df), k0, klo, khi, g, t, antipodal=True)
    Gp = sg.fisher_full(ad, bd, Hd, sg.FGrid(F0, df), k0, klo, khi, g, t, antipodal=False)
    _, anti = sg.healpix_centres(nside)
    torch.cuda.synchronize()
    A = Ga.cpu().numpy().astype(np.float64)
    P = Gp.cpu().numpy().astype(np.float64)
    gh, th = g.cpu().numpy().astype(np.float64), t.cpu().numpy()
    npix = gh.shape[1]
    S_all = sum(_scale(a[r], b[r], H, klo, khi, gh) for r in range(rank))
    assert np.array_equal(A, A.T)
    am = anti.cpu().numpy().astype(np.int64)
    assert np.array_equal(A[np.ix_(am, am)], A)  # G(a(p), a(q)) = G(p, q)
    assert np.max(np.abs(A - P) / S_all) <= 1e-6
    sel = np.arange(npix) if npix <= 200 else np.sort(np.random.default_rng(6).choice(npix, 48, replace=False))
    w = sum(np.outer(a[r].astype(np.float64), b[r].astype(np.float64)) for r in range(rank))
    Go = oracle_mod.fisher_full(w, H.astype(np.float64), F0, df, k0, klo, khi, gh[:, sel], th[:, sel])
    assert np.max(np.abs(A[np.ix_(sel, sel)] - Go) / S_all[np.ix_(sel, sel)]) <= 1e-5


def test_fisher_full_antipodal_rejects_broken_seeds(sg):
    """A delay changed at one pixel of the middle segment breaks the antipodal
    promise: the device check rejects the seeds and the matrix is NaN."""
    nt, nside, k0, nf, df = 20, 4, 100, 32, 0.25
    g, t, a, b, H = _inputs(sg, "AB", nside, None, nt, k0, nf, df, 33)
    t = t.clone()
    t[nt // 2, 3] += 1e-7
    ad, bd, Hd = (torch.from_numpy(x).cuda() for x in (a, b, H))
    G = sg.fisher_full(ad, bd, Hd, sg.FGrid(F0, df), k0, 0, nf, g, t, antipodal=True)
    torch.cuda.synchronize()
    assert bool(torch.isnan(G).all())


@pytest.mark.parametrize("case", [("AB", 4, 40, 100, 64, 0.25, 1, False), ("AC", 8, 60, 53000, 64, 1 / 32, 1, True),
                                  ("AB", 4, 40, 100, 64, 0.25, 3, True), ("BC", 4, 33, 0, 30, 1.0, 2, False)],
                         ids=["AB4", "AC8-anti", "AB4-rank3-anti", "BC4-rank2"])
def test_fisher_full_stream_and_persistent_forms_agree_bitwise(sg, monkeypatch, case):
    """The streaming kernel (the default: one table in LDS, 8 x 4 entries a
    lane) and the persistent LDS kernel (SGWB_FISHER_ONE_TABLE=persistent, 4 x 4
    a thread) add the same float32 terms in the same order: the same bits, also
    over several ranks (the later ranks add to G)."""
    bl, nside, nt, k0, nf, df, rank, anti = case
    g, t, _, _, H = _inputs(sg, bl, nside, None, nt, k0, nf, df, 34)
    rng = np.random.default_rng(35)
    f = freqs(F0, df, k0, nf)
    a = rng.uniform(0.2, 1.0, (rank, nt)).astype(np.float32)
    b = np.stack([(synth.spectrum_H(f) / synth.noise_psd(f) ** 2) * rng.uniform(0.5, 1.5, nf)
                  for _ in range(rank)]).astype(np.float32)
    ad, bd, Hd = (torch.from_numpy(x).cuda() for x in (a, b, H))
    G1 = sg.fisher_full(ad, bd, Hd, sg.FGrid(F0, df), k0, 0, nf, g, t, antipodal=anti)
    monkeypatch.setenv("SGWB_FISHER_ONE_TABLE", "persistent")
    G2 = sg.fisher_full(ad, bd, Hd, sg.FGrid(F0, df), k0, 0, nf, g, t, antipodal=anti)
    monkeypatch.delenv("SGWB_FISHER_ONE_TABLE")
    torch.cuda.synchronize()
    assert torch.equal(G1, G2)
