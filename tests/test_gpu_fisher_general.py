"""Full Fisher matrix of a band for general folded weights (Eq. eq_fisher with
any w(t,c); broadband H weighting of Sec. V) on the GPU against the FP64
oracle, through the C ABI (sgwb_fisher_full_general).

The weights are those of a day whose noise changes shape from segment to
segment (synth.nonstationary_weights: per-segment level and tilt, the scatter
of a 16-average spectral estimate, lines switching on and off), of full rank,
so no sum of a few products a(t) b(c) reproduces them.

The tables' band sums run over the bins (coarse grids, 1/4 Hz and 1 Hz here)
or over Jacobi-Anger moments of 64- or 16-bin strips (1/32 Hz, 1/8 Hz); both
bases are covered.

Tolerance of G: max |G_gpu - G_oracle| / S <= 1e-5 with
S(p,q) = sum_t (sum_c |H w(t,c)|) |gamma_p(t) gamma_q(t)|, the bound of each
term of the band and segment sums.  Budget as for the separable matrix: cubic
Hermite interpolation of each segment's delay table (< 2.4e-7 S), float32 table
entries and interpolation arithmetic (a few 1e-7 S), float32 accumulation over
the segments (~ sqrt(nt) 6e-8 S); the tables' float64 band sums add nothing
visible.  G(p,q) depends only on pixels p and q, so where the whole oracle
matrix is slow it is evaluated on a sampled pixel subset.
"""
import numpy as np
import pytest

import synth
from tests._cases import freqs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F0 = 20.0
CASES = [  # baseline, nside, npix used (None: all), nt, k0, nf, band, df, antipodal
    ("AB", 2, None, 24, 10, 40, (0, 40), 0.25, False),        # 32 Hz: short tables, one ragged tile
    ("AC", 4, None, 40, 4000, 64, (5, 60), 0.25, False),      # 1.0 kHz, AC: tables double-buffered
    ("BC", 4, 150, 33, 0, 30, (0, 30), 1.0, False),           # ragged multi-tile pixels (150 = 2 x 64 + 22)
    ("AB", 8, None, 60, 53000, 64, (0, 64), 1 / 32, False),   # 1.68 kHz, 12 x 12 tiles
    ("AB", 4, 100, 30, 79000, 40, (0, 40), 1 / 32, False),    # 2.49 kHz: tables above the LDS, global-memory form
    ("AC", 4, None, 40, 4000, 64, (5, 60), 0.25, True),       # antipodal blocks, double-buffered tables
    ("AD", 4, None, 30, 53000, 64, (0, 64), 1 / 32, False),   # 39 ms delays at 1.68 kHz: one table buffer
    ("AD", 4, None, 30, 53000, 64, (0, 64), 1 / 32, True),    # the same, antipodal
    ("AB", 8, None, 60, 53000, 64, (0, 64), 1 / 32, True),    # antipodal, 1.68 kHz
    ("BC", 2, None, 20, 39000, 50, (3, 47), 0.125, True),     # antipodal, 4.9 kHz global-memory form
    ("AC", 2, None, 7, 63, 2, (1, 2), 0.25, False),           # single bin, tiny day
    ("AB", 4, None, 30, 53010, 300, (7, 290), 1 / 32, True),  # band from mid-strip to mid-strip, 5 strips
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
    w = synth.nonstationary_weights(f, nt, seed).astype(np.float32)
    H = synth.spectrum_H(f).astype(np.float32)
    return g, t, w, H


def _scale(w, H, klo, khi, gh):
    """S(p,q) = sum_t (sum_c |H w(t,c)|) |gamma_p(t) gamma_q(t)|."""
    hw = np.abs(w[:, klo:khi].astype(np.float64) * H[klo:khi].astype(np.float64)).sum(axis=1)
    ag = np.abs(gh) * hw[:, None]
    return ag.T @ np.abs(gh)


def _oracle(oracle_mod, w, H, df, k0, klo, khi, gh, th, sel):
    return oracle_mod.fisher_full(w.astype(np.float64), H.astype(np.float64), F0, df, k0, klo, khi, gh[:, sel],
                                  th[:, sel])


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{c[1]}-{c[2]}-{c[4]}-{c[7]}-{'a' if c[8] else 'p'}"
                                             for c in CASES])
def test_fisher_full_general_vs_oracle(sg, oracle_mod, case):
    bl, nside, npix_used, nt, k0, nf, (klo, khi), df, anti = case
    g, t, w, H = _inputs(sg, bl, nside, npix_used, nt, k0, nf, df, 41)
    wd, Hd = torch.from_numpy(w).cuda(), torch.from_numpy(H).cuda()
    G = sg.fisher_full_general(wd, Hd, sg.FGrid(F0, df), k0, klo, khi, g, t, antipodal=anti)
    torch.cuda.synchronize()
    Gg = G.cpu().numpy().astype(np.float64)
    gh, th = g.cpu().numpy().astype(np.float64), t.cpu().numpy()
    npix = gh.shape[1]
    sel = np.arange(npix) if npix <= 200 else np.sort(np.random.default_rng(4).choice(npix, 40, replace=False))
    Go = _oracle(oracle_mod, w, H, df, k0, klo, khi, gh, th, sel)
    S = _scale(w, H, klo, khi, gh[:, sel])
    assert np.max(np.abs(Gg[np.ix_(sel, sel)] - Go) / S) <= 1e-5
    assert np.array_equal(Gg, Gg.T)  # both triangles written from one value
    if anti:
        _, am = sg.healpix_centres(nside)
        am = am.cpu().numpy().astype(np.int64)
        assert np.array_equal(Gg[np.ix_(am, am)], Gg)  # G(a(p), a(q)) = G(p, q)


def test_fisher_full_general_full_day(sg, oracle_mod):
    """A whole day (898 segments) at the top of the band (1.67-1.68 kHz; the
    baseline's 10 ms delays reach 2.15e3 of the 9.1e3 table intervals, streamed
    double-buffered), nside 16 with the antipodal blocks; sampled pixels (with
    their antipodes) against the oracle."""
    nt, nside, k0, nf, df = 898, 16, 52900, 512, 1 / 32
    g, t, w, H = _inputs(sg, "AB", nside, None, nt, k0, nf, df, 42)
    wd, Hd = torch.from_numpy(w).cuda(), torch.from_numpy(H).cuda()
    G = sg.fisher_full_general(wd, Hd, sg.FGrid(F0, df), k0, 0, nf, g, t, antipodal=True)
    _, am = sg.healpix_centres(nside)
    torch.cuda.synchronize()
    Gg = G.cpu().numpy().astype(np.float64)
    gh, th = g.cpu().numpy().astype(np.float64), t.cpu().numpy()
    am = am.cpu().numpy().astype(np.int64)
    base = np.random.default_rng(7).choice(gh.shape[1], 12, replace=False)
    sel = np.unique(np.concatenate([base, am[base]]))
    Go = _oracle(oracle_mod, w, H, df, k0, 0, nf, gh, th, sel)
    S = _scale(w, H, 0, nf, gh[:, sel])
    assert np.max(np.abs(Gg[np.ix_(sel, sel)] - Go) / S) <= 1e-5
    assert np.array_equal(Gg, Gg.T)
    assert np.array_equal(Gg[np.ix_(am, am)], Gg)


def test_fisher_full_general_lds_and_global_forms_agree_bitwise(sg, monkeypatch):
    """The streaming LDS form (double-buffered tables for AC at 1 kHz, one buffer
    for AD at 1.68 kHz) and the global-memory form add the same float32 terms in
    the same segment order: the same bits."""
    for bl, k0, df in (("AC", 4000, 0.25), ("AD", 53000, 1 / 32)):
        nt, nside, nf = 40, 4, 64
        g, t, w, H = _inputs(sg, bl, nside, None, nt, k0, nf, df, 43)
        wd, Hd = torch.from_numpy(w).cuda(), torch.from_numpy(H).cuda()
        for anti in (False, True):
            G1 = sg.fisher_full_general(wd, Hd, sg.FGrid(F0, df), k0, 2, nf, g, t, antipodal=anti)
            monkeypatch.setenv("SGWB_FISHER_TABLE", "global")
            G2 = sg.fisher_full_general(wd, Hd, sg.FGrid(F0, df), k0, 2, nf, g, t, antipodal=anti)
            monkeypatch.delenv("SGWB_FISHER_TABLE")
            torch.cuda.synchronize()
            assert torch.equal(G1, G2)


@pytest.mark.parametrize("k0,df", [(4000, 0.25), (53000, 1 / 32), (39000, 0.125)],
                         ids=["direct-bins", "expanded-S64", "expanded-S16"])
def test_fisher_full_general_equals_separable_path_for_rank_one(sg, k0, df):
    """w = a(t) b(c): the general path (a folded into each segment's table; its
    band sum over the bins at 1/4 Hz, over 64- or 16-bin strip moments at 1/32
    and 1/8 Hz) and sgwb_fisher_full (one table, a applied per term) agree to
    float32 rounding (1e-6 of S)."""
    nt, nside, nf = 40, 4, 64
    g, t, _, H = _inputs(sg, "AB", nside, None, nt, k0, nf, df, 44)
    f = freqs(F0, df, k0, nf)
    a = synth.segment_scale(nt, 45).astype(np.float32)
    b = (synth.spectrum_H(f) / synth.noise_psd(f) ** 2).astype(np.float32)
    w = np.outer(a, b).astype(np.float32)
    ad, bd, Hd, wd = (torch.from_numpy(x).cuda() for x in (a, b, H, w))
    for anti in (False, True):
        Gs = sg.fisher_full(ad, bd, Hd, sg.FGrid(F0, df), k0, 3, 60, g, t, antipodal=anti)
        Gw = sg.fisher_full_general(wd, Hd, sg.FGrid(F0, df), k0, 3, 60, g, t, antipodal=anti)
        torch.cuda.synchronize()
        S = _scale(np.outer(a.astype(np.float64), b.astype(np.float64)), H, 3, 60,
                   g.cpu().numpy().astype(np.float64))
        diff = np.abs(Gs.double().cpu().numpy() - Gw.double().cpu().numpy())
        assert np.max(diff / S) <= 1e-6


def test_fisher_full_general_padded_rows_and_determinism(sg):
    """w with padded rows (row stride > nf) gives the same bits as contiguous w,
    and a second call gives the same bits (fixed summation orders)."""
    nt, nside, k0, nf, df = 36, 8, 500, 300, 1 / 32
    g, t, w, H = _inputs(sg, "AC", nside, None, nt, k0, nf, df, 46)
    wd, Hd = torch.from_numpy(w).cuda(), torch.from_numpy(H).cuda()
    wide = torch.zeros((nt, nf + 13), dtype=torch.float32, device="cuda")
    wide[:, :nf] = wd
    G1 = sg.fisher_full_general(wd, Hd, sg.FGrid(F0, df), k0, 0, nf, g, t)
    G2 = sg.fisher_full_general(wide[:, :nf], Hd, sg.FGrid(F0, df), k0, 0, nf, g, t)
    G3 = sg.fisher_full_general(wd, Hd, sg.FGrid(F0, df), k0, 0, nf, g, t)
    torch.cuda.synchronize()
    assert torch.equal(G1, G2)
    assert torch.equal(G1, G3)


def test_fisher_full_general_diagonal_is_the_band_summed_diagonal(sg):
    """diag G = Gbb of the per-bin diagonal Gam for the same general w, reduced
    over the band (Eq. eq_fisher at p = p')."""
    nt, nside, k0, nf, df, klo, khi = 48, 8, 200, 96, 1 / 32, 7, 90
    g, t, w, H = _inputs(sg, "AB", nside, None, nt, k0, nf, df, 47)
    wd, Hd = torch.from_numpy(w).cuda(), torch.from_numpy(H).cuda()
    G = sg.fisher_full_general(wd, Hd, sg.FGrid(F0, df), k0, klo, khi, g, t)
    C = torch.zeros((nt, nf), dtype=torch.complex64, device="cuda")
    _, Gk = sg.make_maps(C, wd, sg.FGrid(F0, df), k0, g, t, antipodal=False)
    _, Gbb = sg.reduce_band(None, Gk, Hd, klo, khi)
    torch.cuda.synchronize()
    d = torch.diagonal(G).double().cpu().numpy()
    ref = Gbb.double().cpu().numpy()
    assert np.max(np.abs(d - ref) / ref) <= 1e-4  # split-bf16 beam bound on the per-bin diagonal


def test_fisher_full_general_noise_free_sky_gives_x_equal_g_p(sg):
    """C = K P without noise (Eq. eq_CSD_conv), non-separable weights: the
    broadband dirty map equals the general full Fisher matrix times the sky."""
    nt, nside, k0, nf, df = 40, 4, 100, 64, 0.25
    g, t, w, H = _inputs(sg, "AC", nside, None, nt, k0, nf, df, 48)
    npix = g.shape[1]
    f = freqs(F0, df, k0, nf)
    gh, th = g.cpu().numpy().astype(np.float64), t.cpu().numpy()
    rng = np.random.default_rng(9)
    P = np.zeros(npix)
    P[rng.choice(npix, 4, replace=False)] = rng.uniform(0.5, 2.0, 4)
    C = np.zeros((nt, nf), dtype=np.complex128)
    for p in np.nonzero(P)[0]:
        synth.add_point_source(C, f, P[p], gh[:, p], th[:, p])
    wd, Hd = torch.from_numpy(w).cuda(), torch.from_numpy(H).cuda()
    Cd = torch.from_numpy(C.astype(np.complex64)).cuda()
    X, Gk = sg.make_maps(Cd, wd, sg.FGrid(F0, df), k0, g, t, antipodal=False)
    Xbb, _ = sg.reduce_band(X, Gk, Hd, 0, nf)
    G = sg.fisher_full_general(wd, Hd, sg.FGrid(F0, df), k0, 0, nf, g, t)
    torch.cuda.synchronize()
    lhs = Xbb.double().cpu().numpy()
    rhs = G.double().cpu().numpy() @ P
    assert np.max(np.abs(lhs - rhs)) <= 1e-4 * np.max(np.abs(lhs))


def test_fisher_full_general_rejects_broken_seeds(sg):
    """Antipodal flag with a delay changed at one pixel of the middle segment:
    the device check rejects the seeds and the matrix is NaN (the streaming
    form skips every segment and writes NaN)."""
    nt, nside, k0, nf, df = 20, 4, 4000, 32, 0.25
    g, t, w, H = _inputs(sg, "AB", nside, None, nt, k0, nf, df, 49)
    t = t.clone()
    t[nt // 2, 3] += 1e-7
    wd, Hd = torch.from_numpy(w).cuda(), torch.from_numpy(H).cuda()
    G = sg.fisher_full_general(wd, Hd, sg.FGrid(F0, df), k0, 0, nf, g, t, antipodal=True)
    torch.cuda.synchronize()
    assert bool(torch.isnan(G).all())


@pytest.mark.parametrize("weights", ["separable", "general"])
def test_fisher_full_nside64_sampled(sg, oracle_mod, weights):
    """nside 64 (49 152 pixels: G has 2.4e9 entries, past 2^31, so the entry
    offsets must be 64-bit), a whole 898-segment day, 256 bins at the top of the
    band, antipodal blocks: sampled rows and columns (with their antipodes)
    against the oracle, for the separable and the general entry point."""
    nt, nside, k0, nf, df = 898, 64, 54336, 256, 1 / 32
    g, t, w, H = _inputs(sg, "AB", nside, None, nt, k0, nf, df, 50)
    Hd = torch.from_numpy(H).cuda()
    if weights == "general":
        G = sg.fisher_full_general(torch.from_numpy(w).cuda(), Hd, sg.FGrid(F0, df), k0, 0, nf, g, t, antipodal=True)
    else:
        f = freqs(F0, df, k0, nf)
        a = synth.segment_scale(nt, 51).astype(np.float32)
        b = (synth.spectrum_H(f) / synth.noise_psd(f) ** 2).astype(np.float32)
        w = np.outer(a, b).astype(np.float32)
        G = sg.fisher_full(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda(), Hd, sg.FGrid(F0, df), k0, 0, nf,
                           g, t, antipodal=True)
    _, am = sg.healpix_centres(nside)
    torch.cuda.synchronize()
    am = am.cpu().numpy().astype(np.int64)
    npix = 12 * nside * nside
    base = np.concatenate([np.random.default_rng(8).choice(npix, 10, replace=False), [0, npix // 2 - 1, npix - 1]])
    sel = np.unique(np.concatenate([base, am[base]]))
    idx = torch.from_numpy(sel).cuda()
    Gs = G.index_select(0, idx).index_select(1, idx).double().cpu().numpy()
    gh, th = g.cpu().numpy().astype(np.float64), t.cpu().numpy()
    Go = _oracle(oracle_mod, w, H, df, k0, 0, nf, gh, th, sel)
    S = _scale(w, H, 0, nf, gh[:, sel])
    assert np.max(np.abs(Gs - Go) / S) <= 1e-5
    # the far corner of the matrix (row and column past 2^31 entries) is the mirror of its transpose
    assert torch.equal(G[npix - 1, :64], G[:64, npix - 1])
    del G
    torch.cuda.empty_cache()
