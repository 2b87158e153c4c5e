"""Every form of the dirty map that the product can take, against the FP64
oracle through the C ABI, with the form that ran read back from the library
(sgwb_last_x_form).  The matrix-core forms follow the largest delay of the
seeds, eta = 2 pi 31.5 df max|tau|: four terms up to 0.07, five with m = 2
unsplit up to 0.17, five with m = 2 split up to 0.29; beyond that the
vector-unit recurrence runs.  Tolerances as everywhere: X within 1e-5 of
S = sum_t |w gamma||C| (Eq. eq_dirtymap split per bin, Eq. eq:narrowband),
Gam within 1e-4 elementwise (Eq. eq_fisher, p = p').  Also: seeds that break
the antipodal promise are refused on the device (NaN maps, an error on read
back), and the overlap-corrected Fisher diagonal of a short day on a long
baseline (pair delays beyond every matrix-core form) takes the vector units."""
import numpy as np
import pytest

import synth
from tests._cases import freqs, g_error, make_csd, x_error

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

X_TOL = 1e-5
G_TOL = 1e-4
F0 = 20.0


@pytest.fixture(scope="module")
def sg():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1803_08285_amd as sg

    return sg


def _geom(sg, bl, nside, nt):
    tg = sg.TGrid(nt, 0.0, 86164.0905 / nt, 86164.0905 / nt)
    g, t = sg.build_geometry(synth.baseline_sites(bl), nside, tg)
    torch.cuda.synchronize()
    return g, t


def _eta(df, t):
    return 2 * np.pi * 31.5 * df * float(t.abs().max())


# baseline, df, expected form, nside, nt, k0, nf
FORM_CASES = [
    ("AB", 1 / 32, "mfma4", 16, 61, 37, 203),
    ("AC", 1 / 32, "mfma5", 16, 61, 37, 203),
    ("AC", 1 / 30, "mfma5_split", 16, 61, 37, 203),   # AC at 1/30 Hz: eta 0.18
    ("AD", 1 / 32, "mfma5_split", 16, 45, 64 * 7 + 5, 190),  # long baseline: eta 0.24
    ("AD", 1 / 32, "mfma5_split", 4, 17, 63, 66),     # one bin short of a strip start, short day
    ("AD", 1 / 29.1, "mfma5_split", 8, 33, 0, 128),   # df just inside the Earth bound: eta 0.27
    ("AD", 0.25, "valu", 8, 33, 0, 128),              # df beyond the matrix-core forms
]


@pytest.mark.parametrize("case", FORM_CASES, ids=[f"{c[0]}-{c[1]:.4f}-{c[2]}-{c[3]}" for c in FORM_CASES])
def test_each_form_vs_oracle(sg, oracle_mod, case):
    bl, df, form, nside, nt, k0, nf = case
    g, t = _geom(sg, bl, nside, nt)
    eta = _eta(df, t)
    f = freqs(F0, df, k0, nf)
    C, w = make_csd(300 + nside, nt, f)
    X, G = sg.make_maps(torch.from_numpy(C).cuda(), torch.from_numpy(w).cuda(), sg.FGrid(F0, df), k0, g, t)
    ran = sg.last_x_form()
    print(f"{bl} df {df:.5f}: eta {eta:.4f}, form {ran}")
    assert ran == form
    Xo, Go, S = oracle_mod.maps(C, w, F0, df, k0, g.cpu().numpy(), t.cpu().numpy(), with_scale=True)
    ex, eg = x_error(X.cpu().numpy(), Xo, S), g_error(G.cpu().numpy(), Go)
    print(f"X err {ex:.3e}  Gam err {eg:.3e}")
    assert ex <= X_TOL
    assert eg <= G_TOL


def test_split_form_band_maps_vs_oracle(sg, oracle_mod):
    """make_maps_band on the split form: the per-strip sums of the dirty map give
    Xbb within 1e-5 of sum_k S (and within a float32 rounding of the oracle's
    band sum of the GPU's own rows)."""
    nside, nt, k0, nf, df, klo, khi = 16, 45, 64 * 3 + 20, 300, 1 / 32, 11, 290
    g, t = _geom(sg, "AD", nside, nt)
    f = freqs(F0, df, k0, nf)
    C, w = make_csd(77, nt, f)
    H = synth.spectrum_H(f).astype(np.float32)
    X, G, Xbb, Gbb = sg.make_maps_band(torch.from_numpy(C).cuda(), torch.from_numpy(w).cuda(), sg.FGrid(F0, df), k0,
                                       g, t, torch.from_numpy(H).cuda(), klo, khi)
    assert sg.last_x_form() == "mfma5_split"
    Xo, Go, S = oracle_mod.maps(C, w, F0, df, k0, g.cpu().numpy(), t.cpu().numpy(), with_scale=True)
    Xbo, Gbo = oracle_mod.band(Xo, Go, H, klo, khi)
    Sb = S[klo:khi].sum(axis=0)
    assert np.max(np.abs(Xbb.cpu().numpy() - Xbo) / Sb) <= X_TOL
    assert np.max(np.abs(Gbb.cpu().numpy() - Gbo) / Gbo) <= 1e-6
    Xh = X.cpu().numpy()
    Xself, _ = oracle_mod.band(Xh, Go, H, klo, khi)
    scale = np.abs(Xh[klo:khi]).sum(axis=0)
    assert np.all(np.abs(Xbb.cpu().numpy() - Xself) <= 2 ** -24 * np.abs(Xself) + 1e-12 * scale)


def test_broken_antipodal_promise_is_refused(sg):
    """Seeds whose antipodal symmetry is broken (one delay changed) under the
    antipodal flag: the device check rejects them, X is NaN and reading the form
    back raises; the same seeds without the flag give a finite map."""
    nside, nt, nf, df = 8, 40, 128, 1 / 32
    g, t = _geom(sg, "AB", nside, nt)
    t = t.clone()
    t[nt // 2, 5] += 1e-6
    f = freqs(F0, df, 0, nf)
    C, w = make_csd(5, nt, f)
    Cd, wd = torch.from_numpy(C).cuda(), torch.from_numpy(w).cuda()
    X, _ = sg.make_maps(Cd, wd, sg.FGrid(F0, df), 0, g, t, want_gamma=False, workspace=sg.make_workspace(nt, nf, 768))
    with pytest.raises(sg.SgwbError, match="antipodal"):
        sg.last_x_form()
    assert bool(torch.isnan(X).all())
    X2, _ = sg.make_maps(Cd, wd, sg.FGrid(F0, df), 0, g, t, antipodal=False, want_gamma=False)
    assert sg.last_x_form() == "valu"
    assert bool(torch.isfinite(X2).all())


def test_short_workspace_is_an_error_not_a_fallback(sg):
    """A workspace that holds the beam but not the matrix-core dirty map's
    operands is refused (SGWB_ENOMEM), not silently served by the vector units."""
    nside, nt, nf, df = 8, 40, 128, 1 / 32
    g, t = _geom(sg, "AB", nside, nt)
    f = freqs(F0, df, 0, nf)
    C, w = make_csd(6, nt, f)
    need = sg.workspace_bytes(nt, nf, 768, True)
    short = torch.empty(need // 4, dtype=torch.uint8, device="cuda")
    with pytest.raises(sg.SgwbError, match="matrix-core"):
        sg.make_maps(torch.from_numpy(C).cuda(), torch.from_numpy(w).cuda(), sg.FGrid(F0, df), 0, g, t,
                     want_gamma=False, workspace=short)
    assert sg.last_x_form() == "none"


@pytest.mark.parametrize("nt", [2, 3, 5])
def test_overlap_fisher_short_day_long_baseline(sg, oracle_mod, nt):
    """Pair delays tau(t+1) - tau(t) of a day of nt segments on the long baseline
    reach far beyond the matrix-core bound at 1/32 Hz: the vector-unit kernel,
    gated on the device's form record, computes the neighbour terms."""
    nside, k0, nf, df = 8, 40, 150, 1 / 32
    tg = sg.TGrid(nt, 0.0, 86164.0905 / nt, 2 * 86164.0905 / nt)
    g, t = sg.build_geometry(synth.baseline_sites("AD"), nside, tg)
    rng = np.random.default_rng(nt)
    f = freqs(F0, df, k0, nf)
    v = (rng.uniform(0.5, 1.5, (nt, 1)) * (synth.spectrum_H(f) / synth.noise_psd(f) ** 2)).astype(np.float32)
    u, w = synth.overlap_series(v.astype(np.float64))
    u[0] = 0.5 * synth.HANN_OVERLAP_W * (v[0] + v[-1])
    w[-1] = u[0]
    u, w = u.astype(np.float32), w.astype(np.float32)
    G = sg.fisher_overlap(*(torch.from_numpy(a).cuda() for a in (v, u, w)), sg.FGrid(F0, df), k0, g, t)
    th = t.cpu().numpy()
    eta_pairs = 2 * np.pi * 31.5 * df * np.abs(np.roll(th, -1, axis=0) - th).max()
    form = sg.last_x_form()
    print(f"nt {nt}: pair eta {eta_pairs:.3f}, form {form}")
    assert form == ("valu" if eta_pairs > 0.29 else "mfma5_split" if eta_pairs > 0.17 else form)
    npix = 12 * nside * nside
    cols = np.repeat(np.arange(nf), npix)
    pix = np.tile(np.arange(npix), nf)
    Go, _, S = oracle_mod.fisher_overlap_at(v, u, w, F0, df, k0, g.cpu().numpy(), th, cols, pix)
    err = np.abs(G.cpu().numpy().reshape(-1).astype(np.float64) - Go) / S
    assert err.max() <= G_TOL


def test_nside128_served_band_sampled(sg, oracle_mod):
    """nside 128 (196608 pixels), the largest served resolution, with the largest
    served band (4096 bins) of the full-day time grid, in the launch
    configuration the server uses (make_maps_band); sampled rows and columns
    against the oracle."""
    tg = synth.TGRID_FULL
    nside, nf, k0, df = 128, 4096, 20000, 1 / 32
    g, t = sg.build_geometry(synth.baseline_sites("AC"), nside, sg.TGrid(tg.nt, tg.t0, tg.stride, tg.dur))
    f = freqs(F0, df, k0, nf)
    C, w = make_csd(128, tg.nt, f)
    H = synth.spectrum_H(f).astype(np.float32)
    X, G, Xbb, Gbb = sg.make_maps_band(torch.from_numpy(C).cuda(), torch.from_numpy(w).cuda(), sg.FGrid(F0, df), k0,
                                       g, t, torch.from_numpy(H).cuda(), 0, nf)
    assert sg.last_x_form() == "mfma5"
    npix = 12 * nside * nside
    rows, cols = synth.random_selection(128, nf, npix, 2, 3)
    ri, ci = torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()
    Xs, Gs = X[ri, ci].cpu().numpy(), G[ri, ci].cpu().numpy()
    gh, th = g.cpu().numpy(), t.cpu().numpy()
    Xo, Go, S = oracle_mod.maps_at(C, w, F0, df, k0, gh, th, rows, cols)
    ex, eg = x_error(Xs, Xo, S), g_error(Gs, Go)
    print(f"nside 128: X err {ex:.3e}  Gam err {eg:.3e}  ({rows.size} samples)")
    assert ex <= X_TOL
    assert eg <= G_TOL
    assert bool((G >= 0).all())
    # broadband maps: each pixel's band sums against the oracle's, on a pixel sample
    pix = np.sort(np.random.default_rng(1).choice(npix, 24, replace=False))
    cc = np.repeat(np.arange(nf), pix.size)
    pp = np.tile(pix, nf)
    Xo2, Go2, S2 = oracle_mod.maps_at(C, w, F0, df, k0, gh, th, cc, pp)
    Xbo = Xo2.reshape(nf, pix.size).sum(axis=0)
    Gbo = (H.astype(np.float64)[:, None] * Go2.reshape(nf, pix.size)).sum(axis=0)
    Sb = S2.reshape(nf, pix.size).sum(axis=0)
    assert np.max(np.abs(Xbb.cpu().numpy()[pix] - Xbo) / Sb) <= X_TOL
    assert np.max(np.abs(Gbb.cpu().numpy()[pix] - Gbo) / Gbo) <= 1e-6
