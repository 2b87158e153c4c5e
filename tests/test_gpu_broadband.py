"""Broadband maps alone through sgwb_broadband_maps.  The delay-table route sums
each segment's band first (Y_t tabulated on a delay grid, 4-point Lagrange
interpolation, float64 carrier phase): its Xbb meets the FP64 oracle's band sum
of the narrowband dirty map within 1e-6 of the band-summed scale
S_bb(p) = sum_k sum_t |w gamma C| (interpolation below 1.9e-8, float32 tables
and phasors ~1e-7).  Its Gbb is the fused call's, bit for bit.  The strips route
is bitwise the broadband-only make_maps_band call."""
import numpy as np
import pytest

import synth
from tests._cases import freqs, make_csd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F0 = 20.0
TOL = 1e-6

CASES = [  # baseline, nside, nt, k0, nf, band, df, antipodal
    ("AB", 8, 60, 0, 640, (0, 640), 1 / 32, True),       # whole call
    ("AC", 8, 61, 37, 203, (5, 190), 1 / 32, True),      # band inside both ends
    ("BC", 4, 33, 64 * 9 + 63, 130, (64, 65), 1 / 32, True),  # one bin: Y_t constant
    ("AB", 4, 30, 11, 40, (3, 5), 1 / 32, True),         # two bins
    ("AC", 8, 40, 10, 300, (17, 299), 0.25, True),       # coarse grid: no matrix-core form exists
    ("BC", 4, 30, 3, 100, (1, 99), 1 / 32, False),       # no antipodal pairing
    ("AD", 4, 25, 0, 257, (0, 257), 1 / 32, True),       # longest baseline, odd band
]


@pytest.fixture(scope="module")
def sg():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1803_08285_amd as sg

    return sg


def _setup(sg, bl, nside, nt, k0, nf, df, seed):
    tg = sg.TGrid(nt, 0.0, 86164.0905 / nt, 86164.0905 / nt)
    g, t = sg.build_geometry(synth.baseline_sites(bl), nside, tg)
    f = freqs(F0, df, k0, nf)
    C, w = make_csd(seed, nt, f)
    H = synth.spectrum_H(f).astype(np.float32)
    return g, t, torch.from_numpy(C).cuda(), torch.from_numpy(w).cuda(), torch.from_numpy(H).cuda()


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{c[1]}-{c[3]}-{c[5]}-{c[6]}-{c[7]}" for c in CASES])
def test_table_route_vs_oracle(sg, oracle_mod, case):
    bl, nside, nt, k0, nf, (klo, khi), df, anti = case
    g, t, C, w, H = _setup(sg, bl, nside, nt, k0, nf, df, 90 + nside)
    fg = sg.FGrid(F0, df)
    tb = sg.baseline_delay_bound(synth.baseline_sites(bl))
    print(f"case {case}", flush=True)
    Xbb, Gbb = sg.broadband_maps(C, w, fg, k0, g, t, H, klo, khi, tau_bound=tb, antipodal=anti, route="table")
    torch.cuda.synchronize()
    assert sg.last_x_form() == "table"
    Xo, _, S = oracle_mod.maps(C.cpu().numpy(), w.cpu().numpy(), F0, df, k0, g.cpu().numpy(), t.cpu().numpy(),
                               with_scale=True)
    Sb = S[klo:khi].sum(axis=0)
    err = np.abs(Xbb.cpu().numpy().astype(np.float64) - Xo[klo:khi].sum(axis=0))
    assert np.all(np.isfinite(err))
    assert np.all(err <= TOL * Sb + 1e-300), float((err / Sb).max())
    # Gbb: the same weight-side kernel as the fused call
    _, _, _, Gref = sg.make_maps_band(C, w, fg, k0, g, t, H, klo, khi, antipodal=anti, want_x=False,
                                      narrowband=False)
    torch.cuda.synchronize()
    assert torch.equal(Gbb, Gref)


def test_the_earth_bound_and_a_tight_bound_agree(sg, oracle_mod):
    """tau_bound = 0 (2R/c, a larger grid) and the baseline's own bound give
    the same maps to the stated tolerance; reruns are bitwise equal."""
    g, t, C, w, H = _setup(sg, "AB", 8, 50, 70, 400, 1 / 32, 9)
    fg = sg.FGrid(F0, 1 / 32)
    tb = sg.baseline_delay_bound(synth.baseline_sites("AB"))
    X1, _ = sg.broadband_maps(C, w, fg, 70, g, t, None, 3, 390, tau_bound=tb, want_gamma=False, route="table")
    X2, _ = sg.broadband_maps(C, w, fg, 70, g, t, None, 3, 390, tau_bound=0.0, want_gamma=False, route="table")
    X3, _ = sg.broadband_maps(C, w, fg, 70, g, t, None, 3, 390, tau_bound=tb, want_gamma=False, route="table")
    torch.cuda.synchronize()
    assert torch.equal(X1, X3)
    _, _, S = oracle_mod.maps(C.cpu().numpy(), w.cpu().numpy(), F0, 1 / 32, 70, g.cpu().numpy(), t.cpu().numpy(),
                              with_scale=True)
    Sb = S[3:390].sum(axis=0)
    assert np.all(np.abs(X1.cpu().numpy().astype(np.float64) - X2.cpu().numpy()) <= 2 * TOL * Sb)


def test_strips_route_is_the_broadband_only_band_call(sg, monkeypatch):
    g, t, C, w, H = _setup(sg, "AC", 8, 61, 37, 203, 1 / 32, 5)
    fg = sg.FGrid(F0, 1 / 32)
    Xbb, Gbb = sg.broadband_maps(C, w, fg, 37, g, t, H, 5, 190, route="strips")
    form = sg.last_x_form()
    _, _, Xr, Gr = sg.make_maps_band(C, w, fg, 37, g, t, H, 5, 190, narrowband=False)
    torch.cuda.synchronize()
    assert form.startswith("mfma")
    assert torch.equal(Xbb, Xr) and torch.equal(Gbb, Gr)
    # the cost rule takes the tables for this small day; the environment can set the route
    Xa, _ = sg.broadband_maps(C, w, fg, 37, g, t, None, 5, 190, want_gamma=False)
    assert sg.last_x_form() == "table"
    monkeypatch.setenv("SGWB_BB_ROUTE", "strips")
    Xs, _ = sg.broadband_maps(C, w, fg, 37, g, t, None, 5, 190, want_gamma=False)
    assert sg.last_x_form().startswith("mfma")
    torch.cuda.synchronize()
    assert torch.equal(Xs, Xbb)


def test_seeds_beyond_the_bound_give_nan_at_their_pixels(sg):
    g, t, C, w, H = _setup(sg, "AC", 4, 30, 0, 64, 1 / 32, 7)
    fg = sg.FGrid(F0, 1 / 32)
    tau_np = t.cpu().numpy()
    bound = 0.5 * np.abs(tau_np).max()  # about half the pixels reach past it in some segment
    beyond = (np.abs(tau_np) > bound).any(axis=0)
    assert beyond.any() and not beyond.all()
    Xbb, _ = sg.broadband_maps(C, w, fg, 0, g, t, None, 0, 64, tau_bound=bound, want_gamma=False, route="table")
    torch.cuda.synchronize()
    x = Xbb.cpu().numpy()
    assert np.all(np.isnan(x[beyond])) and np.all(np.isfinite(x[~beyond]))


def test_rejects_bad_arguments(sg):
    g, t, C, w, H = _setup(sg, "AB", 4, 20, 0, 64, 1 / 32, 3)
    fg = sg.FGrid(F0, 1 / 32)
    with pytest.raises(sg.SgwbError, match="band"):
        sg.broadband_maps(C, w, fg, 0, g, t, H, 10, 65)
    with pytest.raises(sg.SgwbError, match="band"):
        sg.broadband_maps(C, w, fg, 0, g, t, H, 10, 10)
    with pytest.raises(sg.SgwbError, match="strips"):
        sg.broadband_maps(C, w, fg, 0, g, t, H, 0, 64, antipodal=False, route="strips")
    with pytest.raises(sg.SgwbError, match="tau_bound"):
        sg.broadband_maps(C, w, fg, 0, g, t, H, 0, 64, tau_bound=-1.0)


def test_full_day_nside128_band4096_sampled(sg, oracle_mod):
    """The served form's largest query: a full day, nside 128, 4096 bins, the
    route the cost rule picks (the tables), sampled pixels against the oracle."""
    tg = synth.TGRID_FULL
    nside, k0, nf = 128, 1000, 4096
    g, t = sg.build_geometry(synth.baseline_sites("AB"), nside, sg.TGrid(tg.nt, tg.t0, tg.stride, tg.dur))
    f = freqs(F0, 1 / 32, k0, nf)
    C, w = make_csd(11, tg.nt, f)
    Cd, wd = torch.from_numpy(C).cuda(), torch.from_numpy(w).cuda()
    fg = sg.FGrid(F0, 1 / 32)
    tb = sg.baseline_delay_bound(synth.baseline_sites("AB"))
    Xbb, _ = sg.broadband_maps(Cd, wd, fg, k0, g, t, None, 0, nf, tau_bound=tb, want_gamma=False)
    torch.cuda.synchronize()
    assert sg.last_x_form() == "table"
    npix = 12 * nside * nside
    pix = np.random.default_rng(3).choice(npix, 6, replace=False)
    gh, th = g.cpu().numpy(), t.cpu().numpy()
    cols = np.tile(np.arange(nf), pix.size)
    pp = np.repeat(pix, nf)
    Xo, _, S = oracle_mod.maps_at(C, w, F0, 1 / 32, k0, gh, th, cols, pp)
    ref = Xo.reshape(pix.size, nf).sum(axis=1)
    Sb = S.reshape(pix.size, nf).sum(axis=1)
    err = np.abs(Xbb.cpu().numpy()[pix].astype(np.float64) - ref)
    assert np.all(err <= TOL * Sb), float((err / Sb).max())


def test_broken_antipodal_promise_gives_nan_maps(sg):
    """With SGWB_MAPS_ANTIPODAL the table route reads each pixel pair's seeds
    once; seeds that fail the antipodal spot check give NaN maps, not wrong ones."""
    g, t, C, w, H = _setup(sg, "AC", 4, 30, 0, 64, 1 / 32, 8)
    fg = sg.FGrid(F0, 1 / 32)
    t2 = t.clone()
    t2[0, 5] += 1e-6  # segment 0 is one the spot check reads
    Xbb, Gbb = sg.broadband_maps(C, w, fg, 0, g, t2, H, 0, 64, route="table")
    Xok, Gok = sg.broadband_maps(C, w, fg, 0, g, t, H, 0, 64, route="table")
    Xnp, Gnp = sg.broadband_maps(C, w, fg, 0, g, t, H, 0, 64, route="table", antipodal=False)
    torch.cuda.synchronize()
    assert torch.isnan(Xbb).all() and torch.isnan(Gbb).all()
    assert torch.isfinite(Xok).all() and torch.equal(Gok, Gnp)
    # the pair pass and the one-pixel pass agree to the route's tolerance
    assert float((Xok - Xnp).abs().max()) <= 1e-6 * float(Xok.abs().max())
