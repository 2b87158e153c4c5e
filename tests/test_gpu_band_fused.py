"""Narrowband and broadband maps in one call (make_maps_band): the narrowband
maps are bitwise those of make_maps; Xbb, taken inside the dirty-map kernel
(float64 per 64-bin strip, one rounding), meets the oracle's band sum of those
maps to the bound of reduce_band (2^-24 relative plus 1e-12 of sum |X|); Gbb,
computed from its definition with the band sum moved into the weights
(sum_t (sum_k H w) gamma^2, float64), meets the oracle's float64 band sum of its
own Fisher diagonal to one float32 rounding, and the band sum of the split-bf16
per-bin diagonal to the beam's 1e-4."""
import numpy as np
import pytest

import synth
from tests._cases import freqs, make_csd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F0 = 20.0
CASES = [  # baseline, nside, nt, k0, nf, band, df, antipodal, x_kernel
    ("AB", 8, 60, 0, 640, (0, 640), 1 / 32, True, "auto"),        # matrix-core dirty map, whole band
    ("AC", 16, 61, 37, 203, (5, 190), 1 / 32, True, "auto"),      # ragged strips, band inside both ends
    ("BC", 4, 33, 64 * 9 + 63, 130, (64, 65), 1 / 32, True, "auto"),  # one-bin band
    ("AB", 8, 40, 10, 300, (17, 299), 0.25, True, "auto"),        # vector-unit dirty map (df too coarse)
    ("AC", 8, 45, 0, 200, (0, 200), 1 / 32, True, "valu"),
    ("BC", 4, 30, 3, 100, (1, 99), 1 / 32, False, "auto"),        # no antipodal pairing
    ("AB", 4, 20, 0, 64, (30, 30), 1 / 32, True, "auto"),         # empty band
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


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{c[1]}-{c[3]}-{c[5]}-{c[6]}-{c[7]}-{c[8]}" for c in CASES])
def test_fused_band_maps(sg, oracle_mod, case):
    bl, nside, nt, k0, nf, (klo, khi), df, anti, xk = case
    g, t, C, w, H = _setup(sg, bl, nside, nt, k0, nf, df, 40 + nside)
    fg = sg.FGrid(F0, df)
    X, G, Xbb, Gbb = sg.make_maps_band(C, w, fg, k0, g, t, H, klo, khi, antipodal=anti, x_kernel=xk)
    Xr, Gr = sg.make_maps(C, w, fg, k0, g, t, antipodal=anti, x_kernel=xk)
    torch.cuda.synchronize()
    assert torch.equal(X, Xr) and torch.equal(G, Gr)
    Xh, Gh, Hh = X.cpu().numpy(), G.cpu().numpy(), H.cpu().numpy()
    Xo, Go_split = oracle_mod.band(Xh, Gh, Hh, klo, khi)
    scale_x = np.abs(Xh[klo:khi]).sum(axis=0) if khi > klo else np.zeros(Xh.shape[1])
    assert np.all(np.abs(Xbb.cpu().numpy() - Xo) <= 2 ** -24 * np.abs(Xo) + 1e-12 * scale_x + 1e-300)
    # Gbb against the oracle's own float64 diagonal, band-summed
    _, Gexact = oracle_mod.maps(np.zeros(w.shape, np.complex128), w.cpu().numpy(), F0, df, k0,
                                g.cpu().numpy(), t.cpu().numpy())
    _, Go = oracle_mod.band(np.zeros_like(Gexact), Gexact, Hh, klo, khi)
    Gg = Gbb.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(Gg - Go) <= 2 ** -24 * np.abs(Go) * 1.01 + 1e-300)
    assert np.all(np.abs(Gg - Go_split) <= 1e-4 * Go + 1e-300)


def test_fused_band_maps_single_outputs_and_determinism(sg):
    """Either pair alone gives the same bits as both together; reruns are bitwise equal."""
    g, t, C, w, H = _setup(sg, "AC", 8, 50, 70, 400, 1 / 32, 9)
    fg = sg.FGrid(F0, 1 / 32)
    X, G, Xbb, Gbb = sg.make_maps_band(C, w, fg, 70, g, t, H, 3, 390)
    X1, _, Xbb1, _ = sg.make_maps_band(C, w, fg, 70, g, t, None, 3, 390, want_gamma=False)
    _, G2, _, Gbb2 = sg.make_maps_band(C, w, fg, 70, g, t, H, 3, 390, want_x=False)
    X3, G3, Xbb3, Gbb3 = sg.make_maps_band(C, w, fg, 70, g, t, H, 3, 390)
    torch.cuda.synchronize()
    assert torch.equal(X, X1) and torch.equal(Xbb, Xbb1)
    assert torch.equal(G, G2) and torch.equal(Gbb, Gbb2)
    assert torch.equal(X, X3) and torch.equal(G, G3) and torch.equal(Xbb, Xbb3) and torch.equal(Gbb, Gbb3)


@pytest.mark.parametrize("case", [c for c in CASES if c[7] and c[6] <= 1 / 32 and c[8] == "auto"],
                         ids=lambda c: f"{c[0]}-{c[1]}-{c[3]}-{c[5]}")
def test_broadband_alone_bitwise_and_vs_oracle(sg, oracle_mod, case):
    """The broadband maps alone (no narrowband map written, no beam GEMM) are
    bitwise those of the call with the narrowband maps, and Xbb meets the FP64
    oracle's band-summed dirty map within 1e-5 of its band-summed scale."""
    bl, nside, nt, k0, nf, (klo, khi), df, anti, xk = case
    g, t, C, w, H = _setup(sg, bl, nside, nt, k0, nf, df, 70 + nside)
    fg = sg.FGrid(F0, df)
    X, G, Xbb, Gbb = sg.make_maps_band(C, w, fg, k0, g, t, H, klo, khi)
    X0, G0, Xbb0, Gbb0 = sg.make_maps_band(C, w, fg, k0, g, t, H, klo, khi, narrowband=False)
    _, _, Xbb1, _ = sg.make_maps_band(C, w, fg, k0, g, t, None, klo, khi, want_gamma=False, narrowband=False)
    _, _, _, Gbb2 = sg.make_maps_band(C, w, fg, k0, g, t, H, klo, khi, want_x=False, narrowband=False)
    torch.cuda.synchronize()
    assert X0 is None and G0 is None
    assert torch.equal(Xbb, Xbb0) and torch.equal(Gbb, Gbb0)
    assert torch.equal(Xbb, Xbb1) and torch.equal(Gbb, Gbb2)
    Xo, _, S = oracle_mod.maps(C.cpu().numpy(), w.cpu().numpy(), F0, df, k0, g.cpu().numpy(), t.cpu().numpy(),
                               with_scale=True)
    Sb = S[klo:khi].sum(axis=0)
    err = np.abs(Xbb0.cpu().numpy().astype(np.float64) - Xo[klo:khi].sum(axis=0))
    assert np.all(err <= 1e-5 * Sb + 1e-300)


def test_broadband_alone_needs_the_matrix_core_form(sg):
    g, t, C, w, H = _setup(sg, "AB", 4, 20, 0, 64, 1 / 32, 3)
    fg = sg.FGrid(F0, 1 / 32)
    with pytest.raises(sg.SgwbError, match="matrix-core"):
        sg.make_maps_band(C, w, fg, 0, g, t, H, 0, 64, x_kernel="valu", narrowband=False)
    with pytest.raises(sg.SgwbError, match="matrix-core"):
        sg.make_maps_band(C, w, fg, 0, g, t, H, 0, 64, antipodal=False, narrowband=False)
    # the beam's broadband map alone needs no particular form
    _, _, _, Gbb = sg.make_maps_band(C, w, fg, 0, g, t, H, 0, 64, antipodal=False, want_x=False, narrowband=False)
    _, _, _, Gref = sg.make_maps_band(C, w, fg, 0, g, t, H, 0, 64, antipodal=False, want_x=False)
    torch.cuda.synchronize()
    assert torch.equal(Gbb, Gref)


def test_fused_band_maps_rejects_bad_arguments(sg):
    g, t, C, w, H = _setup(sg, "AB", 4, 20, 0, 64, 1 / 32, 3)
    fg = sg.FGrid(F0, 1 / 32)
    with pytest.raises(sg.SgwbError, match="band"):
        sg.make_maps_band(C, w, fg, 0, g, t, H, 10, 65)
    with pytest.raises(sg.SgwbError, match="H"):
        sg.make_maps_band(C, w, fg, 0, g, t, None, 0, 64)
