"""Overlap-corrected Fisher diagonal (Sec. II.B, Eq. fwGamma with p = p') on the
GPU against the FP64 oracle, through the C ABI.

Tolerances: the v term is the split-bf16 beam (<= 1e-4 of the plain diagonal,
elementwise); the neighbour terms are a dirty-map-shaped sum and meet the
dirty-map bound, max |dG| / S_nb <= 1e-5, S_nb = sum over pairs of
|u + w| |gamma gamma'|, checked on the difference against the plain diagonal of
the same call path (one float32 rounding of the sum allowed for)."""
import numpy as np
import pytest

import synth
from tests._cases import freqs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F0 = 20.0
CASES = [  # baseline, nside, nt, k0, nf, df, antipodal, x_kernel
    ("AB", 8, 60, 0, 200, 1 / 32, True, "auto"),
    ("AC", 16, 45, 77, 130, 1 / 32, True, "auto"),
    ("BC", 8, 50, 5, 96, 0.25, True, "auto"),
    ("AB", 4, 33, 64, 70, 1 / 32, True, "valu"),
    ("AC", 4, 40, 3, 50, 1 / 32, False, "auto"),
    # segments of a full-resolution day: pair delays so small (eta <= 1e-3)
    # that the expansion's higher terms nearly vanish
    ("AB", 4, 898, 0, 64, 1 / 32, True, "auto"),
    ("BC", 2, 1200, 100, 70, 1 / 32, True, "auto"),
]


@pytest.fixture(scope="module")
def sg():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1803_08285_amd as sg

    return sg


def _inputs(sg, bl, nside, nt, k0, nf, df, seed):
    tg = sg.TGrid(nt, 0.0, 86164.0905 / nt, 2 * 86164.0905 / nt)
    g, t = sg.build_geometry(synth.baseline_sites(bl), nside, tg)
    rng = np.random.default_rng(seed)
    f = freqs(F0, df, k0, nf)
    v = (rng.uniform(0.5, 1.5, (nt, 1)) * (synth.spectrum_H(f) / synth.noise_psd(f) ** 2)).astype(np.float32)
    u, w = synth.overlap_series(v.astype(np.float64))
    # pairs across the day boundary, as in folded data of several days
    u[0] = 0.5 * synth.HANN_OVERLAP_W * (v[0] + v[-1])
    w[-1] = u[0]
    return g, t, v, u.astype(np.float32), w.astype(np.float32)


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}-{c[1]}-{c[5]}-{c[6]}-{c[7]}" for c in CASES])
def test_overlap_fisher_vs_oracle(sg, oracle_mod, case):
    bl, nside, nt, k0, nf, df, anti, xk = case
    g, t, v, u, w = _inputs(sg, bl, nside, nt, k0, nf, df, 11)
    vd, ud, wd = (torch.from_numpy(a).cuda() for a in (v, u, w))
    G = sg.fisher_overlap(vd, ud, wd, sg.FGrid(F0, df), k0, g, t, antipodal=anti, x_kernel=xk)
    # plain diagonal of the same call path (no neighbours): the v term alone
    z = torch.zeros_like(vd)
    G0 = sg.fisher_overlap(vd, z, z, sg.FGrid(F0, df), k0, g, t, antipodal=anti, x_kernel=xk)
    torch.cuda.synchronize()
    npix = 12 * nside * nside
    rows, cols = synth.random_selection(3, nf, npix, 4, 6)
    gh, th = g.cpu().numpy(), t.cpu().numpy()
    if nt >= 898:  # the case is there for tiny pair delays: check that they are
        dtau = np.abs(np.roll(th, -1, axis=0) - th).max()
        assert 2 * np.pi * 31.5 * df * dtau <= 1e-3
    Go, _, S = oracle_mod.fisher_overlap_at(v, u, w, F0, df, k0, gh, th, rows, cols)
    zh = np.zeros_like(v)
    Go0, _, _ = oracle_mod.fisher_overlap_at(v, zh, zh, F0, df, k0, gh, th, rows, cols)
    Gg = G.cpu().numpy()[rows, cols].astype(np.float64)
    Gg0 = G0.cpu().numpy()[rows, cols].astype(np.float64)
    # whole value: v term within the beam bound
    assert np.max(np.abs(Gg - Go) / S) <= 1e-4
    # neighbour terms alone
    S_nb = S - np.abs(Go0)
    err_nb = np.abs((Gg - Gg0) - (Go - Go0)) / S_nb
    round_once = 2.0 ** -23 * np.abs(Gg) / S_nb
    assert np.max(err_nb - round_once) <= 1e-5


def test_no_neighbours_is_bitwise_the_plain_diagonal(sg):
    g, t, v, u, w = _inputs(sg, "AB", 8, 48, 13, 150, 1 / 32, 12)
    vd = torch.from_numpy(v).cuda()
    z = torch.zeros_like(vd)
    G = sg.fisher_overlap(vd, z, z, sg.FGrid(F0, 1 / 32), 13, g, t)
    C = torch.zeros(vd.shape, dtype=torch.complex64, device="cuda")
    _, Gp = sg.make_maps(C, vd, sg.FGrid(F0, 1 / 32), 13, g, t, want_x=False)
    torch.cuda.synchronize()
    assert torch.equal(G, Gp)


def test_overlap_fisher_deterministic_and_single_segment(sg):
    g, t, v, u, w = _inputs(sg, "BC", 8, 40, 0, 128, 1 / 32, 13)
    u[0] = 0.0
    w[-1] = 0.0
    vd, ud, wd = (torch.from_numpy(a).cuda() for a in (v, u, w))
    A = sg.fisher_overlap(vd, ud, wd, sg.FGrid(F0, 1 / 32), 0, g, t)
    B = sg.fisher_overlap(vd, ud, wd, sg.FGrid(F0, 1 / 32), 0, g, t)
    torch.cuda.synchronize()
    assert torch.equal(A, B)
    # one segment of a single day (u = w = 0): the plain diagonal
    z1 = torch.zeros_like(vd[:1])
    G1 = sg.fisher_overlap(vd[:1], z1, z1, sg.FGrid(F0, 1 / 32), 0, g[:1].contiguous(), t[:1].contiguous())
    C = torch.zeros((1, 128), dtype=torch.complex64, device="cuda")
    _, Gp = sg.make_maps(C, vd[:1], sg.FGrid(F0, 1 / 32), 0, g[:1].contiguous(), t[:1].contiguous(), want_x=False)
    torch.cuda.synchronize()
    assert torch.equal(G1, Gp)


def test_overlap_fisher_full_band_nside32_sampled(sg, oracle_mod):
    """The configuration the overlap leg of the benchmark times: the full band
    (54 592 bins of 1/32 Hz from 20 Hz), a whole 898-segment day, nside 32,
    antipodal seeds; 3000 sampled (bin, pixel) outputs against the oracle, the
    whole value at the beam bound and the neighbour terms alone at the
    dirty-map bound."""
    nt, nside, k0, nf, df = 898, 32, 0, 54592, 1 / 32
    g, t, v, u, w = _inputs(sg, "AB", nside, nt, k0, nf, df, 12)
    vd, ud, wd = (torch.from_numpy(a).cuda() for a in (v, u, w))
    G = sg.fisher_overlap(vd, ud, wd, sg.FGrid(F0, df), k0, g, t, antipodal=True)
    z = torch.zeros_like(vd)
    G0 = sg.fisher_overlap(vd, z, z, sg.FGrid(F0, df), k0, g, t, antipodal=True)
    npix = 12 * nside * nside
    rng = np.random.default_rng(13)
    rows = np.concatenate([rng.integers(0, nf, 2992), [0, 63, 64, 127, 128, nf - 65, nf - 64, nf - 1]])
    cols = rng.integers(0, npix, rows.size)
    ri, ci = torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()
    Gg = G[ri, ci].double().cpu().numpy()
    Gg0 = G0[ri, ci].double().cpu().numpy()
    del G, G0
    torch.cuda.empty_cache()
    gh, th = g.cpu().numpy(), t.cpu().numpy()
    Go, _, S = oracle_mod.fisher_overlap_at(v, u, w, F0, df, k0, gh, th, rows, cols)
    zh = np.zeros_like(v)
    Go0, _, _ = oracle_mod.fisher_overlap_at(v, zh, zh, F0, df, k0, gh, th, rows, cols)
    assert np.max(np.abs(Gg - Go) / S) <= 1e-4
    S_nb = S - np.abs(Go0)
    err_nb = np.abs((Gg - Gg0) - (Go - Go0)) / S_nb
    round_once = 2.0 ** -23 * np.abs(Gg) / S_nb
    assert np.max(err_nb - round_once) <= 1e-5
