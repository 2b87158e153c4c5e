"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (derivation in the design notes):
  * X, float32 path: max |dX| / S <= 1e-5 with S(k,p) = sum_t |w gamma| |C|.
  * Gam, split-bfloat16 path: elementwise |dGam| / Gam <= 1e-4.
  * float64 path: X within 1e-12 of S, Gam within 1e-12 relative.
  * seeds: gamma within float32 rounding of the float64 value, tau within 1e-15 s.
Kernel parity feeds the oracle the exact stored GPU inputs (float32 C, w, gamma
and float64 tau, widened to float64).
"""
import numpy as np
import pytest

import synth
from tests._cases import freqs, g_error, make_csd, x_error

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

X_TOL = 1e-5
G_TOL = 1e-4


@pytest.fixture(scope="module")
def sg():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1803_08285_amd as sg

    assert sg.device_supported(), "not a gfx950 device"
    return sg


def _geom(sg, bl, nside, tg, dtype=torch.float32):
    g, t = sg.build_geometry(synth.baseline_sites(bl), nside, sg.TGrid(tg.nt, tg.t0, tg.stride, tg.dur), dtype=dtype)
    torch.cuda.synchronize()
    return g, t


# --------------------------------------------------------------------------- HEALPix / geometry
@pytest.mark.parametrize("nside", [1, 2, 8, 64])
def test_healpix_centres_and_antipodes(sg, oracle_mod, nside):
    xyz, anti = sg.healpix_centres(nside)
    torch.cuda.synchronize()
    ref = oracle_mod.healpix_centres(nside)
    np.testing.assert_allclose(xyz.cpu().numpy(), ref, atol=2e-15)
    a = anti.cpu().numpy()
    np.testing.assert_allclose(ref[a], -ref, atol=1e-14)
    assert np.array_equal(a[a], np.arange(a.size))


@pytest.mark.parametrize("bl,nside", [("AB", 8), ("AC", 2), ("BC", 16)])
def test_geometry_full_small(sg, oracle_mod, bl, nside):
    tg = synth.TGRID_TINY
    g, t = _geom(sg, bl, nside, tg)
    go, to = oracle_mod.geometry(synth.baseline_sites(bl), nside, tg.nt, tg.t0, tg.stride, tg.dur)
    gg = g.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(gg - go) / np.maximum(np.abs(go), 1e-30)) <= 2 ** -24 * 1.01 or \
        np.max(np.abs(gg - go)) <= 1e-14
    np.testing.assert_allclose(t.cpu().numpy(), to, rtol=0, atol=1e-15)
    g64, t64 = _geom(sg, bl, nside, tg, dtype=torch.float64)
    np.testing.assert_allclose(g64.cpu().numpy(), go, rtol=0, atol=2e-15)


def test_geometry_full_day_nside64_rows(sg, oracle_mod):
    tg = synth.TGRID_FULL
    g, t = _geom(sg, "AB", 64, tg)
    det = synth.baseline_sites("AB")
    for k in (0, 1, 450, 897):
        go, to = oracle_mod.geometry(det, 64, 1, tg.t0 + k * tg.stride, tg.stride, tg.dur)
        gg = g[k].cpu().numpy().astype(np.float64)
        err = np.abs(gg - go[0])
        assert np.all(err <= 2 ** -24 * np.abs(go[0]) + 1e-15), (k, err.max())
        np.testing.assert_allclose(t[k].cpu().numpy(), to[0], rtol=0, atol=1e-15)


# --------------------------------------------------------------------------- maps, small sizes
def _run_maps(sg, C, w, f0, df, k0, g, t, antipodal):
    Cd = torch.from_numpy(C).cuda()
    wd = torch.from_numpy(w).cuda()
    X, G = sg.make_maps(Cd, wd, sg.FGrid(f0, df), k0, g, t, antipodal=antipodal)
    torch.cuda.synchronize()
    return X.cpu().numpy(), G.cpu().numpy()


@pytest.mark.parametrize("antipodal", [True, False])
@pytest.mark.parametrize("bl,nside,nf,k0,nt", [
    ("AB", 8, 1024, 0, 240),     # tiny workload shape
    ("AC", 16, 203, 37, 61),     # ragged bins, unaligned anchor, several pixel tiles
    ("BC", 2, 70, 64 * 9 + 63, 5),  # band starts one bin before an anchor
    ("AB", 1, 1, 12345, 1),      # single bin, single segment, 12 pixels
])
def test_maps_float32_vs_oracle(sg, oracle_mod, antipodal, bl, nside, nf, k0, nt):
    f0, df = 20.0, 0.25
    tg = synth.TGrid(nt, 0.0, 86164.0905 / nt, 86164.0905 / nt)
    g, t = _geom(sg, bl, nside, tg)
    f = freqs(f0, df, k0, nf)
    C, w = make_csd(7 + nside, nt, f)
    Xg, Gg = _run_maps(sg, C, w, f0, df, k0, g, t, antipodal)
    Xo, Go, S = oracle_mod.maps(C, w, f0, df, k0, g.cpu().numpy(), t.cpu().numpy(), with_scale=True)
    ex, eg = x_error(Xg, Xo, S), g_error(Gg, Go)
    print(f"X err {ex:.3e}  Gam err {eg:.3e}")
    assert ex <= X_TOL
    assert eg <= G_TOL


# df = 1/32 Hz: the matrix-core dirty map applies with antipodal seeds; the
# vector-unit recurrence is forced with x_kernel="valu".  Both against the oracle.
@pytest.mark.parametrize("x_kernel", ["auto", "valu"])
@pytest.mark.parametrize("bl,nside,nf,k0,nt", [
    ("AB", 8, 640, 0, 240),
    ("AC", 16, 203, 37, 61),       # ragged strips and chunks, 1536 pairs = 6 workgroups
    ("BC", 4, 130, 64 * 9 + 63, 17),
    ("AC", 32, 64, 128, 33),       # exactly one strip, nt not a multiple of 16
    ("AB", 1, 3, 5, 1),            # one segment, 6 pairs
])
def test_maps_df32_both_kernels_vs_oracle(sg, oracle_mod, x_kernel, bl, nside, nf, k0, nt):
    f0, df = 20.0, 1.0 / 32.0
    tg = synth.TGrid(nt, 0.0, 86164.0905 / nt, 86164.0905 / nt)
    g, t = _geom(sg, bl, nside, tg)
    f = freqs(f0, df, k0, nf)
    C, w = make_csd(70 + nside, nt, f)
    Xd, Gd = sg.make_maps(torch.from_numpy(C).cuda(), torch.from_numpy(w).cuda(), sg.FGrid(f0, df), k0, g, t,
                          x_kernel=x_kernel)
    torch.cuda.synchronize()
    Xo, Go, S = oracle_mod.maps(C, w, f0, df, k0, g.cpu().numpy(), t.cpu().numpy(), with_scale=True)
    ex, eg = x_error(Xd.cpu().numpy(), Xo, S), g_error(Gd.cpu().numpy(), Go)
    print(f"{x_kernel}: X err {ex:.3e}  Gam err {eg:.3e}")
    assert ex <= X_TOL
    assert eg <= G_TOL


def test_matrix_core_map_scale_extremes(sg, oracle_mod):
    """Bins whose data differ by 2^40 in scale and a bin of zeros: the per-bin
    float16 scaling keeps every bin within tolerance."""
    nside, nt, nf, k0, f0, df = 8, 40, 128, 0, 20.0, 1.0 / 32.0
    g, t = _geom(sg, "AB", nside, synth.TGrid(nt, 0.0, 2154.0, 2154.0))
    f = freqs(f0, df, k0, nf)
    C, w = make_csd(3, nt, f)
    w = w * np.where(np.arange(nf) % 2 == 0, 2.0 ** -20, 2.0 ** 20).astype(np.float32)[None, :]
    C[:, 7] = 0
    Xd, _ = sg.make_maps(torch.from_numpy(C).cuda(), torch.from_numpy(w).cuda(), sg.FGrid(f0, df), k0, g, t)
    Xo, Go, S = oracle_mod.maps(C, w, f0, df, k0, g.cpu().numpy(), t.cpu().numpy(), with_scale=True)
    Xh = Xd.cpu().numpy()
    assert np.all(Xh[7] == 0)
    ok = S > 0
    assert np.max(np.abs(Xh[ok] - Xo[ok]) / S[ok]) <= X_TOL


def test_maps_float64_tiny_workload(sg, oracle_mod):
    """The tiny workload in float64: same kernels instantiated for double."""
    wl = synth.workload(1)
    tg = wl.tgrid
    g, t = _geom(sg, wl.baseline, wl.nside, tg, dtype=torch.float64)
    f = wl.fgrid.freqs()
    C, w = make_csd(wl.noise_seed, tg.nt, f, dtype=np.complex128)
    gh, th = g.cpu().numpy(), t.cpu().numpy()
    for p, A in zip(wl.src_pix, wl.src_amp):
        synth.add_point_source(C, f, A, gh[:, p], th[:, p])
    Xg, Gg = _run_maps(sg, C, w, wl.fgrid.f0, wl.fgrid.df, wl.fgrid.k0, g, t, True)
    Xo, Go, S = oracle_mod.maps(C, w, wl.fgrid.f0, wl.fgrid.df, wl.fgrid.k0, gh, th, with_scale=True)
    assert x_error(Xg, Xo, S) <= 1e-12
    assert g_error(Gg, Go) <= 1e-12


def test_point_source_recovered_on_gpu(sg):
    """Noise-free source at a pixel centre: X(k,p0) = A H(f_k) Gam(k,p0)."""
    nside, nt, nf, k0 = 8, 240, 300, 0
    g, t = _geom(sg, "AB", nside, synth.TGRID_TINY)
    f = freqs(20.0, 0.25, k0, nf)
    p0, A = 100, 0.1
    C = np.zeros((nt, nf), np.complex128)
    synth.add_point_source(C, f, A, g[:, p0].cpu().numpy(), t[:, p0].cpu().numpy())
    w = synth.weights(f, np.ones(nt)).astype(np.float32)
    Xg, Gg = _run_maps(sg, C.astype(np.complex64), w, 20.0, 0.25, k0, g, t, True)
    H = synth.spectrum_H(f)
    S = (np.abs(w) * np.abs(C).astype(np.float64)).T @ np.abs(g.cpu().numpy().astype(np.float64))
    err = np.abs(Xg[:, p0] - A * H * Gg[:, p0]) / (S[:, p0] + A * H * Gg[:, p0])
    assert err.max() <= 2e-4


def test_determinism_and_subband_bitwise(sg):
    nside, nt, nf = 8, 120, 640
    g, t = _geom(sg, "BC", nside, synth.TGrid(nt, 0.0, 718.0, 718.0))
    f = freqs(20.0, 1 / 32, 0, nf)
    C, w = make_csd(3, nt, f)
    Cd, wd = torch.from_numpy(C).cuda(), torch.from_numpy(w).cuda()
    fg = sg.FGrid(20.0, 1 / 32)
    X1, G1 = sg.make_maps(Cd, wd, fg, 0, g, t)
    X2, G2 = sg.make_maps(Cd, wd, fg, 0, g, t)
    lo, hi = 77, 389
    Xs, Gs = sg.make_maps(Cd[:, lo:hi], wd[:, lo:hi], fg, lo, g, t)
    torch.cuda.synchronize()
    assert torch.equal(X1, X2) and torch.equal(G1, G2)
    assert torch.equal(Xs, X1[lo:hi])  # absolute anchor grid: bitwise equal rows


# --------------------------------------------------------------------------- band reduce
@pytest.mark.parametrize("klo,khi", [(0, 1024), (5, 6), (300, 300), (17, 1000)])
def test_reduce_band_vs_oracle(sg, oracle_mod, klo, khi):
    nside, nt, nf = 8, 60, 1024
    g, t = _geom(sg, "AB", nside, synth.TGrid(nt, 0.0, 1436.0, 1436.0))
    f = freqs(20.0, 0.25, 0, nf)
    C, w = make_csd(5, nt, f)
    X, G = sg.make_maps(torch.from_numpy(C).cuda(), torch.from_numpy(w).cuda(), sg.FGrid(20.0, 0.25), 0, g, t)
    H = torch.from_numpy(synth.spectrum_H(f).astype(np.float32)).cuda()
    Xbb, Gbb = sg.reduce_band(X, G, H, klo, khi)
    torch.cuda.synchronize()
    Xh, Gh, Hh = X.cpu().numpy(), G.cpu().numpy(), H.cpu().numpy()
    Xo, Go = oracle_mod.band(Xh, Gh, Hh, klo, khi)
    scale_x = np.abs(Xh[klo:khi]).sum(axis=0) if khi > klo else np.zeros(Xh.shape[1])
    assert np.all(np.abs(Xbb.cpu().numpy() - Xo) <= 2 ** -24 * np.abs(Xo) + 1e-12 * scale_x + 1e-300)
    assert np.all(np.abs(Gbb.cpu().numpy() - Go) <= 2 ** -24 * np.abs(Go) * 1.01 + 1e-300)


def test_reduce_band_single_pass_matches_split(sg):
    nside, nt, nf = 16, 40, 3000
    g, t = _geom(sg, "AC", nside, synth.TGrid(nt, 0.0, 2154.0, 2154.0))
    f = freqs(20.0, 1 / 32, 0, nf)
    C, w = make_csd(8, nt, f)
    X, G = sg.make_maps(torch.from_numpy(C).cuda(), torch.from_numpy(w).cuda(), sg.FGrid(20.0, 1 / 32), 0, g, t)
    H = torch.from_numpy(synth.spectrum_H(f).astype(np.float32)).cuda()
    a = sg.reduce_band(X, G, H, 11, 2990, workspace=True)
    b = sg.reduce_band(X, G, H, 11, 2990, workspace=None)
    c = sg.reduce_band(X, G, H, 11, 2990, workspace=True)
    torch.cuda.synchronize()
    for u, v in zip(a, b):
        torch.testing.assert_close(u, v, rtol=2 ** -23, atol=0)
    assert torch.equal(a[0], c[0]) and torch.equal(a[1], c[1])


def test_reduce_band_float64(sg, oracle_mod):
    nside, nt, nf = 2, 10, 100
    g, t = _geom(sg, "AB", nside, synth.TGrid(nt, 0.0, 8616.0, 8616.0), dtype=torch.float64)
    f = freqs(20.0, 0.25, 0, nf)
    C, w = make_csd(6, nt, f, dtype=np.complex128)
    X, G = sg.make_maps(torch.from_numpy(C).cuda(), torch.from_numpy(w).cuda(), sg.FGrid(20.0, 0.25), 0, g, t)
    H = torch.from_numpy(synth.spectrum_H(f)).cuda()
    Xbb, Gbb = sg.reduce_band(X, G, H, 3, 97)
    Xo, Go = oracle_mod.band(X.cpu().numpy(), G.cpu().numpy(), H.cpu().numpy(), 3, 97)
    np.testing.assert_allclose(Xbb.cpu().numpy(), Xo, rtol=1e-13, atol=1e-13 * np.abs(Xo).max())
    np.testing.assert_allclose(Gbb.cpu().numpy(), Go, rtol=1e-13)


# --------------------------------------------------------------------------- full-size workloads (sampled)
@pytest.mark.parametrize("cfg", [2, 3])
def test_full_band_workload_sampled(sg, oracle_mod, cfg):
    """The full-band workloads at their real sizes, in the launch configuration
    the benchmark times; sampled rows and columns against the oracle."""
    wl = synth.workload(cfg)
    tg, fgd = wl.tgrid, wl.fgrid
    g, t = _geom(sg, wl.baseline, wl.nside, tg)
    f = fgd.freqs()
    C, w = make_csd(wl.noise_seed, tg.nt, f)
    gh = g.cpu().numpy()
    th = t.cpu().numpy()
    # sources in the directions of the nside-32 source pixels (nearest centre at nside 64)
    npix = gh.shape[1]
    src = list(wl.src_pix)
    if wl.nside != 32:
        c32, _ = sg.healpix_centres(32)
        cN, _ = sg.healpix_centres(wl.nside)
        src = [int(torch.argmax(cN @ c32[p])) for p in src]
    Cc = C.astype(np.complex128)
    for p, A in zip(src, wl.src_amp):
        synth.add_point_source(Cc, f, A, gh[:, p], th[:, p])
    C = Cc.astype(np.complex64)
    del Cc
    Cd, wd = torch.from_numpy(C).cuda(), torch.from_numpy(w).cuda()
    X, G = sg.make_maps(Cd, wd, sg.FGrid(fgd.f0, fgd.df), fgd.k0, g, t)
    torch.cuda.synchronize()
    rows, cols = synth.random_selection(40 + cfg, fgd.nf, npix, 4, 3)
    Xs = X[torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()].cpu().numpy()
    Gs = G[torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda()].cpu().numpy()
    Xo, Go, S = oracle_mod.maps_at(C, w, fgd.f0, fgd.df, fgd.k0, gh, th, rows, cols)
    ex, eg = x_error(Xs, Xo, S), g_error(Gs, Go)
    print(f"cfg {cfg}: X err {ex:.3e}  Gam err {eg:.3e}  ({rows.size} samples)")
    assert ex <= X_TOL
    assert eg <= G_TOL
    # properties that hold everywhere: Gam >= 0 and antipodal symmetry of Gam
    assert bool((G >= 0).all())
    _, anti = sg.healpix_centres(wl.nside)
    assert torch.equal(G[:, anti.long()], G)
