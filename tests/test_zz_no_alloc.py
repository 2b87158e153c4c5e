"""sgwb_make_maps_band_noalloc (the allocation-free variant of
sgwb_make_maps_band, workspace in the library's fixed scratch array) against
the workspace entry point, through the C ABI: bitwise the same maps on two calls
in a row, the second smaller (the array keeps the first call's contents), and a
call too large for the array refused before any device work."""
import numpy as np
import pytest

import synth
from tests._cases import freqs, make_csd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F0, DF = 20.0, 1 / 32


@pytest.fixture(scope="module")
def sg():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1803_08285_amd as sg

    return sg


def _case(sg, bl, nside, nt, k0, nf, seed):
    tg = sg.TGrid(nt, 0.0, 86164.0905 / nt, 86164.0905 / nt)
    g, t = sg.build_geometry(synth.baseline_sites(bl), nside, tg)
    f = freqs(F0, DF, k0, nf)
    C, w = make_csd(seed, nt, f)
    H = synth.spectrum_H(f).astype(np.float32)
    return g, t, torch.from_numpy(C).cuda(), torch.from_numpy(w).cuda(), torch.from_numpy(H).cuda()


def _outs(nf, npix):
    return tuple(torch.empty(s, dtype=torch.float32, device="cuda") for s in ((nf, npix), (nf, npix), (npix,), (npix,)))


@pytest.mark.parametrize("first,second", [
    (("AC", 16, 120, 37, 700, (5, 690)), ("AB", 8, 60, 64 * 3 + 1, 130, (0, 130))),
    (("AD", 8, 90, 0, 900, (100, 800)), ("BC", 4, 33, 5, 66, (7, 60))),
])
def test_noalloc_matches_workspace_call_twice(sg, first, second):
    for bl, nside, nt, k0, nf, (klo, khi) in (first, second):
        print(f"case {bl} nside {nside} nt {nt} k0 {k0} nf {nf} band {klo}:{khi}", flush=True)
        g, t, C, w, H = _case(sg, bl, nside, nt, k0, nf, 7 + nside)
        npix = 12 * nside * nside
        need = sg.band_maps_workspace_bytes(nt, nf, npix)
        assert need <= sg.SGWB_NOALLOC_SCRATCH_BYTES
        ref = sg.make_maps_band(C, w, sg.FGrid(F0, DF), k0, g, t, H, klo, khi)
        got = sg.make_maps_band(C, w, sg.FGrid(F0, DF), k0, g, t, H, klo, khi, noalloc=True, out=_outs(nf, npix))
        form = sg.last_x_form()
        torch.cuda.synchronize()
        assert form.startswith("mfma")
        for a, b in zip(ref, got):
            assert torch.equal(a, b)


def test_noalloc_refuses_a_call_beyond_the_scratch_array(sg):
    nside, nt, nf = 64, 898, 64
    npix = 12 * nside * nside
    assert sg.band_maps_workspace_bytes(nt, nf, npix) > sg.SGWB_NOALLOC_SCRATCH_BYTES
    g = torch.zeros((nt, npix), dtype=torch.float32, device="cuda")
    t = torch.zeros((nt, npix), dtype=torch.float64, device="cuda")
    C = torch.zeros((nt, nf), dtype=torch.complex64, device="cuda")
    w = torch.zeros((nt, nf), dtype=torch.float32, device="cuda")
    H = torch.zeros(nf, dtype=torch.float32, device="cuda")
    with pytest.raises(sg.SgwbError, match="scratch"):
        sg.make_maps_band(C, w, sg.FGrid(F0, DF), 0, g, t, H, 0, nf, noalloc=True, out=_outs(nf, npix))
