"""The C-ABI library loads on the CPU host and exports every entry point that
include/sgwb.h declares (no compute calls: there may be no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sgwb.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sgwb_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_calls():
    names = declared_functions()
    for n in ("sgwb_build_geometry", "sgwb_make_maps", "sgwb_reduce_band", "sgwb_status_string"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1803_08285_amd as sg

    if not os.path.exists(sg.LIB_PATH):
        pytest.fail("libsgwb.so is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(sg.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(declared_functions()) == sorted(sg.exported_symbols())


def test_status_strings_without_gpu():
    import paper_1803_08285_amd as sg

    L = sg.lib()
    assert L.sgwb_status_string(0) == b"ok"
    assert L.sgwb_status_string(-1) == b"invalid argument"


def test_host_side_validation_rejects_before_any_device_work():
    """Bad arguments are refused on the host, so no GPU is touched."""
    import paper_1803_08285_amd as sg

    L = sg.lib()
    bl = sg._baseline((46.5, -119.4, 126.0, 30.6, -90.8, 198.0))
    tg = sg._TGrid(10, 0.0, 96.0, 192.0)
    dummy = ctypes.c_void_p(256)
    rc = L.sgwb_build_geometry(ctypes.byref(bl), 12, ctypes.byref(tg), dummy, dummy, None)
    assert rc == -1 and b"power of two" in L.sgwb_last_error()
    fg = sg._FGrid(20.0, 0.25)
    rc = L.sgwb_make_maps(dummy, dummy, 5, 10, 8, ctypes.byref(fg), 0, dummy, dummy, 768, 1, dummy, None, None, 0,
                          None)
    assert rc == -1 and b"ldc" in L.sgwb_last_error()
    rc = L.sgwb_make_maps(dummy, dummy, 8, 10, 8, ctypes.byref(fg), 0, dummy, dummy, 700, 1, dummy, None, None, 0,
                          None)
    assert rc == -1 and b"ANTIPODAL" in L.sgwb_last_error()
    rc = L.sgwb_make_maps(dummy, dummy, 8, 10, 8, ctypes.byref(fg), 0, dummy, dummy, 768, 1, None, dummy, None, 0,
                          None)
    assert rc == -2
    rc = L.sgwb_reduce_band(dummy, dummy, dummy, 10, 768, 4, 11, dummy, dummy, None, 0, None)
    assert rc == -1
    bad = sg._FGrid(20.0, 0.0)
    rc = L.sgwb_make_maps(dummy, dummy, 8, 10, 8, ctypes.byref(bad), 0, dummy, dummy, 768, 1, dummy, None, None, 0,
                          None)
    assert rc == -1


def test_fisher_overlap_validation_on_the_host():
    import paper_1803_08285_amd as sg

    L = sg.lib()
    fg = sg._FGrid(20.0, 1 / 32)
    d = ctypes.c_void_p(256)
    # null neighbour series with nt >= 2
    rc = L.sgwb_fisher_overlap(d, None, d, 8, 10, 8, ctypes.byref(fg), 0, d, d, 768, 1, d, d, 1 << 30, None)
    assert rc == -1 and b"neighbour" in L.sgwb_last_error()
    # no output
    rc = L.sgwb_fisher_overlap(d, d, d, 8, 10, 8, ctypes.byref(fg), 0, d, d, 768, 1, None, d, 1 << 30, None)
    assert rc == -1
    # ldc < nf
    rc = L.sgwb_fisher_overlap(d, d, d, 4, 10, 8, ctypes.byref(fg), 0, d, d, 768, 1, d, d, 1 << 30, None)
    assert rc == -1 and b"ldc" in L.sgwb_last_error()
    # workspace too small
    rc = L.sgwb_fisher_overlap(d, d, d, 8, 10, 8, ctypes.byref(fg), 0, d, d, 768, 1, d, d, 256, None)
    assert rc == -2
    # sizes grow with the number of segments
    one = L.sgwb_fisher_overlap_workspace_size(1, 8, 768, 1)
    two = L.sgwb_fisher_overlap_workspace_size(2, 8, 768, 1)
    assert 0 < one < two


def test_fold_validation_on_the_host():
    import paper_1803_08285_amd as sg

    L = sg.lib()
    d = ctypes.c_void_p(256)
    rc = L.sgwb_fold(d, None, d, 8, 2, 10, 8, 0.05, d, d, d, d, None)
    assert rc == -1 and b"null" in L.sgwb_last_error()
    rc = L.sgwb_fold(d, d, d, 4, 2, 10, 8, 0.05, d, d, d, d, None)
    assert rc == -1 and b"ldc" in L.sgwb_last_error()
    rc = L.sgwb_fold(d, d, d, 8, 2, 10, 8, float("nan"), d, d, d, d, None)
    assert rc == -1 and b"W" in L.sgwb_last_error()


def test_network_sum_and_contraction_validation_on_the_host():
    import paper_1803_08285_amd as sg

    L = sg.lib()
    d = ctypes.c_void_p(256)
    arr = (ctypes.c_void_p * 2)(256, None)
    rc = L.sgwb_network_sum(arr, 2, 100, d, None)
    assert rc == -1 and b"map 1" in L.sgwb_last_error()
    rc = L.sgwb_network_sum(arr, 0, 100, d, None)
    assert rc == -1
    rc = L.sgwb_contract_pixels(d, 0, 768, None, 0, d, None)
    assert rc == -1
    rc = L.sgwb_contract_pixels(d, 4, 768, d, -3, d, None)
    assert rc == -1 and b"nsel" in L.sgwb_last_error()


def test_fisher_full_and_clean_map_validation_on_the_host():
    import paper_1803_08285_amd as sg

    L = sg.lib()
    fg = sg._FGrid(20.0, 1 / 32)
    d = ctypes.c_void_p(256)
    big = 1 << 30
    # band outside the columns
    rc = L.sgwb_fisher_full(d, d, 1, d, 10, ctypes.byref(fg), 0, 4, 11, d, d, 8, 768, 0, d, d, big, None)
    assert rc == -1 and b"band" in L.sgwb_last_error()
    rc = L.sgwb_fisher_full(d, d, 1, d, 10, ctypes.byref(fg), 0, 5, 5, d, d, 8, 768, 0, d, d, big, None)
    assert rc == -1
    for rank in (0, 65):
        rc = L.sgwb_fisher_full(d, d, rank, d, 10, ctypes.byref(fg), 0, 0, 10, d, d, 8, 768, 0, d, d, big, None)
        assert rc == -1 and b"rank" in L.sgwb_last_error()
    # null output
    rc = L.sgwb_fisher_full(d, d, 1, d, 10, ctypes.byref(fg), 0, 0, 10, d, d, 8, 768, 0, None, d, big, None)
    assert rc == -1
    # misaligned tau (float64)
    rc = L.sgwb_fisher_full(d, d, 1, d, 10, ctypes.byref(fg), 0, 0, 10, d, ctypes.c_void_p(260), 8, 768, 0, d, d, big,
                            None)
    assert rc == -1 and b"misaligned" in L.sgwb_last_error()
    # workspace too small; the table grows with the top frequency of the band
    rc = L.sgwb_fisher_full(d, d, 1, d, 10, ctypes.byref(fg), 0, 0, 10, d, d, 8, 768, 0, d, d, 256, None)
    assert rc == -2
    low = L.sgwb_fisher_full_workspace_size(ctypes.byref(fg), 0, 10, 8, 768)
    high = L.sgwb_fisher_full_workspace_size(ctypes.byref(fg), 50000, 10, 8, 768)
    more = L.sgwb_fisher_full_workspace_size(ctypes.byref(fg), 50000, 10, 9, 768)
    assert 0 < low < high < more
    bad = sg._FGrid(20.0, 0.0)
    assert L.sgwb_fisher_full_workspace_size(ctypes.byref(bad), 0, 10, 8, 768) == 0
    # the fixed-point delays cover bands up to 24 kHz
    assert L.sgwb_fisher_full_workspace_size(ctypes.byref(fg), 32 * 30000, 10, 8, 768) == 0
    rc = L.sgwb_fisher_full(d, d, 1, d, 10, ctypes.byref(fg), 32 * 30000, 0, 10, d, d, 8, 768, 0, d, d, big, None)
    assert rc == -1 and b"24 kHz" in L.sgwb_last_error()
    # clean map
    rc = L.sgwb_clean_map_cg(d, d, 0, 5, d, d, big, None)
    assert rc == -1
    rc = L.sgwb_clean_map_cg(d, d, 10, -1, d, d, big, None)
    assert rc == -1
    rc = L.sgwb_clean_map_cg(d, d, 10, 5, d, d, 8, None)
    assert rc == -2
    assert L.sgwb_clean_map_workspace_size(0) == 0 < L.sgwb_clean_map_workspace_size(10)


def test_fisher_full_general_validation_on_the_host():
    import paper_1803_08285_amd as sg

    L = sg.lib()
    fg = sg._FGrid(20.0, 1 / 32)
    d = ctypes.c_void_p(256)
    big = 1 << 40
    F = L.sgwb_fisher_full_general
    # band outside the columns, empty band
    rc = F(d, 10, d, 10, ctypes.byref(fg), 0, 4, 11, d, d, 8, 768, 0, d, d, big, None)
    assert rc == -1 and b"band" in L.sgwb_last_error()
    assert F(d, 10, d, 10, ctypes.byref(fg), 0, 5, 5, d, d, 8, 768, 0, d, d, big, None) == -1
    # row stride below the row length
    rc = F(d, 9, d, 10, ctypes.byref(fg), 0, 0, 10, d, d, 8, 768, 0, d, d, big, None)
    assert rc == -1 and b"ldw" in L.sgwb_last_error()
    # segment count beyond the table grid
    rc = F(d, 10, d, 10, ctypes.byref(fg), 0, 0, 10, d, d, 65536, 768, 0, d, d, big, None)
    assert rc == -1 and b"65535" in L.sgwb_last_error()
    # null weights, null output, misaligned tau
    assert F(None, 10, d, 10, ctypes.byref(fg), 0, 0, 10, d, d, 8, 768, 0, d, d, big, None) == -1
    assert F(d, 10, d, 10, ctypes.byref(fg), 0, 0, 10, d, d, 8, 768, 0, None, d, big, None) == -1
    rc = F(d, 10, d, 10, ctypes.byref(fg), 0, 0, 10, d, ctypes.c_void_p(260), 8, 768, 0, d, d, big, None)
    assert rc == -1 and b"misaligned" in L.sgwb_last_error()
    # flags: unknown bits; antipodal with a non-HEALPix pixel count
    rc = F(d, 10, d, 10, ctypes.byref(fg), 0, 0, 10, d, d, 8, 768, 4, d, d, big, None)
    assert rc == -1 and b"flag" in L.sgwb_last_error()
    rc = F(d, 10, d, 10, ctypes.byref(fg), 0, 0, 10, d, d, 8, 700, 1, d, d, big, None)
    assert rc == -1 and b"12 nside^2" in L.sgwb_last_error()
    # workspace too small, or misaligned
    assert F(d, 10, d, 10, ctypes.byref(fg), 0, 0, 10, d, d, 8, 768, 0, d, d, 256, None) == -2
    assert F(d, 10, d, 10, ctypes.byref(fg), 0, 0, 10, d, d, 8, 768, 0, d, ctypes.c_void_p(260), big, None) == -1
    # sizes: grow with the top frequency (table length), the segment count and
    # the band's bins (more bin ranges of partial sums); out of range -> 0
    W = L.sgwb_fisher_full_general_workspace_size
    low = W(ctypes.byref(fg), 0, 0, 10, 8, 768, 0)
    high = W(ctypes.byref(fg), 50000, 0, 10, 8, 768, 0)
    more = W(ctypes.byref(fg), 50000, 0, 10, 9, 768, 0)
    assert 0 < low < high < more
    assert W(ctypes.byref(fg), 50000, 0, 10, 9, 768, 0) < W(ctypes.byref(fg), 50000, 0, 4096, 9, 768, 0)
    assert W(ctypes.byref(fg), 50000, 0, 10, 64, 768, 1) == W(ctypes.byref(fg), 50000, 0, 10, 64, 768, 0)
    bad = sg._FGrid(20.0, 0.0)
    assert W(ctypes.byref(bad), 0, 0, 10, 8, 768, 0) == 0
    assert W(ctypes.byref(fg), 32 * 30000, 0, 10, 8, 768, 0) == 0
    rc = F(d, 10, d, 10, ctypes.byref(fg), 32 * 30000, 0, 10, d, d, 8, 768, 0, d, d, big, None)
    assert rc == -1 and b"24 kHz" in L.sgwb_last_error()


def test_make_maps_band_validation_on_the_host():
    import paper_1803_08285_amd as sg

    L = sg.lib()
    fg = sg._FGrid(20.0, 1 / 32)
    d = ctypes.c_void_p(256)
    big = 1 << 40
    # X without Xbb
    rc = L.sgwb_make_maps_band(d, d, 8, 10, 8, ctypes.byref(fg), 0, d, d, 768, 1, d, 0, 8, d, None, None, None, d,
                               big, None)
    assert rc == -1 and b"X needs Xbb" in L.sgwb_last_error()
    # Xbb alone needs the matrix-core dirty map: refused with a vector-unit request, or at df = 1/4 Hz
    rc = L.sgwb_make_maps_band(d, d, 8, 10, 8, ctypes.byref(fg), 0, d, d, 768, 1 | 2, d, 0, 8, None, None, d, d, d,
                               big, None)
    assert rc == -1 and b"matrix-core" in L.sgwb_last_error()
    coarse = sg._FGrid(20.0, 0.25)
    rc = L.sgwb_make_maps_band(d, d, 8, 10, 8, ctypes.byref(coarse), 0, d, d, 768, 1, d, 0, 8, None, None, d, None,
                               d, big, None)
    assert rc == -1 and b"matrix-core" in L.sgwb_last_error()
    # nothing asked for
    rc = L.sgwb_make_maps_band(d, d, 8, 10, 8, ctypes.byref(fg), 0, d, d, 768, 1, d, 0, 8, None, None, None, None,
                               d, big, None)
    assert rc == -1
    # band beyond the columns
    rc = L.sgwb_make_maps_band(d, d, 8, 10, 8, ctypes.byref(fg), 0, d, d, 768, 1, d, 0, 9, d, d, d, d, d, big,
                               None)
    assert rc == -1 and b"band" in L.sgwb_last_error()
    # Gbb without H
    rc = L.sgwb_make_maps_band(d, d, 8, 10, 8, ctypes.byref(fg), 0, d, d, 768, 1, None, 0, 8, d, d, d, d, d, big,
                               None)
    assert rc == -1 and b"H" in L.sgwb_last_error()
    # workspace too small; its size covers make_maps' and grows with the bins
    rc = L.sgwb_make_maps_band(d, d, 8, 10, 8, ctypes.byref(fg), 0, d, d, 768, 1, d, 0, 8, d, d, d, d, d, 256,
                               None)
    assert rc == -2
    assert L.sgwb_make_maps_band_workspace_size(10, 8, 768, 1) > L.sgwb_make_maps_workspace_size(10, 8, 768, 1)
    assert L.sgwb_make_maps_band_workspace_size(10, 800, 768, 1) > L.sgwb_make_maps_band_workspace_size(10, 8, 768, 1)


def test_short_matrix_core_workspace_is_refused_on_the_host():
    """With the antipodal flag at df = 1/32 Hz the matrix-core dirty map applies;
    a workspace too small for it is an error (SGWB_ENOMEM), not a silent switch
    to the vector units, and the form record then says no dirty map ran."""
    import paper_1803_08285_amd as sg

    L = sg.lib()
    fg = sg._FGrid(20.0, 1 / 32)
    d = ctypes.c_void_p(256)
    rc = L.sgwb_make_maps(d, d, 8, 10, 8, ctypes.byref(fg), 0, d, d, 768, 1, d, None, d, 256, None)
    assert rc == -2 and b"matrix-core" in L.sgwb_last_error()
    form = ctypes.c_int32(-7)
    assert L.sgwb_last_x_form(ctypes.byref(form)) == 0 and form.value == 0
    # unknown flag bits are refused before anything else
    rc = L.sgwb_make_maps(d, d, 8, 10, 8, ctypes.byref(fg), 0, d, d, 768, 1 | 8, d, None, d, 256, None)
    assert rc == -1 and b"flag" in L.sgwb_last_error()


def test_broadband_route_bound_and_validation_on_the_host():
    """Delay bound of a baseline (its chord / c, the R7 Earth model), the
    broadband call's route choice and workspace size, and its refusals, all on
    the host."""
    import numpy as np

    import paper_1803_08285_amd as sg
    import synth

    L = sg.lib()
    R, c = 6.371e6, 299792458.0
    for name, want_ms in (("AB", 9.993), ("AC", 27.207), ("BC", 26.391)):
        s = synth.baseline_sites(name)
        pos = []
        for lat, lon in ((s[0], s[1]), (s[3], s[4])):
            la, lo = np.radians(lat), np.radians(lon)
            pos.append(R * np.array([np.cos(la) * np.cos(lo), np.cos(la) * np.sin(lo), np.sin(la)]))
        chord = np.linalg.norm(pos[0] - pos[1]) / c
        b = sg.baseline_delay_bound(s)
        assert chord <= b <= chord * (1 + 1e-8) + 1e-14
        assert abs(b * 1e3 - want_ms) < 1e-3
    fg = sg.FGrid(20.0, 1.0 / 32.0)
    tb = sg.baseline_delay_bound(synth.baseline_sites("AB"))
    nt = 898
    # a GPU-filling band at nside 128 takes the tables, the same band at nside 8 the strips
    big = sg.broadband_maps_workspace_bytes(nt, 4096, 196608, fg, 0, 4096, tb)
    forced = sg.broadband_maps_workspace_bytes(nt, 4096, 196608, fg, 0, 4096, tb, route="table")
    assert big == forced > 0
    small = sg.broadband_maps_workspace_bytes(nt, 4096, 768, fg, 0, 4096, tb)
    assert small == sg.band_maps_workspace_bytes(nt, 4096, 768) > 0
    # the tables need no antipodal seeds and no matrix-core grid; the strips do
    assert sg.broadband_maps_workspace_bytes(nt, 64, 700, sg.FGrid(20.0, 0.25), 0, 64, tb, antipodal=False) > 0
    for kw in (dict(route="strips", antipodal=False), dict(tau_bound=-1.0), dict(tau_bound=float("nan"))):
        args = dict(tau_bound=tb)
        args.update(kw)
        assert sg.broadband_maps_workspace_bytes(nt, 64, 768, fg, 0, 64, **args) == 0
    assert sg.broadband_maps_workspace_bytes(nt, 64, 768, fg, 5, 5, tb) == 0  # empty band
    # a band whose table would pass 2^21 + 3 nodes: strips when they apply, else refused
    assert sg.broadband_maps_workspace_bytes(nt, 54592, 768, fg, 0, 54592, 10.0) == 0
    assert sg.broadband_maps_workspace_bytes(nt, 54592, 768, fg, 0, 54592, 0.04) == sg.band_maps_workspace_bytes(
        nt, 54592, 768)
    dummy = ctypes.c_void_p(256)
    cfg = sg._FGrid(20.0, 1.0 / 32.0)
    rc = L.sgwb_broadband_maps(dummy, dummy, 64, 10, 64, ctypes.byref(cfg), 0, dummy, dummy, 768,
                               sg.SGWB_BB_TABLE | sg.SGWB_BB_STRIPS | 1, tb, dummy, 0, 64, dummy, dummy, dummy, 1 << 20,
                               None)
    assert rc == -1 and b"both routes" in L.sgwb_last_error()
    rc = L.sgwb_broadband_maps(dummy, dummy, 64, 10, 64, ctypes.byref(cfg), 0, dummy, dummy, 768, 16 | 1, tb, dummy,
                               0, 64, dummy, dummy, dummy, 1 << 20, None)
    assert rc == -1 and b"flag" in L.sgwb_last_error()
    rc = L.sgwb_broadband_maps(dummy, dummy, 64, 10, 64, ctypes.byref(cfg), 0, dummy, dummy, 768, 1, tb, dummy, 0, 64,
                               None, None, dummy, 1 << 20, None)
    assert rc == -1 and b"nothing" in L.sgwb_last_error()
    rc = L.sgwb_broadband_maps(dummy, dummy, 64, 10, 64, ctypes.byref(cfg), 0, dummy, dummy, 768,
                               sg.SGWB_BB_TABLE | 1, tb, dummy, 0, 64, dummy, dummy, dummy, 256, None)
    assert rc == -2 and b"workspace" in L.sgwb_last_error()


def test_broadband_cost_rule_picks_the_measured_winner():
    """The route the host's cost rule picks for full-day queries (898 segments,
    1/32 Hz) against the faster route measured on one MI355X for each of them
    (strips / tables, ms): only the widest bands at the lowest resolutions
    keep the strips."""
    import paper_1803_08285_amd as sg
    import synth

    measured = {  # (baseline, nside, bins): (strips ms, tables ms)
        ("AB", 8, 16): (0.205, 0.040), ("AB", 8, 1024): (0.202, 0.086), ("AB", 8, 4096): (0.229, 0.294),
        ("AB", 16, 4096): (0.409, 0.311), ("AB", 32, 4096): (1.200, 0.317), ("AB", 128, 16): (1.521, 0.409),
        ("AB", 128, 4096): (17.016, 0.659), ("AC", 8, 4096): (0.259, 0.584), ("AC", 16, 1024): (0.247, 0.093),
        ("AC", 16, 4096): (0.461, 0.570), ("AC", 32, 4096): (1.352, 0.584), ("AC", 128, 4096): (20.190, 0.979),
    }
    fg = sg.FGrid(20.0, 1 / 32)
    for (bl, nside, nb), (t_strips, t_table) in measured.items():
        tb = sg.baseline_delay_bound(synth.baseline_sites(bl))
        npix = 12 * nside * nside
        auto = sg.broadband_maps_workspace_bytes(898, nb, npix, fg, 0, nb, tb)
        table = sg.broadband_maps_workspace_bytes(898, nb, npix, fg, 0, nb, tb, route="table")
        picked_table = auto == table
        assert picked_table == (t_table < t_strips), (bl, nside, nb)
