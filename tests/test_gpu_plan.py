"""Batched plans on the GPU: several baselines, resolutions and uneven bands in
one persistent launch per kernel, replayed from a HIP graph.

The plan's maps must be bitwise equal to the single-call path (make_maps_band,
which the parity tests compare with the oracle), on every graph replay, with
eager work between replays; autotuned, cached and graph-free plans must agree too.
"""
import json

import numpy as np
import pytest

import synth
from tests._cases import freqs, g_error, make_csd, x_error

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

JOBS = [  # baseline, nside, nt, k0, nf, band, antipodal pairing, df (1/32: matrix-core dirty map)
    ("AB", 16, 60, 0, 700, (0, 700), True, 0.25),
    ("AC", 8, 45, 100, 300, (13, 290), True, 0.25),
    ("BC", 4, 60, 1000, 130, (0, 130), False, 0.25),
    ("AB", 2, 7, 63, 2, (0, 2), True, 0.25),
    ("AC", 16, 50, 197, 400, (3, 399), True, 1 / 32),
    ("BC", 8, 33, 0, 64, (0, 64), True, 1 / 32),
    ("AB", 8, 40, 70, 200, (1, 199), True, 1 / 32),  # short baseline: the four-term matrix-core form
]
F0 = 20.0


@pytest.fixture(scope="module")
def sg():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1803_08285_amd as sg

    return sg


def _make_jobs(sg):
    jobs, refs, host = [], [], []
    for i, (bl, nside, nt, k0, nf, band, anti, DF) in enumerate(JOBS):
        tg = sg.TGrid(nt, 0.0, 86164.0905 / nt, 86164.0905 / nt)
        g, t = sg.build_geometry(synth.baseline_sites(bl), nside, tg)
        f = freqs(F0, DF, k0, nf)
        C, w = make_csd(30 + i, nt, f)
        Cd, wd = torch.from_numpy(C).cuda(), torch.from_numpy(w).cuda()
        H = torch.from_numpy(synth.spectrum_H(f).astype(np.float32)).cuda()
        npix = 12 * nside * nside
        X = torch.full((nf, npix), float("nan"), device="cuda")
        G = torch.full((nf, npix), float("nan"), device="cuda")
        Xbb = torch.full((npix,), float("nan"), device="cuda")
        Gbb = torch.full((npix,), float("nan"), device="cuda")
        jobs.append(sg.Job(Cd, wd, sg.FGrid(F0, DF), k0, g, t, X=X, G=G, H=H, band=band, Xbb=Xbb, Gbb=Gbb,
                           antipodal=anti))
        Xr, Gr, Xbr, Gbr = sg.make_maps_band(Cd, wd, sg.FGrid(F0, DF), k0, g, t, H, *band, antipodal=anti)
        refs.append((Xr, Gr, Xbr, Gbr))
        host.append((C, w, g, t, k0, DF))
    torch.cuda.synchronize()
    return jobs, refs, host


def _assert_equal(jobs, refs):
    for j, (Xr, Gr, Xbr, Gbr) in zip(jobs, refs):
        assert torch.equal(j.X, Xr)
        assert torch.equal(j.G, Gr)
        assert torch.equal(j.Xbb, Xbr)
        assert torch.equal(j.Gbb, Gbr)


def test_plan_graph_replays_bitwise(sg, tmp_path, monkeypatch):
    monkeypatch.setenv("SGWB_TUNE_CACHE", str(tmp_path / "tune.json"))
    jobs, refs, _ = _make_jobs(sg)
    plan = sg.Plan(jobs, autotune=True, graph=True)
    d = plan.describe()
    assert d["graph"] and d["tuned"] and not d["from_cache"]
    for rep in range(3):
        for j in jobs:  # poison outputs between replays
            for t in (j.X, j.G, j.Xbb, j.Gbb):
                t.fill_(float("nan"))
        scratch = torch.randn(1 << 20, device="cuda")  # eager work between replays
        scratch.sum().item()
        plan.launch()
        torch.cuda.synchronize()
        _assert_equal(jobs, refs)
    plan.close()
    # a second plan over the same shapes hits the tuning cache
    plan2 = sg.Plan(jobs, autotune=True, graph=False)
    d2 = plan2.describe()
    assert d2["from_cache"] and not d2["graph"]
    for j in jobs:
        j.X.zero_()
    plan2.launch()
    torch.cuda.synchronize()
    _assert_equal(jobs, refs)
    assert d2["x_strip_major"] == d["x_strip_major"] and d2["beam_shape"] == d["beam_shape"]


def test_plan_every_schedule_gives_the_same_maps(sg, tmp_path, monkeypatch):
    """Untuned default schedule vs autotuned schedule: identical bits."""
    monkeypatch.setenv("SGWB_TUNE_CACHE", str(tmp_path / "tune.json"))
    jobs, refs, _ = _make_jobs(sg)
    for autotune in (False, True):
        plan = sg.Plan(jobs, autotune=autotune)
        for j in jobs:
            j.X.fill_(float("nan"))
            j.G.fill_(float("nan"))
        plan.launch()
        torch.cuda.synchronize()
        _assert_equal(jobs, refs)
        plan.close()


@pytest.mark.parametrize("xm_per_job,beam_shape,beam_grid,branches",
                         [(1, 1, 0, 0), (0, 1, 0, 1), (1, 0, 2, 1), (0, 0, 8, 0)])
def test_plan_forced_schedules_give_the_same_maps(sg, tmp_path, monkeypatch, xm_per_job, beam_shape, beam_grid,
                                                  branches):
    """Each schedule candidate, forced through the tuning cache: identical bits.

    beam_shape 1 is the 2x4 wave tile, 0 the 4x4; beam_grid 0 is one workgroup per
    tile group (no persistent loop); xm_per_job 1 launches the single-call
    dirty-map kernel once per job instead of the multi-job kernel; branches 1
    puts the beams on a second graph branch beside the dirty maps."""
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("SGWB_TUNE_CACHE", str(cache))
    jobs, refs, _ = _make_jobs(sg)
    p0 = sg.Plan(jobs, autotune=False)
    key = p0.describe()["key"]
    p0.close()
    cache.write_text(json.dumps({key: {"x_strip_major": 0, "x_grid_per_cu": 4, "beam_shape": beam_shape,
                                       "beam_grid_per_cu": beam_grid, "xm_per_job": xm_per_job,
                                       "branches": branches}}))
    plan = sg.Plan(jobs, autotune=True)
    d = plan.describe()
    assert d["from_cache"] and d["xm_per_job"] == xm_per_job and d["beam_grid_per_cu"] == beam_grid
    assert d["branches"] == branches
    assert d["beam_shape"] == ("2x4" if beam_shape == 1 else "4x4")
    for j in jobs:
        for t in (j.X, j.G, j.Xbb, j.Gbb):
            t.fill_(float("nan"))
    plan.launch()
    torch.cuda.synchronize()
    _assert_equal(jobs, refs)
    plan.close()


def test_plan_against_oracle(sg, oracle_mod):
    jobs, _, host = _make_jobs(sg)
    plan = sg.Plan(jobs, autotune=False)
    plan.launch()
    torch.cuda.synchronize()
    for j, (C, w, g, t, k0, DF) in zip(jobs, host):
        nf, npix = j.X.shape
        rows, cols = synth.random_selection(9, nf, npix, 3, 5)
        Xo, Go, S = oracle_mod.maps_at(C, w, F0, DF, k0, g.cpu().numpy(), t.cpu().numpy(), rows, cols)
        Xg = j.X.cpu().numpy()[rows, cols]
        Gg = j.G.cpu().numpy()[rows, cols]
        assert x_error(Xg, Xo, S) <= 1e-5
        assert g_error(Gg, Go) <= 1e-4


def test_plan_rejects_bad_jobs(sg):
    jobs, _, _ = _make_jobs(sg)
    jobs[1].band = (5, 10_000)
    with pytest.raises(sg.SgwbError, match="band"):
        sg.Plan(jobs, autotune=False)
