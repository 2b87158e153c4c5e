"""Network sums and directed/isotropic contractions (Sec. V) on the GPU against
the oracle: float64 sums rounded once, so within one float32 ulp of the sum of
absolute values."""
import numpy as np
import pytest

import synth
from tests._cases import freqs, make_csd, x_error

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sg():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1803_08285_amd as sg

    return sg


def test_network_sum_vs_oracle(sg, oracle_mod):
    rng = np.random.default_rng(3)
    maps = [rng.standard_normal((33, 3072)).astype(np.float32) for _ in range(3)]
    out = sg.network_sum([torch.from_numpy(m).cuda() for m in maps]).cpu().numpy()
    ref = oracle_mod.network_sum(maps)
    scale = oracle_mod.network_sum([np.abs(m) for m in maps])
    assert np.all(np.abs(out - ref) <= 2.0 ** -23 * scale)


@pytest.mark.parametrize("shape,offset", [((5, 7), 0), ((33, 3072), 1), ((4, 4096), 0)])
def test_network_sum_scalar_and_vector_paths(sg, oracle_mod, shape, offset):
    """Sizes not a multiple of 4 and maps not 16-byte aligned take the scalar
    kernel, the rest the 16-byte one; both give the oracle's float64 sums."""
    rng = np.random.default_rng(shape[1] + offset)
    n = shape[0] * shape[1]
    maps = [rng.standard_normal(n + offset).astype(np.float32) for _ in range(4)]
    dev = [torch.from_numpy(m).cuda()[offset:] for m in maps]
    out = sg.network_sum(dev).cpu().numpy()
    ref = oracle_mod.network_sum([m[offset:] for m in maps])
    scale = oracle_mod.network_sum([np.abs(m[offset:]) for m in maps])
    assert np.all(np.abs(out - ref) <= 2.0 ** -23 * scale)


@pytest.mark.parametrize("npix,sel", [(768, [100]), (12288, [5, 77, 4000, 12287]), (3072, None), (49152, None)])
def test_contractions_vs_oracle(sg, oracle_mod, npix, sel):
    rng = np.random.default_rng(npix)
    M = rng.standard_normal((21, npix)).astype(np.float32)
    pix = None if sel is None else torch.tensor(sel, device="cuda")
    out = sg.contract_pixels(torch.from_numpy(M).cuda(), pix).cpu().numpy()
    ref = oracle_mod.contract(M, None if sel is None else np.array(sel))
    scale = oracle_mod.contract(np.abs(M), None if sel is None else np.array(sel))
    assert np.all(np.abs(out - ref) <= 2.0 ** -23 * scale)


def test_directed_search_recovers_an_injected_source(sg):
    """Through the whole GPU path: X of a noise-free source at p0, contracted over
    {p0}, equals A H Gamma(k,p0) within the dirty-map tolerance."""
    nside, nt, nf, df = 8, 48, 128, 1 / 32
    tg = sg.TGrid(nt, 0.0, 86164.0905 / nt, 86164.0905 / nt)
    g, t = sg.build_geometry(synth.baseline_sites("AB"), nside, tg)
    f = freqs(20.0, df, 0, nf)
    w = synth.weights(f, np.ones(nt)).astype(np.float32)
    C = np.zeros((nt, nf), dtype=np.complex128)
    p0 = 300
    synth.add_point_source(C, f, 0.1, g[:, p0].cpu().numpy(), t[:, p0].cpu().numpy())
    X, G = sg.make_maps(torch.from_numpy(C.astype(np.complex64)).cuda(), torch.from_numpy(w).cuda(),
                        sg.FGrid(20.0, df), 0, g, t)
    d = sg.contract_pixels(X, torch.tensor([p0], device="cuda")).cpu().numpy().astype(np.float64)
    ref = 0.1 * synth.spectrum_H(f) * G[:, p0].cpu().numpy().astype(np.float64)
    S = 0.1 * synth.spectrum_H(f) * np.sum(w * np.abs(g[:, p0].cpu().numpy()[:, None]) ** 2, axis=0)
    assert np.max(np.abs(d - ref) / S) <= 1e-4  # X (1e-5) and the split-bf16 Gamma (1e-4)
