"""Folding (Sec. II.B) on the GPU against the FP64 oracle, through the C ABI.
The kernel sums in float64 in the oracle's order and rounds once to float32, so
each output is within half a float32 ulp of its scale (sum of absolute terms)."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

W = synth.HANN_OVERLAP_W


@pytest.fixture(scope="module")
def sg():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1803_08285_amd as sg

    return sg


def _days(seed, ndays, nt, nf, p_missing):
    rng = np.random.default_rng(seed)
    present = synth.day_presence(seed + 1, ndays, nt, p_missing)
    s = (rng.uniform(0.5, 2.0, (ndays, nt, nf)) * present[:, :, None]).astype(np.float32)
    C = ((rng.standard_normal((ndays, nt, nf)) + 1j * rng.standard_normal((ndays, nt, nf)))
         * present[:, :, None]).astype(np.complex64)
    return C, s, present


# nt = 37 and 898 leave a ragged last group of the four segments a thread
# folds; nt = 3 and 1 are a single ragged group (every neighbour in another day)
@pytest.mark.parametrize("ndays,nt,nf,p_missing", [(5, 37, 300, 0.1), (1, 16, 256, 0.0), (3, 8, 1, 0.3),
                                                    (2, 898, 70, 0.02), (4, 3, 50, 0.2), (3, 1, 40, 0.0)])
def test_fold_vs_oracle(sg, oracle_mod, ndays, nt, nf, p_missing):
    C, s, present = _days(7 + nt, ndays, nt, nf, p_missing)
    v, u, w, x = sg.fold(torch.from_numpy(C).cuda(), torch.from_numpy(s).cuda(), torch.from_numpy(present).cuda(), W)
    torch.cuda.synchronize()
    vo, uo, wo, xo = oracle_mod.fold(C, s, present, W)
    _, ua, wa, xa = oracle_mod.fold(np.abs(C), s, present, -W)  # scales: sums of absolute terms
    half_ulp = 2.0 ** -24 * (1 + 1e-9)
    for got, ref, scale in ((v, vo, vo), (u, uo, np.abs(ua)), (w, wo, np.abs(wa))):
        g = got.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(g - ref) <= half_ulp * scale + 1e-30)
    xg = x.cpu().numpy().astype(np.complex128)
    assert np.all(np.abs(xg.real - xo.real) <= half_ulp * xa.real + 1e-30)
    assert np.all(np.abs(xg.imag - xo.imag) <= half_ulp * xa.real + 1e-30)
    if ndays == 1:
        assert not u.cpu().numpy()[0].any() and not w.cpu().numpy()[-1].any()


def test_fold_column_window(sg, oracle_mod):
    """A window of bins of wider arrays (row stride > nf) folds like the dense copy."""
    C, s, present = _days(3, 3, 20, 200, 0.1)
    Cd, sd = torch.from_numpy(C).cuda(), torch.from_numpy(s).cuda()
    pd = torch.from_numpy(present).cuda()
    full = sg.fold(Cd, sd, pd, W)
    win = sg.fold(Cd[:, :, 50:130], sd[:, :, 50:130], pd, W)
    torch.cuda.synchronize()
    for a, b in zip(full, win):
        assert torch.equal(a[:, 50:130], b)
