"""Both wave-tile shapes of the beam GEMM give the same bits.

The 2x4 shape (default) shares the pixel-side fragments of a workgroup through
LDS; the 4x4 shape (picked by the plan autotuner, or SGWB_BEAM_SHAPE=4x4 for
single calls) reads both operands per wave.  Every output accumulates the
same products in the same order in both, so Gamma must be bitwise equal.  The
shape of single calls is read once per process, so the 4x4 side runs in a
child process on the same inputs.  Cases cover ragged bin and pixel blocks
(padding blocks of the fragment arrays) and 1, 2, 3 and 4 K-steps (every
tail of the K loop, which is unrolled by three).  The 2x4 results are checked
against the oracle elsewhere.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

import synth
from tests._cases import freqs, make_csd

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CASES = [  # baseline, nside, nf, nt, antipodal
    ("AC", 16, 203, 61, True),   # 7 bin blocks, 4 K-steps
    ("AB", 8, 96, 33, True),     # 3 bin blocks, 3 K-steps
    ("BC", 4, 300, 17, False),   # 10 bin blocks, 2 K-steps, no antipodal pairs
    ("AB", 2, 31, 5, True),      # one partial block, one K-step
]

CHILD = r"""
import sys, numpy as np, torch
sys.path.insert(0, sys.argv[1])
import paper_1803_08285_amd as sg
d = np.load(sys.argv[2])
out = {}
for i in range(int(d["n"])):
    w = torch.from_numpy(d[f"w{i}"]).cuda()
    g = torch.from_numpy(d[f"g{i}"]).cuda()
    t = torch.from_numpy(d[f"t{i}"]).cuda()
    C = torch.zeros(w.shape, dtype=torch.complex64, device="cuda")
    _, G = sg.make_maps(C, w, sg.FGrid(20.0, 0.25), 0, g, t, antipodal=bool(d[f"a{i}"]), want_x=False)
    torch.cuda.synchronize()
    out[f"G{i}"] = G.cpu().numpy()
np.savez(sys.argv[3], **out)
print("child done", flush=True)
"""


@pytest.fixture(scope="module")
def sg():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    import paper_1803_08285_amd as sg

    return sg


def test_beam_4x4_matches_2x4_bitwise(sg, tmp_path):
    inputs, ref = {"n": len(CASES)}, []
    for i, (bl, nside, nf, nt, anti) in enumerate(CASES):
        tg = sg.TGrid(nt, 0.0, 86164.0905 / nt, 86164.0905 / nt)
        g, t = sg.build_geometry(synth.baseline_sites(bl), nside, tg)
        _, w = make_csd(11 + i, nt, freqs(20.0, 0.25, 0, nf))
        wt = torch.from_numpy(w).cuda()
        C = torch.zeros(wt.shape, dtype=torch.complex64, device="cuda")
        _, G = sg.make_maps(C, wt, sg.FGrid(20.0, 0.25), 0, g, t, antipodal=anti, want_x=False)
        torch.cuda.synchronize()
        ref.append(G.cpu().numpy())
        inputs.update({f"w{i}": w, f"g{i}": g.cpu().numpy(), f"t{i}": t.cpu().numpy(), f"a{i}": anti})
    src, dst = tmp_path / "in.npz", tmp_path / "out.npz"
    np.savez(src, **inputs)
    env = dict(os.environ, SGWB_BEAM_SHAPE="4x4")
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, str(src), str(dst)], env=env, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    got = np.load(dst)
    for i, G in enumerate(ref):
        assert np.array_equal(got[f"G{i}"], G), f"case {CASES[i]}"
