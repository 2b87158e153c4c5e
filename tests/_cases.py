"""Seeded test cases shared by the GPU parity tests (host side, NumPy)."""
from __future__ import annotations

import numpy as np

import synth


def freqs(f0, df, k0, nf):
    return f0 + (k0 + np.arange(nf, dtype=np.float64)) * df


def make_csd(seed, nt, f, nonstationary=True, dtype=np.complex64):
    """Noise CSD and weights of the workload noise model (R13 variant: per-segment factor)."""
    C = synth.noise_csd(seed, nt, f, dtype=np.complex128)
    a_t = synth.segment_scale(nt, 100 + seed if nonstationary else None)
    w = synth.weights(f, a_t)
    rdt = np.float32 if dtype == np.complex64 else np.float64
    return C.astype(dtype), w.astype(rdt)


def x_error(Xg, Xo, S):
    """max |X_gpu - X_oracle| / S (S = sum_t |w gamma| |C|)."""
    return float(np.max(np.abs(np.asarray(Xg, np.float64) - Xo) / np.maximum(S, 1e-300)))


def g_error(Gg, Go):
    """max elementwise |G_gpu - G_oracle| / G_oracle (G >= 0)."""
    Go = np.asarray(Go, np.float64)
    return float(np.max(np.abs(np.asarray(Gg, np.float64) - Go) / np.maximum(Go, 1e-300)))
