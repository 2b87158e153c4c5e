"""The paper's own per-bin route to the narrowband maps (Secs. III.C-III.E).

TEST INFRASTRUCTURE ONLY.  For each frequency bin the overlap reduction
function is materialised from the two seed matrices (Fig. 3: the delay map
times 2 pi i f, exponentiated, multiplied pixel by pixel with the combined
antenna-pattern map), and the weighted CSD column for that bin is multiplied
with it (Sec. III.E), giving one narrowband map per bin.  Complex128 NumPy
matrix products; independent of the C loops in ``sgwb_oracle.c`` and meant for
small brute-force cross-checks (memory grows as nt * npix per bin).
"""
from __future__ import annotations

import numpy as np


def narrowband_maps(C, w, freqs, gamma, tau):
    """X[nf][npix] by materialised ORF per bin; the real part is kept."""
    C = np.asarray(C, dtype=np.complex128)
    w = np.asarray(w, dtype=np.float64)
    gamma = np.asarray(gamma, dtype=np.float64)
    tau = np.asarray(tau, dtype=np.float64)
    freqs = np.asarray(freqs, dtype=np.float64)
    x = w * C  # folded, weighted CSD (the x_{f t} of Eq. fwX with sigma^-2 inside w)
    out = np.empty((freqs.size, gamma.shape[1]))
    for k, f in enumerate(freqs):
        orf = gamma * np.exp(2j * np.pi * f * tau)  # [nt][npix]
        out[k] = (x[:, k] @ orf).real
    return out


def fisher_diagonal(w, gamma):
    """G[nf][npix] = W^T (gamma^2), a plain matrix product."""
    w = np.asarray(w, dtype=np.float64)
    gamma = np.asarray(gamma, dtype=np.float64)
    return w.T @ (gamma * gamma)
