"""The delay-grid spacing of the band-first broadband maps, checked on the CPU.

Y(tau) = sum_k y_k e^{2 pi i (k - kc) df tau} (one segment's band sum) is read
from its values on the nodes tau_j = (j - m - 1) h by 4-point Lagrange
interpolation.  The stated bound on the error is
(2 pi F h)^4 (9/16) / 24 * sum_k |y_k|,  F = (nb - 1) df / 2,
and the library takes 2 pi F h = 0.03, i.e. at most 1.9e-8 of sum_k |y_k|.
Checked here in float64 against the exact sum at random delays, for several
band widths, with the worst case (all y_k of one phase, so the top frequency
carries the whole sum) among them; a spacing twice as wide must give about 16x
the error (the fourth-order law)."""
import numpy as np
import pytest


def _interp_error(y, df, h, tau):
    nb = y.size
    kc = 0.5 * (nb - 1)
    k = np.arange(nb) - kc

    def Y(t):
        return np.exp(2j * np.pi * np.outer(t, k) * df) @ y

    u = tau / h
    j = np.floor(u)
    x = u - j
    nodes = (j[:, None] + np.array([-1.0, 0.0, 1.0, 2.0])[None, :]) * h
    vals = Y(nodes.ravel()).reshape(nodes.shape)
    L = np.stack([-x * (x - 1) * (x - 2) / 6, (x + 1) * (x - 1) * (x - 2) / 2,
                  -(x + 1) * x * (x - 2) / 2, (x + 1) * x * (x - 1) / 6], axis=1)
    return np.abs((L * vals).sum(axis=1) - Y(tau))


@pytest.mark.parametrize("nb, df", [(2, 1 / 32), (37, 1 / 32), (300, 1 / 32), (4096, 1 / 32), (40, 0.25)])
def test_spacing_meets_the_stated_bound(nb, df):
    rng = np.random.default_rng(nb)
    F = 0.5 * (nb - 1) * df
    h = 0.03 / (2 * np.pi * F)
    bound = (0.03 ** 4) * (9 / 16) / 24
    assert bound < 1.9e-8
    tau = rng.uniform(-0.03, 0.03, 400)
    for y in (rng.normal(size=nb) + 1j * rng.normal(size=nb),
              np.ones(nb, dtype=complex),  # one phase for every bin
              np.exp(2j * np.pi * rng.uniform(size=nb))):
        err = _interp_error(y, df, h, tau)
        assert err.max() <= bound * np.abs(y).sum() * (1 + 1e-6) + 1e-13 * np.abs(y).sum()


def test_error_follows_the_fourth_power_of_the_spacing():
    rng = np.random.default_rng(5)
    nb, df = 512, 1 / 32
    F = 0.5 * (nb - 1) * df
    y = rng.normal(size=nb) + 1j * rng.normal(size=nb)
    tau = rng.uniform(-0.02, 0.02, 2000)
    e1 = _interp_error(y, df, 0.03 / (2 * np.pi * F), tau).max()
    e2 = _interp_error(y, df, 0.06 / (2 * np.pi * F), tau).max()
    assert 8.0 < e2 / e1 < 32.0
