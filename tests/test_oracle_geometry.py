"""Pins for the oracle's ORF seeds gamma(t,p), tau(t,p) (Sec. III.D, Fig. 3).

What fixes them besides the oracle itself:
  * textbook antenna patterns of a detector with arms along x and y
    (F+ = -(1 + cos^2 theta) cos 2 phi / 2, Fx = cos theta sin 2 phi with the
    oracle's polarisation basis m = (sin phi, -cos phi, 0),
    n = (cos theta cos phi, cos theta sin phi, -sin theta); F+^2 + Fx^2 is basis-free);
  * the projector identity sum_A F^A_1 F^A_2 = 2 tr(P D1 P D2) - tr(P D1) tr(P D2),
    P = I - Omega Omega^T (a different formula from the oracle's explicit basis);
  * a co-located, co-aligned pair averages to 2/5 over the sky;
  * the normalised isotropic overlap (5 / 8 pi) int gamma cos(2 pi f tau) of the
    LIGO Hanford-Livingston pair: about -0.89 at f = 0, first zero near 64 Hz
    (textbook values, e.g. Flanagan 1993; Allen & Romano 1999), and it does not
    change with sidereal time;
  * antipodal symmetry gamma(-Omega) = gamma(Omega), tau(-Omega) = -tau(Omega);
  * |tau| <= |x_1 - x_2| / c, reached in the chord direction with a + sign;
  * the sidereal period and the eastward rotation sense.
"""
import numpy as np
import pytest

import synth

C = 299792458.0
R_E = 6.371e6


def test_detector_tensor_properties(oracle_mod):
    for site in synth.DETECTORS.values():
        r, D = oracle_mod.detector(*site)
        np.testing.assert_allclose(np.linalg.norm(r), R_E, rtol=1e-15)
        np.testing.assert_allclose(D, D.T, atol=1e-16)
        assert abs(np.trace(D)) < 1e-15
        np.testing.assert_allclose(D @ (r / R_E), 0.0, atol=1e-15)  # arms horizontal
        np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(D)), [-0.5, 0.0, 0.5], atol=1e-15)


@pytest.mark.parametrize("theta,phi", [(0.3, 0.2), (1.1, 2.5), (2.0, -1.0), (np.pi / 2, 0.7)])
def test_textbook_antenna_patterns(oracle_mod, theta, phi):
    D = 0.5 * (np.diag([1.0, 0, 0]) - np.diag([0, 1.0, 0]))
    fp, fx = oracle_mod.antenna(D, theta, phi)
    ct = np.cos(theta)
    np.testing.assert_allclose(fp, -0.5 * (1 + ct * ct) * np.cos(2 * phi), atol=1e-15)
    np.testing.assert_allclose(fx, ct * np.sin(2 * phi), atol=1e-15)
    # basis-free: F+^2 + Fx^2 = (1 + c^2)^2 cos^2 2phi / 4 + c^2 sin^2 2phi
    want = 0.25 * (1 + ct * ct) ** 2 * np.cos(2 * phi) ** 2 + ct * ct * np.sin(2 * phi) ** 2
    np.testing.assert_allclose(fp * fp + fx * fx, want, atol=1e-15)


def _projector_gamma(DA, DB, omega):
    P = np.eye(3)[None] - omega[:, :, None] * omega[:, None, :]
    PA = P @ DA
    PB = P @ DB
    return 2 * np.einsum("nij,nji->n", PA, PB) - np.trace(PA, axis1=1, axis2=2) * np.trace(PB, axis1=1, axis2=2)


def _rotz(th):
    c, s = np.cos(th), np.sin(th)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1.0]])


@pytest.mark.parametrize("bl", ["AB", "AC", "BC"])
def test_projector_identity_and_tau(oracle_mod, bl):
    det = synth.baseline_sites(bl)
    nside, nt, stride = 4, 5, 9000.0
    g, tau = oracle_mod.geometry(det, nside, nt, 0.0, stride, stride)
    om = oracle_mod.healpix_centres(nside)
    rA, DA = oracle_mod.detector(*det[:3])
    rB, DB = oracle_mod.detector(*det[3:])
    for k in range(nt):
        th = 2 * np.pi * (k * stride + stride / 2) / 86164.0905
        R = _rotz(th)
        want = _projector_gamma(R @ DA @ R.T, R @ DB @ R.T, om)
        np.testing.assert_allclose(g[k], want, atol=1e-14)
        np.testing.assert_allclose(tau[k], om @ (R @ (rA - rB)) / C, atol=1e-18)


def test_colocated_sky_average_two_fifths(oracle_mod):
    site = synth.DETECTORS["A"]
    g, _ = oracle_mod.geometry(site + site, 16, 3, 0.0, 20000.0, 20000.0)
    np.testing.assert_allclose(g.mean(axis=1), 0.4, atol=2e-4)


def test_isotropic_overlap_hanford_livingston(oracle_mod):
    nside = 16
    g, tau = oracle_mod.geometry(synth.baseline_sites("AB"), nside, 6, 0.0, 13000.0, 100.0)
    npix = 12 * nside * nside

    def overlap(f):
        return (5 / (8 * np.pi)) * (4 * np.pi / npix) * np.sum(g * np.cos(2 * np.pi * f * tau), axis=1)

    o0 = overlap(0.0)
    assert np.all(np.abs(o0 + 0.89) < 0.01)
    # rotation-invariant up to the pixel quadrature error
    np.testing.assert_allclose(o0, o0[0], rtol=1e-7)
    fs = np.arange(40.0, 90.0, 0.25)
    vals = np.array([overlap(f)[0] for f in fs])
    first_zero = fs[np.argmax(vals > 0)]
    assert 60.0 <= first_zero <= 68.0
    for f in (30.0, 100.0):
        o = overlap(f)
        np.testing.assert_allclose(o, o[0], atol=1e-6)


@pytest.mark.parametrize("nside", [2, 8])
def test_antipodal_seeds(oracle_mod, nside):
    g, tau = oracle_mod.geometry(synth.baseline_sites("AC"), nside, 4, 0.0, 7000.0, 7000.0)
    om = oracle_mod.healpix_centres(nside)
    q = np.argmax(om @ (-om).T, axis=1)
    np.testing.assert_allclose(g[:, q], g, atol=1e-15)
    np.testing.assert_allclose(tau[:, q], -tau, atol=1e-17)


@pytest.mark.parametrize("bl,chord_km", [("AB", 2995.8), ("AC", 8156.5), ("BC", 7911.8)])
def test_delay_bounds_and_sign(oracle_mod, bl, chord_km):
    det = synth.baseline_sites(bl)
    rA, _ = oracle_mod.detector(*det[:3])
    rB, _ = oracle_mod.detector(*det[3:])
    d = np.linalg.norm(rA - rB)
    np.testing.assert_allclose(d / 1e3, chord_km, atol=0.1)
    _, tau = oracle_mod.geometry(det, 16, 3, 0.0, 30000.0, 0.0)
    assert np.all(np.abs(tau) <= d / C * (1 + 1e-15))
    assert np.max(np.abs(tau)) > 0.99 * d / C
    # At t = 0 (no rotation) the direction of x_A - x_B gives tau = +|dx| / c:
    # a single pixel is placed there by building the geometry for nside 1 and
    # comparing the sign of tau with the dot product of the centres with dx.
    g1, tau1 = oracle_mod.geometry(det, 1, 1, 0.0, 0.0, 0.0)
    om = oracle_mod.healpix_centres(1)
    np.testing.assert_allclose(tau1[0], om @ (rA - rB) / C, atol=1e-18)


def test_sidereal_period_and_rotation_sense(oracle_mod):
    """Geometry is periodic in T_s, and time t equals moving both sites east by 2 pi t / T_s."""
    det = np.array(synth.baseline_sites("AB"))
    Ts = 86164.0905
    g0, t0 = oracle_mod.geometry(det, 4, 3, 0.0, 5000.0, 0.0)
    g1, t1 = oracle_mod.geometry(det, 4, 3, Ts, 5000.0, 0.0)
    np.testing.assert_allclose(g1, g0, atol=1e-12)
    np.testing.assert_allclose(t1, t0, atol=1e-15)
    dt = 10000.0
    moved = det.copy()
    moved[1] += 360.0 * dt / Ts
    moved[4] += 360.0 * dt / Ts
    ga, ta = oracle_mod.geometry(det, 4, 1, dt, 0.0, 0.0)
    gb, tb = oracle_mod.geometry(moved, 4, 1, 0.0, 0.0, 0.0)
    np.testing.assert_allclose(ga, gb, atol=1e-13)
    np.testing.assert_allclose(ta, tb, atol=1e-16)


def test_seed_matrix_size_model():
    """Sec. III.E / IV: two 3072 x 3314 real seed matrices are ~156 MB in float64,
    and 3314 half-overlapping 52 s frames span one sidereal day."""
    assert abs(2 * 3072 * 3314 * 8 / 2**20 - 155.3) < 0.1
    assert abs(3314 * 26 - 86164) < 26
    # Sec. III.D: the full ORF (complex128, 1920 bins of 0.25 Hz) would take ~292 GB.
    assert abs(3314 * 3072 * 1920 * 16 / 2**30 - 291.3) < 0.1
