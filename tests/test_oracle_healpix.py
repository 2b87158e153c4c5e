"""Pins for the oracle's HEALPix RING centres (Sec. III.B).

Closed forms of the HEALPix tessellation (Gorski et al. 2005): 12 nside^2
pixels on 4 nside - 1 iso-latitude rings, ring heights, pixels per ring,
uniform azimuthal spacing, the nside = 1 base pixels (golden fixture),
antipodal closure of the centre set and the equal-area quadrature property.
"""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def ring_table(nside):
    """(ring z, pixels per ring) from the closed form, north to south."""
    out = []
    for i in range(1, 4 * nside):
        ni = i if i <= 2 * nside else 4 * nside - i
        if ni < nside:
            z, n = 1 - ni * ni / (3 * nside * nside), 4 * ni
        else:
            z, n = 4 / 3 - 2 * ni / (3 * nside), 4 * nside
        out.append((z if i <= 2 * nside else -z, n))
    return out


@pytest.mark.parametrize("nside", [1, 2, 4, 8, 16, 32])
def test_counts_rings_and_heights(oracle_mod, nside):
    xyz = oracle_mod.healpix_centres(nside)
    assert xyz.shape == (12 * nside * nside, 3)
    np.testing.assert_allclose(np.linalg.norm(xyz, axis=1), 1.0, atol=1e-15)
    p = 0
    for z, n in ring_table(nside):
        ring = xyz[p:p + n]
        np.testing.assert_allclose(ring[:, 2], z, atol=1e-15)
        phi = np.unwrap(np.arctan2(ring[:, 1], ring[:, 0]))
        np.testing.assert_allclose(np.diff(phi), 2 * np.pi / n, atol=1e-12)
        p += n
    assert p == 12 * nside * nside
    assert len(ring_table(nside)) == 4 * nside - 1


def test_base_pixels_golden(oracle_mod):
    ref = np.loadtxt(os.path.join(GOLDEN, "healpix_nside1_ring.txt"))
    xyz = oracle_mod.healpix_centres(1)
    z = ref[:, 1]
    phi = ref[:, 2] * np.pi
    st = np.sqrt(1 - z * z)
    want = np.c_[st * np.cos(phi), st * np.sin(phi), z]
    np.testing.assert_allclose(xyz, want, atol=1e-15)


@pytest.mark.parametrize("nside", [1, 2, 4, 8])
def test_antipodal_closure(oracle_mod, nside):
    """Every centre's antipode is a centre; pixel p < npix/2 maps into the other half."""
    xyz = oracle_mod.healpix_centres(nside)
    npix = xyz.shape[0]
    d = xyz @ (-xyz).T  # cos of angle between p and -q
    q = np.argmax(d, axis=1)
    np.testing.assert_allclose(d[np.arange(npix), q], 1.0, atol=1e-13)
    assert np.all(q[: npix // 2] >= npix // 2)
    assert np.array_equal(q[q], np.arange(npix))


@pytest.mark.parametrize("nside", [4, 8, 16])
def test_equal_area_quadrature(oracle_mod, nside):
    """Equal-area pixels: (4 pi / npix) sum f(Omega_p) -> integral of f.

    Monopole, dipole and quadrupole moments: sum z = 0 and sum x = sum y = 0
    exactly (symmetry); mean z^2 -> 1/3 with an O(1/npix) error.
    """
    xyz = oracle_mod.healpix_centres(nside)
    npix = xyz.shape[0]
    np.testing.assert_allclose(xyz.sum(axis=0), 0.0, atol=1e-11)
    m2 = (xyz[:, :, None] * xyz[:, None, :]).mean(axis=0)
    np.testing.assert_allclose(m2, np.eye(3) / 3, atol=2.0 / npix)
