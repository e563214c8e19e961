"""Pins for the oracle's HEALPix directions and split radius (section 2.1 and 2.4: ray
directions from the HEALPix nested scheme, children at the next level).

The pins do not reuse the oracle's own formulas: closed-form level-0 centres, ring
structure, invariants (unit norm, zero sum, 4-fold symmetry), and a round trip through an
independent nested ang2pix written here from the published scheme (Gorski et al. 2005)."""
import math

import numpy as np
import pytest

import oracle


def ang2pix_nest(level: int, v: np.ndarray) -> np.ndarray:
    """Nested pixel index of unit vectors v [n,3] (Gorski et al. 2005, sections 4-5):
    locate the base face from the position relative to the face edges, then the
    (x, y) position inside the face, then interleave the bits."""
    ns = 1 << level
    z = v[:, 2] / np.linalg.norm(v, axis=1)
    phi = np.arctan2(v[:, 1], v[:, 0])
    tt = np.mod(phi / (np.pi / 2), 4.0)
    za = np.abs(z)
    out = np.empty(len(v), np.int64)
    for i in range(len(v)):
        if za[i] <= 2.0 / 3.0:
            # equatorial region: edges are the lines phi/(pi/2) +- 3z/4 = const
            t1 = ns * (0.5 + tt[i])
            t2 = ns * z[i] * 0.75
            jp = int(math.floor(t1 - t2))
            jm = int(math.floor(t1 + t2))
            ifp, ifm = jp // ns, jm // ns
            if ifp == ifm:
                face = (ifp % 4) + 4
            elif ifp < ifm:
                face = ifp % 4
            else:
                face = (ifm % 4) + 8
            ix = jm % ns
            iy = ns - (jp % ns) - 1
        else:
            ntt = min(3, int(tt[i]))
            tp = tt[i] - ntt
            tmp = ns * math.sqrt(3.0 * (1.0 - za[i]))
            jp = min(int(tp * tmp), ns - 1)
            jm = min(int((1.0 - tp) * tmp), ns - 1)
            if z[i] >= 0:
                face, ix, iy = ntt, ns - jm - 1, ns - jp - 1
            else:
                face, ix, iy = ntt + 8, jp, jm
        p = 0
        for b in range(level):
            p |= ((ix >> b) & 1) << (2 * b)
            p |= ((iy >> b) & 1) << (2 * b + 1)
        out[i] = face * ns * ns + p
    return out


def centres(level):
    return oracle.healpix_vec(level, np.arange(oracle.npix(level)))


def test_npix_and_level1_is_48_rays():
    # section 2.1: "typically HEALPix level 1, or 48 photon packets"
    assert [oracle.npix(l) for l in range(5)] == [12, 48, 192, 768, 3072]


def test_level0_closed_form():
    v = centres(0)
    z23 = 2.0 / 3.0
    for f in range(12):
        if f < 4:
            z, phi = z23, math.pi / 4 + f * math.pi / 2
        elif f < 8:
            z, phi = 0.0, (f - 4) * math.pi / 2
        else:
            z, phi = -z23, math.pi / 4 + (f - 8) * math.pi / 2
        st = math.sqrt(1 - z * z)
        np.testing.assert_allclose(v[f], [st * math.cos(phi), st * math.sin(phi), z], atol=1e-15)
    # the four equatorial centres lie exactly on the axes
    assert np.array_equal(v[4], [1.0, 0.0, 0.0])
    assert np.array_equal(np.abs(v[5]), [0.0, 1.0, 0.0])


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4, 5])
def test_invariants(level):
    v = centres(level)
    assert len(v) == 12 * 4 ** level
    np.testing.assert_allclose(np.linalg.norm(v, axis=1), 1.0, atol=2e-16 * 4)
    assert len(np.unique(np.round(v, 12), axis=0)) == len(v)
    assert np.abs(v.sum(axis=0)).max() < 1e-12


@pytest.mark.parametrize("level", [1, 2, 3, 4])
def test_ring_structure(level):
    """Pixel centres sit on 4 Nside - 1 rings of constant z: polar-cap ring i holds 4i
    pixels at z = 1 - i^2/(3 Nside^2), belt ring i holds 4 Nside at 4/3 - 2i/(3 Nside)."""
    ns = 1 << level
    v = centres(level)
    zs, counts = np.unique(np.round(v[:, 2], 12), return_counts=True)
    expect = {}
    for i in range(1, ns):
        expect[round(1 - i * i / (3 * ns * ns), 12)] = 4 * i
        expect[round(-(1 - i * i / (3 * ns * ns)), 12)] = 4 * i
    for i in range(ns, 3 * ns + 1):
        expect[round(4 / 3 - 2 * i / (3 * ns), 12)] = 4 * ns
    assert dict(zip(zs.tolist(), counts.tolist())) == pytest.approx(expect)


def test_fourfold_symmetry():
    v = centres(3)
    rot = np.stack([-v[:, 1], v[:, 0], v[:, 2]], axis=1)
    a = np.round(v, 11)
    b = np.round(rot, 11) + 0.0
    assert {tuple(r) for r in a} == {tuple(r) for r in b}


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4, 5])
def test_round_trip_independent_ang2pix(level):
    v = centres(level)
    assert np.array_equal(ang2pix_nest(level, v), np.arange(len(v)))


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_children_lie_in_parent(level):
    """Nested scheme: the children of pixel p are 4p .. 4p+3 and lie inside p."""
    child = centres(level + 1)
    assert np.array_equal(ang2pix_nest(level, child), np.arange(len(child)) // 4)


def test_equal_area():
    """Uniform directions fall evenly into the pixels (chi-square, level 2)."""
    rng = np.random.default_rng(7)
    n = 192 * 200
    u = rng.standard_normal((n, 3))
    counts = np.bincount(ang2pix_nest(2, u), minlength=192)
    chi2 = ((counts - 200.0) ** 2 / 200.0).sum()
    assert chi2 < 191 + 5 * math.sqrt(2 * 191)


def test_t_split_solid_angle():
    """Split radius: the ray's cross-section equals one cell face over Phi."""
    for phi in (1.0, 3.0, 4.0, 16.0):
        for level in range(0, 13):
            r = oracle.t_split(phi, level)
            area = 4 * math.pi / (12 * 4 ** level) * r * r
            assert area == pytest.approx(1.0 / phi, rel=2e-7)
    assert oracle.t_split(4.0, 0) == pytest.approx(math.sqrt(3 / (4 * math.pi)), rel=1e-7)


def test_auto_max_level():
    # smallest level whose split radius reaches the box diagonal
    for n, lmax in [(64, 8), (128, 9), (256, 10), (512, 11), (1024, 12)]:
        assert oracle.auto_max_level((n, n, n), 4.0) == lmax
        assert oracle.t_split(4.0, lmax) >= math.sqrt(3) * n > oracle.t_split(4.0, lmax - 1)
