"""Pins of the seeded input generators against mathematics (no oracle involved)."""
import math

import numpy as np
import pytest

from paper_2205_08417_amd import inputs as I


@pytest.mark.parametrize("npol,naz", [(8, 8), (16, 16), (32, 32), (16, 32), (3, 5)])
def test_product_quadrature_moments(npol, naz):
    omega, w = I.product_quadrature(npol, naz)
    assert omega.shape == (npol * naz, 3) and w.shape == (npol * naz,)
    np.testing.assert_allclose(np.linalg.norm(omega, axis=1), 1.0, rtol=0, atol=1e-15)
    # exact integrals over the unit sphere
    assert abs(w.sum() - 4 * math.pi) <= 4e-15 * 4 * math.pi
    mu = omega[:, 2]
    np.testing.assert_allclose(np.sum(w * mu * mu), 4 * math.pi / 3, rtol=1e-14)
    if npol >= 3:
        np.testing.assert_allclose(np.sum(w * mu ** 4), 4 * math.pi / 5, rtol=1e-14)
    if naz >= 3:
        np.testing.assert_allclose(np.sum(w * omega[:, 0] ** 2), 4 * math.pi / 3, rtol=1e-13)
        np.testing.assert_allclose(np.sum(w * omega[:, 1] ** 2), 4 * math.pi / 3, rtol=1e-13)
    for a, b in [(0, 1), (0, 2), (1, 2)]:
        assert abs(np.sum(w * omega[:, a] * omega[:, b])) < 1e-13
    for a in range(3):
        assert abs(np.sum(w * omega[:, a])) < 1e-13


def test_product_quadrature_layout_matches_paper():
    """phi_l = l*2pi/N (l=1..N), w = 2 pi w^G_k / N, polar index outer (Sec. 3.2)."""
    omega, w = I.product_quadrature(2, 4)
    # two-point Gauss rule: mu = -+1/sqrt(3), weights 1
    mu = omega[:, 2]
    np.testing.assert_allclose(mu[:4], -1 / math.sqrt(3), rtol=1e-15)
    np.testing.assert_allclose(mu[4:], 1 / math.sqrt(3), rtol=1e-15)
    np.testing.assert_allclose(w, 2 * math.pi / 4, rtol=1e-15)
    st = math.sqrt(1 - 1 / 3)
    phi = np.array([1, 2, 3, 4]) * math.pi / 2
    np.testing.assert_allclose(omega[:4, 0], st * np.sin(phi), atol=1e-15)
    np.testing.assert_allclose(omega[:4, 1], st * np.cos(phi), atol=1e-15)


@pytest.mark.parametrize("n,lo,hi,seed,line", [(12, -1.5, 1.5, 7, None), (15, 0.0, 7.0, 3, 2),
                                               (45, -1.5, 1.5, 1001, None)])
def test_jittered_mesh_geometry(n, lo, hi, seed, line):
    m = I.jittered_delaunay_mesh(n, lo, hi, seed, line_every=line)
    nc = m.ncells
    assert nc == 2 * n * n - 4 * (n - 1) - 2
    assert np.all(m.area > 0)
    np.testing.assert_allclose(m.area.sum(), (hi - lo) ** 2, rtol=1e-13)
    # closed cells: outward normals times length sum to zero
    closure = m.face_normal.sum(axis=1)
    assert np.max(np.abs(closure)) < 1e-14 * (hi - lo)
    # interior faces: neighbour holds the exact negation; adjacency is symmetric
    nb = m.face_nbr
    for c in range(nc):
        for f in range(3):
            j = nb[c, f]
            if j >= 0:
                fj = np.nonzero(nb[j] == c)[0]
                assert fj.size == 1
                assert np.array_equal(m.face_normal[j, fj[0]], -m.face_normal[c, f])
    # boundary faces: numbered 0..nbf-1 once each, total length = perimeter
    b = -1 - nb[nb < 0]
    assert np.array_equal(np.sort(b), np.arange(4 * (n - 1)))
    blen = np.linalg.norm(m.face_normal[nb < 0], axis=1).sum()
    np.testing.assert_allclose(blen, 4 * (hi - lo), rtol=1e-13)


def test_four_triangle_mesh_matches_fixture():
    import json
    import os
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "four_triangles.json")))
    m = I.four_triangle_mesh()
    assert np.array_equal(m.face_nbr, np.array(d["face_nbr"]))
    assert np.array_equal(m.face_normal, np.array(d["face_normal"]))
    assert np.array_equal(m.area, np.array(d["area"]))


def test_periodic_mesh():
    m = I.periodic_mesh(5, 2.0)
    assert m.ncells == 50 and m.nbfaces == 0
    assert np.all(m.face_nbr >= 0)
    assert np.max(np.abs(m.face_normal.sum(axis=1))) == 0.0
    np.testing.assert_allclose(m.area, 0.5 * (2.0 / 5) ** 2, rtol=1e-15)
    for c in range(m.ncells):
        for f in range(3):
            j = m.face_nbr[c, f]
            fj = np.nonzero(m.face_nbr[j] == c)[0]
            assert any(np.array_equal(m.face_normal[j, k], -m.face_normal[c, f]) for k in fj)


@pytest.mark.parametrize("g", [0.5, 0.9, 0.95])
def test_hg_kernel_normalisation(g):
    omega, w = I.product_quadrature(8, 16)
    K = I.henyey_greenstein_kernel(omega, w, g)
    np.testing.assert_allclose(w @ K, 1.0, rtol=1e-14)
    assert not np.allclose(K, K.T)          # column scaling breaks symmetry
    K0 = I.henyey_greenstein_kernel(omega, w, 0.0)
    np.testing.assert_allclose(K0, 1 / (4 * math.pi), rtol=1e-14)


def test_hg_kernel_unnormalised_integrates_to_one():
    """For a mildly peaked kernel the raw HG density already integrates to ~1 on S^2."""
    omega, w = I.product_quadrature(32, 64)
    K = I.henyey_greenstein_kernel(omega, w, 0.3, normalise=False)
    np.testing.assert_allclose(w @ K, 1.0, rtol=1e-6)


def test_csd_energy_transform():
    from scipy.integrate import quad
    for E in [0.1, 1.0, 7.5, 19.9]:
        ref = quad(lambda e: 1.0 / (2.0 * e ** -0.3), E, 20.0, epsabs=0, epsrel=1e-13)[0]
        np.testing.assert_allclose(I.csd_pseudo_time(E), ref, rtol=1e-11)
        np.testing.assert_allclose(I.csd_energy(I.csd_pseudo_time(E)), E, rtol=1e-12)
    np.testing.assert_allclose(I.csd_pseudo_time(0.1), 18.877, rtol=1e-4)


def test_checkerboard_layout():
    ab = I.checkerboard_absorbers()
    assert len(ab) == 11 and (3, 3) not in ab and (3, 5) not in ab
    P = I.build("checkerboard_s16", n_side=36, nsteps=5)
    assert P.ncells == 2 * 36 * 36 - 4 * 35 - 2
    absorb = P.sigma_t == 10.0
    # each absorber is 1 unit^2 of the 49 unit^2 domain; centroid assignment is close
    np.testing.assert_allclose(P.mesh.area[absorb].sum(), 11.0, rtol=0.02)
    np.testing.assert_allclose(P.mesh.area[P.source > 0].sum(), 1.0, rtol=0.05)
    assert np.all(P.sigma_s[absorb] == 0) and np.all(P.sigma_s[~absorb] == 1)


def test_cfl_dt_bound():
    P = I.build("linesource_s8", n_side=20, nsteps=1)
    n = P.mesh.face_normal
    s = np.einsum("cfd,qd->cfq", n, P.omega[:, :2])
    out = np.maximum(s, 0).sum(axis=1)                    # [nc, nq]
    ratio = P.dt * out / P.mesh.area[:, None]
    np.testing.assert_allclose(ratio.max(), 0.5, rtol=1e-14)
