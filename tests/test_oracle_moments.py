"""Pins of the oracle's moment-projected scattering O Sigma M (eq. SNEqns2).

Independent checks: the addition theorem of spherical harmonics against scipy's Legendre
polynomials, orthonormality of the basis under a product rule that integrates it exactly,
degree-1 functions being linear in Omega, the isotropic special case, conservation, and
convergence of the truncated Henyey-Greenstein expansion to the kernel itself.
"""
import dataclasses

import numpy as np
import pytest
from scipy.special import eval_legendre

from _util import small_problem

from oracle import moments as mo
from oracle import oracle as o
from paper_2205_08417_amd import inputs as I


def _unit(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


@pytest.mark.parametrize("N", [1, 4, 8, 12])
def test_addition_theorem(N):
    """sum_k m_l^k(a) m_l^k(b) = (2l+1)/(4 pi) P_l(a.b) for every degree l <= N."""
    rng = np.random.default_rng(N)
    a, b = _unit(rng, 40), _unit(rng, 40)
    ma, mb = mo.real_sh(a, N), mo.real_sh(b, N)
    cos = np.sum(a * b, axis=1)
    for l in range(N + 1):
        sl = slice(l * l, (l + 1) * (l + 1))
        lhs = np.sum(ma[:, sl] * mb[:, sl], axis=1)
        rhs = (2 * l + 1) / (4 * np.pi) * eval_legendre(l, cos)
        np.testing.assert_allclose(lhs, rhs, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("N,npol,naz", [(4, 5, 10), (8, 9, 18), (8, 16, 32)])
def test_orthonormal_under_exact_quadrature(N, npol, naz):
    """M O = I when the product rule integrates every product of two degree-N harmonics."""
    omega, w = I.product_quadrature(npol, naz)
    O, M = mo.moment_matrices(omega, w, N)
    np.testing.assert_allclose(M @ O, np.eye((N + 1) ** 2), atol=1e-12)


def test_degree_one_is_linear_in_omega():
    rng = np.random.default_rng(3)
    om = _unit(rng, 50)
    m = mo.real_sh(om, 1)
    assert np.allclose(m[:, 0], 1 / np.sqrt(4 * np.pi))
    for j in (1, 2, 3):
        coef, res, *_ = np.linalg.lstsq(om, m[:, j], rcond=None)
        assert np.allclose(om @ coef, m[:, j], atol=1e-13)
        np.testing.assert_allclose(np.linalg.norm(coef), np.sqrt(3 / (4 * np.pi)), rtol=1e-12)


def test_isotropic_moments_reproduce_isotropic_path():
    P = small_problem(I.jittered_delaunay_mesh(9, 0.0, 1.0, seed=2), 4, 8, seed=2,
                      source=True, inflow=True)
    K = mo.moment_kernel(P.omega, P.w, np.array([1.0, 0.0, 0.0, 0.0]))
    np.testing.assert_allclose(K, 1 / (4 * np.pi), atol=1e-15)
    op = o.OracleProblem.from_problem(P)
    a = o.step(op, P.psi0, P.dt)
    b = o.step(op.replace(K=K), P.psi0, P.dt)
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-15)


def test_moment_form_equals_kernel_form():
    """O Sigma M psi computed through the moments equals the kernel written as a matrix."""
    omega, w = I.product_quadrature(6, 12)
    sig = 0.7 ** np.arange(6)
    psi = np.random.default_rng(4).uniform(0, 1, (25, w.size))
    S1 = mo.moment_scattering(omega, w, sig, psi)
    K = mo.moment_kernel(omega, w, sig)
    S2 = (K * w[None, :]) @ psi.T
    np.testing.assert_allclose(S1, S2.T, rtol=1e-12, atol=1e-14)


def test_conserves_particles_under_exact_quadrature():
    """sum_q w_q S_q = sigma_0 sum_q w_q psi_q: the degree >= 1 moments integrate to zero."""
    omega, w = I.product_quadrature(10, 20)
    sig = np.array([1.0, 0.9, 0.81, 0.7, 0.6, 0.5, 0.4, 0.3, 0.2])
    psi = np.random.default_rng(5).uniform(0, 1, (30, w.size))
    S = mo.moment_scattering(omega, w, sig, psi)
    np.testing.assert_allclose(S @ w, psi @ w, rtol=1e-12)


def test_henyey_greenstein_truncation_converges():
    """With sigma_l = g^l the degree-N kernel approaches the continuous HG kernel
    k(mu) = (1-g^2)/(4 pi (1+g^2-2 g mu)^{3/2}) like g^(N+1)."""
    g = 0.5
    omega, w = I.product_quadrature(12, 24)
    mu = np.clip(omega @ omega.T, -1.0, 1.0)
    exact = (1 - g * g) / (4 * np.pi * (1 + g * g - 2 * g * mu) ** 1.5)
    errs = []
    for N in (2, 4, 6, 8, 10):
        K = mo.moment_kernel(omega, w, I.hg_legendre_moments(g, N))
        errs.append(np.abs(K - exact).max())
    errs = np.array(errs)
    assert np.all(np.diff(errs) < 0)
    ratios = errs[1:] / errs[:-1]
    assert np.all(ratios < 0.4)             # tends to g^2 = 0.25 per two degrees


def test_moment_step_conserves_mass_on_torus():
    mesh = I.periodic_mesh(6)
    omega, w = I.product_quadrature(8, 16)
    K = mo.moment_kernel(omega, w, I.hg_legendre_moments(0.8, 6))
    P = small_problem(mesh, omega_w=(omega, w), K=K, seed=6)
    P = dataclasses.replace(P, sigma_s=P.sigma_t.copy())
    op = o.OracleProblem.from_problem(P)
    out = o.step(op, P.psi0, P.dt)
    assert abs(o.mass(op, out) - o.mass(op, P.psi0)) <= 1e-13 * o.mass(op, P.psi0)
