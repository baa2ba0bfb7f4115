"""Pins of the oracle's second-order scheme (Sec. 4.2, second order finite volume schemes:
Green-Gauss gradient, Barth-Jespersen limiter, linear reconstruction, Heun time step).

Each pin checks a property the paper's definitions fix independently of the oracle's code:
closed forms (Heun amplification of pure absorption, a uniform state being stationary),
exactness of Green-Gauss for linear data on a uniform rectangular grid, the bounds a limiter
exists to enforce, exact conservation, and the convergence order the scheme is built for.
"""
import dataclasses

import numpy as np
import pytest

from _util import small_problem

from oracle import oracle as o
from paper_2205_08417_amd import inputs as I


@pytest.mark.parametrize("mesh_kind", ["periodic", "delaunay_dirichlet", "delaunay_neumann"])
def test_uniform_state_is_stationary(mesh_kind):
    """Isotropic scattering with sigma_s = sigma_t keeps a uniform state (and its matching
    inflow ghost) unchanged: every gradient vanishes and the face sums close."""
    if mesh_kind == "periodic":
        mesh = I.periodic_mesh(6)
    else:
        mesh = I.jittered_delaunay_mesh(9, 0.0, 1.0, seed=3)
    P = small_problem(mesh, seed=1)
    sig = np.full(P.ncells, 1.3)
    P = dataclasses.replace(P, sigma_t=sig, sigma_s=sig, psi0=np.full((P.ncells, P.nq), 0.7),
                            inflow=np.full((mesh.nbfaces, P.nq), 0.7) if mesh.nbfaces else None)
    op = o.OracleProblem.from_problem(P, neumann=(mesh_kind == "delaunay_neumann"))
    out = o.step2(op, P.psi0, P.dt)
    np.testing.assert_allclose(out, 0.7, rtol=0, atol=1e-14)


def test_heun_amplification_of_pure_absorption():
    """Uniform state on a torus, sigma_s = 0: each stage multiplies by (1 - dt sigma), so the
    Heun step multiplies by 1 - dt sigma + (dt sigma)^2 / 2."""
    mesh = I.periodic_mesh(5)
    P = small_problem(mesh, seed=2)
    sig = 3.0
    P = dataclasses.replace(P, sigma_t=np.full(P.ncells, sig), sigma_s=np.zeros(P.ncells),
                            psi0=np.full((P.ncells, P.nq), 2.0))
    x = P.dt * sig
    out = o.step2(o.OracleProblem.from_problem(P), P.psi0, P.dt)
    np.testing.assert_allclose(out, 2.0 * (1 - x + 0.5 * x * x), rtol=1e-14)
    # and it is not the first-order factor
    assert abs(out[0, 0] - 2.0 * (1 - x)) > 1e-3 * x * x


def test_green_gauss_is_exact_for_linear_data_on_rectangles():
    """Face averages of a linear field on a uniform rectangular grid are its face-midpoint
    values, so the interior gradient is exact; the limiter then sees an increment of half the
    neighbour difference (ratio 2) and leaves it alone."""
    nx = ny = 7
    mesh = I.quad_grid_mesh(nx, ny, (0.0, 0.0), (1.4, 0.7))
    P = small_problem(mesh, npol=2, naz=4, seed=3)
    rng = np.random.default_rng(0)
    a, bx, by = rng.uniform(1, 2, P.nq), rng.uniform(-1, 1, P.nq), rng.uniform(-1, 1, P.nq)
    c = mesh.centroid
    psi = a[None, :] + c[:, :1] * bx[None, :] + c[:, 1:] * by[None, :]
    gx, gy = o.limited_gradient(o.OracleProblem.from_problem(P), psi)
    ii, jj = np.arange(mesh.ncells) % nx, np.arange(mesh.ncells) // nx
    interior = (ii > 0) & (ii < nx - 1) & (jj > 0) & (jj < ny - 1)
    np.testing.assert_allclose(gx[interior], np.broadcast_to(bx, gx[interior].shape), rtol=1e-12)
    np.testing.assert_allclose(gy[interior], np.broadcast_to(by, gy[interior].shape), rtol=1e-12)


@pytest.mark.parametrize("rho", [False, True])
def test_limiter_keeps_reconstruction_within_neighbourhood_extremes(rho):
    """Barth-Jespersen as read: every reconstructed face value lies between the smallest and
    the largest of u_i and the values across cell i's faces.  (With the printed factor 1/2
    in Delta_2 the slope could double and overshoot; this pin fails for that reading.)"""
    mesh = I.jittered_delaunay_mesh(12, 0.0, 1.0, seed=5)
    P = small_problem(mesh, seed=4, rho=rho, inflow=True)
    rng = np.random.default_rng(9)
    psi = rng.uniform(0.0, 1.0, (P.ncells, P.nq))
    op = o.OracleProblem.from_problem(P)
    gx, gy = o.limited_gradient(op, psi, inflow_scale=0.8)
    rho_v = op.rho if op.rho is not None else np.ones(op.nc)
    u = psi / rho_v[:, None]
    lo, hi = u.copy(), u.copy()
    faces = []
    for f in range(op.mf):
        j = op.face_nbr[:, f]
        fv = np.zeros_like(u)
        fv[j >= 0] = u[j[j >= 0]]
        fv[j < 0] = op.inflow[-1 - j[j < 0]] * 0.8
        lo, hi = np.minimum(lo, fv), np.maximum(hi, fv)
        r = op.face_mid[:, f] - op.centroid
        faces.append(u + gx * r[:, :1] + gy * r[:, 1:])
    tol = 1e-12 * np.maximum(np.abs(u), 1.0)
    for rec in faces:
        assert np.all(rec >= lo - tol) and np.all(rec <= hi + tol)
    # the limiter is active somewhere, and most slopes survive
    unl_x, unl_y = _unlimited_gradient(op, psi, 0.8)
    assert np.any(np.abs(gx) < 0.999 * np.abs(unl_x))
    assert np.mean(np.abs(gx) + np.abs(gy) > 0) > 0.5


def _unlimited_gradient(op, psi, inflow_scale):
    """Green-Gauss with face averages, written out with numpy (an independent evaluation)."""
    rho = op.rho if op.rho is not None else np.ones(op.nc)
    u = psi / rho[:, None]
    gx = np.zeros_like(u)
    gy = np.zeros_like(u)
    for f in range(op.mf):
        j = op.face_nbr[:, f]
        used = j != np.iinfo(np.int32).min
        fv = np.zeros_like(u)
        fv[j >= 0] = u[j[j >= 0]]
        bnd = used & (j < 0)
        if op.neumann:
            fv[bnd] = u[bnd]
        elif op.inflow is not None:
            fv[bnd] = op.inflow[-1 - j[bnd]] * inflow_scale
        avg = np.where(used[:, None], 0.5 * (u + fv), 0.0)
        gx += avg * op.face_normal[:, f, :1]
        gy += avg * op.face_normal[:, f, 1:]
    return gx / op.area[:, None], gy / op.area[:, None]


def test_limited_gradient_is_scaled_green_gauss():
    """The limited gradient is a per-(cell, ordinate) scaling in [0, 1] of the Green-Gauss
    gradient computed independently here."""
    mesh = I.jittered_delaunay_mesh(10, 0.0, 1.0, seed=6)
    P = small_problem(mesh, seed=6, inflow=True)
    psi = np.random.default_rng(1).uniform(0.0, 1.0, (P.ncells, P.nq))
    op = o.OracleProblem.from_problem(P)
    gx, gy = o.limited_gradient(op, psi, inflow_scale=1.0)
    ux, uy = _unlimited_gradient(op, psi, 1.0)
    big = np.hypot(ux, uy) > 1e-9
    lim_x = gx[big] / np.where(np.abs(ux[big]) > 1e-12, ux[big], 1.0)
    lim_y = gy[big] / np.where(np.abs(uy[big]) > 1e-12, uy[big], 1.0)
    use_x = np.abs(ux[big]) > np.abs(uy[big])
    lim = np.where(use_x, lim_x, lim_y)
    assert np.all(lim >= -1e-12) and np.all(lim <= 1 + 1e-12)
    np.testing.assert_allclose(gx[big], lim * ux[big], atol=1e-12 * np.abs(ux).max())
    np.testing.assert_allclose(gy[big], lim * uy[big], atol=1e-12 * np.abs(uy).max())


def test_local_maximum_gets_zero_slope():
    mesh = I.jittered_delaunay_mesh(9, 0.0, 1.0, seed=7)
    P = small_problem(mesh, seed=7)
    rng = np.random.default_rng(3)
    psi = rng.uniform(0.0, 0.5, (P.ncells, P.nq))
    k = P.ncells // 2
    psi[k] = 1.0
    gx, gy = o.limited_gradient(o.OracleProblem.from_problem(P), psi)
    assert np.all(gx[k] == 0.0) and np.all(gy[k] == 0.0)


def test_mass_is_conserved_on_a_torus_with_hg_scattering():
    """Shared faces see the same reconstructed pair from both sides and the column-normalised
    kernel conserves particles, so with sigma_t = sigma_s the total mass is unchanged."""
    mesh = I.periodic_mesh(6)
    omega, w = I.product_quadrature(4, 8)
    K = I.henyey_greenstein_kernel(omega, w, 0.6)
    P = small_problem(mesh, omega_w=(omega, w), K=K, seed=8)
    P = dataclasses.replace(P, sigma_s=P.sigma_t.copy())
    op = o.OracleProblem.from_problem(P)
    out = o.step2(op, P.psi0, P.dt)
    m0, m1 = o.mass(op, P.psi0), o.mass(op, out)
    assert abs(m1 - m0) <= 1e-13 * m0


def test_dense_isotropic_matrix_equals_isotropic_path():
    mesh = I.jittered_delaunay_mesh(8, 0.0, 1.0, seed=9)
    P = small_problem(mesh, seed=9, inflow=True, source=True)
    op = o.OracleProblem.from_problem(P)
    a = o.step2(op, P.psi0, P.dt, inflow_scale=0.5)
    b = o.step2(op.replace(K=I.isotropic_kernel(P.nq)), P.psi0, P.dt, inflow_scale=0.5)
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-15)


def _advection_error(n, second, T=0.25, flip=False, limiter="barth-jespersen"):
    """Free streaming of a smooth profile on the unit torus; L1 error at the centroids."""
    mesh = I.periodic_mesh(n, diagonal_flip=flip)
    omega, w = I.product_quadrature(2, 4)
    nc, nq = mesh.ncells, w.size

    def exact(t):
        x = mesh.centroid[:, None, 0] - omega[None, :, 0] * t
        y = mesh.centroid[:, None, 1] - omega[None, :, 1] * t
        return 2.0 + np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y)

    P = I.Problem(name="advect", mesh=mesh, omega=omega, w=w, K=None,
                  sigma_t=np.zeros(nc), sigma_s=np.zeros(nc), rho=None, source=None,
                  inflow=None, psi0=exact(0.0), dt=0.0, nsteps=0)
    dt0 = I.cfl_dt(mesh, omega, 0.3)
    steps = int(np.ceil(T / dt0))
    dt = T / steps
    op = o.OracleProblem.from_problem(P)
    psi = P.psi0
    for _ in range(steps):
        psi = o.step2(op, psi, dt, limiter=limiter) if second else o.step(op, psi, dt)
    return float(np.sum(mesh.area[:, None] * np.abs(psi - exact(T)))) / nq


def _reconstruction_bounds_hold(op, psi, gx, gy, inflow_scale):
    rho_v = op.rho if op.rho is not None else np.ones(op.nc)
    u = psi / rho_v[:, None]
    lo, hi = u.copy(), u.copy()
    faces = []
    for f in range(op.mf):
        j = op.face_nbr[:, f]
        fv = np.zeros_like(u)
        fv[j >= 0] = u[j[j >= 0]]
        fv[j < 0] = op.inflow[-1 - j[j < 0]] * inflow_scale
        lo, hi = np.minimum(lo, fv), np.maximum(hi, fv)
        r = op.face_mid[:, f] - op.centroid
        faces.append(u + gx * r[:, :1] + gy * r[:, 1:])
    tol = 1e-12 * np.maximum(np.abs(u), 1.0)
    return all(np.all(rec >= lo - tol) and np.all(rec <= hi + tol) for rec in faces)


def test_venkatakrishnan_limits():
    """Venkatakrishnan (Sec. 4.2 names it beside Barth-Jespersen): with a vanishing threshold
    eps its smooth limiter function stays below d1/d2, so reconstructions keep within the
    neighbourhood extremes; with a huge threshold it leaves the Green-Gauss gradient (computed
    independently here) untouched."""
    mesh = I.jittered_delaunay_mesh(12, 0.0, 1.0, seed=5)
    P = small_problem(mesh, seed=4, rho=True, inflow=True)
    psi = np.random.default_rng(9).uniform(0.0, 1.0, (P.ncells, P.nq))
    op = o.OracleProblem.from_problem(P)
    gx, gy = o.limited_gradient(op, psi, 0.8, limiter="venkatakrishnan", vk_k=0.0)
    assert _reconstruction_bounds_hold(op, psi, gx, gy, 0.8)
    ux, uy = _unlimited_gradient(op, psi, 0.8)
    assert np.any(np.abs(gx) < 0.99 * np.abs(ux))
    gx, gy = o.limited_gradient(op, psi, 0.8, limiter="venkatakrishnan", vk_k=1e6)
    np.testing.assert_allclose(gx, ux, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(gy, uy, rtol=1e-9, atol=1e-12)


def test_venkatakrishnan_convergence():
    """With eps^2 = (K h)^3, K = 1, the scheme with the Venkatakrishnan limiter is second order
    on smooth data (its smooth limiter function scales slopes by less than 1 away from
    extrema too, so its error is of the Barth-Jespersen size, not below it)."""
    e_vk = [_advection_error(n, True, limiter="venkatakrishnan") for n in (24, 48, 96)]
    e_bj = _advection_error(96, True)
    p = np.log2(e_vk[1] / e_vk[2])
    print(f"Venkatakrishnan errors {e_vk}, order {p:.2f}; Barth-Jespersen at 96: {e_bj}")
    assert p > 1.8
    assert e_vk[2] < 1.5 * e_bj


def test_convergence_order():
    """The scheme the section builds is second order on smooth data, the first-order scheme
    first order: observed orders between tori of 24, 48 and 96 squares per side whose
    diagonals all run the same way (where the face-average Green-Gauss gradient is
    consistent)."""
    e2 = [_advection_error(n, True) for n in (24, 48, 96)]
    e1 = [_advection_error(n, False) for n in (24, 48, 96)]
    p2 = np.log2(e2[1] / e2[2])
    p1 = np.log2(e1[1] / e1[2])
    print(f"second-order errors {e2}, order {p2:.2f}; first-order errors {e1}, order {p1:.2f}")
    assert p2 > 1.8
    assert 0.8 < p1 < 1.2
    assert e2[2] < 0.1 * e1[2]


def test_green_gauss_accuracy_depends_on_the_mesh():
    """Face-average Green-Gauss is first-order accurate where the diagonals are aligned and
    inconsistent (an O(1) error that does not shrink) where they alternate -- a property of
    the gradient formula, pinned so that a change to it shows."""
    def grad_error(n, flip):
        mesh = I.periodic_mesh(n, diagonal_flip=flip)
        omega, w = I.product_quadrature(1, 2)
        c = mesh.centroid
        u = np.repeat((2 + np.sin(2 * np.pi * c[:, 0]) * np.sin(2 * np.pi * c[:, 1]))[:, None],
                      w.size, axis=1)
        P = I.Problem(name="g", mesh=mesh, omega=omega, w=w, K=None, sigma_t=np.zeros(len(c)),
                      sigma_s=np.zeros(len(c)), rho=None, source=None, inflow=None, psi0=u,
                      dt=0.0, nsteps=0)
        ux, _ = _unlimited_gradient(o.OracleProblem.from_problem(P), u, 1.0)
        ex = 2 * np.pi * np.cos(2 * np.pi * c[:, 0]) * np.sin(2 * np.pi * c[:, 1])
        return np.abs(ux[:, 0] - ex).max()
    a24, a96 = grad_error(24, False), grad_error(96, False)
    f24, f96 = grad_error(24, True), grad_error(96, True)
    assert 3.5 < a24 / a96 < 4.5
    assert f96 > 1.0 and abs(f96 - f24) < 0.05 * f24
