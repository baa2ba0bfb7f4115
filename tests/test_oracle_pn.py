"""Pins of the P_N oracle (Sec. 3.1 P_N closure, Sec. 4.3 upwind flux with A^+/A^-) against
facts that do not come from the oracle itself:

* the spectrum of every flux Jacobian A_l = int m m^T Omega_l: by rotation invariance it is
  the same for x, y and z, and for A_z it is, per order k of the harmonics, the zeros of the
  orthogonal polynomial of degree N+1-k for the weight (1-mu^2)^k -- Gauss-Legendre nodes for
  k = 0, Gegenbauer C^(k+1/2) zeros (twice, cosine and sine harmonics) for k > 0 -- taken
  from scipy;
* the first row of A_l in closed form (1/sqrt(3) on the degree-1 harmonic along Omega_l);
* the algebra of the split: A^+ + A^- = A, A^+ >= 0 >= A^-, A^+ A^- = 0;
* degree 0: no transport, the closed-form collision update;
* conservation of every moment and a stationary uniform state on a periodic mesh, and the
  non-increasing L2 energy of the upwind scheme;
* the split of the 2-D system into z-even and z-odd moments that never meet (both
  streaming directions are even under z -> -z);
* the slab equivalence: on a grid whose state depends on x only, with zonal angular data
  about the x-axis, P_N with the characteristic upwind flux is exactly the 1-D S_{N+1}
  scheme with Gauss-Legendre ordinates (the eigenvectors of the x-zonal Jacobi matrix are
  the Legendre polynomials at its Gauss nodes).  The 1-D scheme here is written out in the
  test; the same for y.
"""
import math

import numpy as np
import pytest
import scipy.special as sp

from paper_2205_08417_amd import inputs as I
from oracle import oracle as o
from oracle import pn
from oracle.moments import real_sh


def _expected_spectrum(N):
    ev = list(sp.roots_legendre(N + 1)[0])
    for k in range(1, N + 1):
        r = sp.roots_gegenbauer(N + 1 - k, k + 0.5)[0]
        ev += list(r) + list(r)
    return np.sort(np.array(ev))


@pytest.mark.parametrize("N", [0, 1, 2, 3, 5, 8, 13])
def test_jacobian_spectra(N):
    ref = _expected_spectrum(N)
    for A in pn.flux_jacobians(N):
        assert np.abs(A - A.T).max() < 1e-14
        assert np.abs(np.sort(np.linalg.eigvalsh(A)) - ref).max() < 1e-12


def test_jacobian_first_rows_closed_form():
    """A_l[0][j] = int m_0 m_j Omega_l = 1/sqrt(3) on the degree-1 harmonic proportional to
    Omega_l (m_1^-1 ~ Omega_x, m_1^1 ~ Omega_y, m_1^0 ~ Omega_z), zero elsewhere."""
    Ax, Ay, Az = pn.flux_jacobians(4)
    for A, j in ((Ax, 1), (Ay, 3), (Az, 2)):
        e = np.zeros(A.shape[0])
        e[j] = 1.0 / math.sqrt(3.0)
        assert np.abs(A[0] - e).max() < 1e-14


@pytest.mark.parametrize("N", [1, 3, 5, 7])
def test_split_algebra(N):
    for A in pn.flux_jacobians(N)[:2]:
        Ap, Am = pn.split(A)
        assert np.abs(Ap + Am - A).max() < 1e-13
        assert np.linalg.eigvalsh(Ap).min() > -1e-13
        assert np.linalg.eigvalsh(Am).max() < 1e-13
        assert np.abs(Ap @ Am).max() < 1e-13
        # |A| = A^+ - A^- squares to A^2
        Ab = Ap - Am
        assert np.abs(Ab @ Ab - A @ A).max() < 1e-13


def test_sphere_rule_orthonormal():
    for N in (0, 3, 8):
        omega, w = pn.sphere_rule(N)
        assert abs(w.sum() - 4 * math.pi) < 1e-12
        m = real_sh(omega, N + 1)
        assert np.abs(m.T @ (w[:, None] * m) - np.eye(m.shape[1])).max() < 1e-12


def _op(mesh, nm, seed, rho=False, source=False, inflow=False, neumann=False, scale=(1.0, 1.0)):
    rng = np.random.default_rng(seed)
    nc = mesh.face_nbr.shape[0]
    nbf = int(np.sum(mesh.face_nbr < 0) - np.sum(mesh.face_nbr == np.iinfo(np.int32).min))
    return o.OracleProblem(
        face_nbr=mesh.face_nbr, face_normal=mesh.face_normal, area=mesh.area,
        omega=np.zeros((1, 3)), w=np.ones(1),
        sigma_t=rng.uniform(0.5, 1.5, nc) * scale[0], sigma_s=rng.uniform(0.1, 0.9, nc) * scale[1],
        rho=rng.uniform(0.5, 2.0, nc) if rho else None,
        source=rng.uniform(0.0, 1.0, nc) if source else None,
        inflow=rng.standard_normal((max(nbf, 1), nm)) if inflow else None, neumann=neumann)


def test_degree_zero_is_the_collision_ode():
    mesh = I.jittered_delaunay_mesh(7, 0.0, 1.0, seed=1)
    sys0 = pn.PNSystem(0)
    op = _op(mesh, 1, seed=2, rho=True, source=True, inflow=True)
    u = np.random.default_rng(3).uniform(0.5, 1.5, (op.nc, 1))
    dt, at, as_ = 0.01, 1.3, 0.7
    got = pn.pn_step(op, sys0, u, dt, alpha_t=at, alpha_s=as_)
    ref = u[:, 0] * (1 - dt * at * op.sigma_t + dt * as_ * op.sigma_s) \
        + dt * math.sqrt(4 * math.pi) * op.source
    assert np.abs(got[:, 0] - ref).max() < 1e-15


@pytest.mark.parametrize("N", [1, 3, 5])
def test_periodic_conservation_and_uniform_state(N):
    mesh = I.periodic_mesh(10)
    S = pn.PNSystem(N)
    op = _op(mesh, S.nm, seed=4, scale=(0.0, 0.0))
    rng = np.random.default_rng(5)
    u = rng.standard_normal((op.nc, S.nm))
    dt = pn.pn_cfl_dt(op, S, 0.5)
    v = pn.pn_step(op, S, u, dt)
    tot0 = op.area @ u
    tot1 = op.area @ v
    assert np.abs(tot1 - tot0).max() < 1e-13 * np.abs(u).max() * op.area.sum()
    c = rng.standard_normal(S.nm)
    uni = np.tile(c, (op.nc, 1))
    assert np.abs(pn.pn_step(op, S, uni, dt) - uni).max() < 1e-13


@pytest.mark.parametrize("N", [1, 3, 5])
def test_energy_non_increasing(N):
    """sum_i A_i |u_i|^2 never grows for the upwind scheme at CFL 0.5 on a periodic mesh
    (sigma = 0); a rough state loses energy at every step (the flux is dissipative)."""
    mesh = I.periodic_mesh(12)
    S = pn.PNSystem(N)
    op = _op(mesh, S.nm, seed=6, scale=(0.0, 0.0))
    u = np.random.default_rng(7).standard_normal((op.nc, S.nm))
    dt = pn.pn_cfl_dt(op, S, 0.5)
    e = [float(op.area @ np.sum(u * u, axis=1))]
    for _ in range(20):
        u = pn.pn_step(op, S, u, dt)
        e.append(float(op.area @ np.sum(u * u, axis=1)))
    d = np.diff(e)
    assert np.all(d < 0.0)


def test_subset_matches_full():
    mesh = I.jittered_delaunay_mesh(8, 0.0, 1.0, seed=8)
    S = pn.PNSystem(3, I.hg_legendre_moments(0.6, 3))
    op = _op(mesh, S.nm, seed=9, rho=True, source=True, inflow=True)
    u = np.random.default_rng(10).standard_normal((op.nc, S.nm))
    full = pn.pn_step(op, S, u, 0.01, alpha_t=1.2, alpha_s=0.8, inflow_scale=0.5)
    cells = np.array([0, 5, 17, op.nc - 1])
    part = pn.pn_step(op, S, u, 0.01, alpha_t=1.2, alpha_s=0.8, inflow_scale=0.5, cells=cells)
    assert np.array_equal(part, full[cells])


def _slab(N, axis, nsteps, neumann, seed):
    """P_N on a strip varying along ``axis`` (periodic across it) against the 1-D S_{N+1}
    Gauss scheme; returns the largest nodal difference relative to the state's size."""
    n = 24
    if axis == 0:
        mesh = I.quad_grid_mesh(n, 2, hi=(1.0, 2.0 / n), periodic_y=True)
        pos = lambda c: c % n
    else:
        mesh = I.quad_grid_mesh(2, n, hi=(2.0 / n, 1.0), periodic_x=True)
        pos = lambda c: c // 2
    rng = np.random.default_rng(seed)
    sigma_l = I.hg_legendre_moments(0.5, N)
    S = pn.PNSystem(N, sigma_l)
    mu, wq = sp.roots_legendre(N + 1)
    P = np.array([sp.eval_legendre(l, mu) for l in range(N + 1)])      # [l][q]
    nc = mesh.face_nbr.shape[0]
    ix = np.array([pos(c) for c in range(nc)])
    # per-strip-position data
    g = rng.uniform(0.2, 2.0, (n, N + 1))                     # nodal values at the Gauss nodes
    rho_x = rng.uniform(0.5, 2.0, n)
    st_x = rng.uniform(0.0, 1.0, n)
    ss_x = rng.uniform(0.0, 1.0, n)
    q_x = rng.uniform(0.0, 1.0, n)
    gL, gR = rng.uniform(0.0, 1.0, N + 1), rng.uniform(0.0, 1.0, N + 1)

    # zonal functions about the strip axis -> P_N moments (exact: the rule integrates degree 2N+3)
    omega, w = pn.sphere_rule(N)
    m = real_sh(omega, N)                                      # [Q][nm]
    legQ = np.array([sp.eval_legendre(l, omega[:, axis]) for l in range(N + 1)])   # [l][Q]

    def moments(nodal):
        a = (2 * np.arange(N + 1) + 1) / 2 * (P @ (wq * nodal))          # Legendre coefficients
        f = a @ legQ                                                       # f(Omega_axis) on rule
        return m.T @ (w * f)

    u0 = np.array([moments(g[ix[c]]) for c in range(nc)])
    bc, bf = np.nonzero((mesh.face_nbr < 0) & (mesh.face_nbr != np.iinfo(np.int32).min))
    order = np.argsort(-1 - mesh.face_nbr[bc, bf])
    inflow = np.zeros((bc.size, S.nm))
    for b, (c, f) in enumerate(zip(bc[order], bf[order])):
        low = mesh.face_normal[c, f, axis] < 0
        inflow[b] = moments(gL if low else gR)
    op = o.OracleProblem(face_nbr=mesh.face_nbr, face_normal=mesh.face_normal, area=mesh.area,
                         omega=np.zeros((1, 3)), w=np.ones(1), sigma_t=st_x[ix],
                         sigma_s=ss_x[ix], rho=rho_x[ix], source=q_x[ix],
                         inflow=None if neumann else inflow, neumann=neumann)
    h = 1.0 / n
    dt = 0.4 * h * rho_x.min()
    u = pn.pn_rollout(op, S, u0, dt, nsteps)

    # 1-D S_{N+1} with Gauss ordinates mu_q, upwind, same collision and ghosts
    G = g.copy()
    mup, mum = np.maximum(mu, 0.0), np.minimum(mu, 0.0)
    coef = (2 * np.arange(N + 1) + 1) / 2 * sigma_l
    for _ in range(nsteps):
        up = G / rho_x[:, None]
        left = np.vstack([up[:1] if neumann else gL[None], up[:-1]])
        right = np.vstack([up[1:], up[-1:] if neumann else gR[None]])
        flux = mup * (up - left) + mum * (right - up)
        scat = ((G @ (wq[:, None] * P.T)) * coef) @ P                    # sum_l coef P_l(mu)..
        G = (G - dt / h * flux - dt * st_x[:, None] * G + dt * ss_x[:, None] * scat
             + dt * q_x[:, None])
    # P_N state at the Gauss nodes along the axis
    dirs = np.zeros((N + 1, 3))
    dirs[:, axis] = mu
    dirs[:, 1 - axis] = np.sqrt(1.0 - mu * mu)
    nodal = u @ real_sh(dirs, N).T                                         # [nc][q]
    ref = G[ix]
    return np.abs(nodal - ref).max() / np.abs(ref).max()


@pytest.mark.parametrize("N", [1, 2, 3, 5])
@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("neumann", [False, True])
def test_slab_equivalence_with_gauss_sn(N, axis, neumann):
    assert _slab(N, axis, nsteps=15, neumann=neumann, seed=11 + N) < 1e-12


def _zodd(N):
    """Moments odd under z -> -z: (-1)^(l+|k|) = -1."""
    return np.array([((l + abs(k)) % 2) == 1 for l in range(N + 1) for k in range(-l, l + 1)])


@pytest.mark.parametrize("N", [2, 5])
def test_z_parity_subsystems_decouple(N):
    """Omega_x and Omega_y are even under z -> -z, so in 2-D the z-even and z-odd moments form
    independent systems: zero z-odd data stays zero, and each half evolves on its own."""
    mesh = I.jittered_delaunay_mesh(9, 0.0, 1.0, seed=20)
    S = pn.PNSystem(N, I.hg_legendre_moments(0.5, N))
    op = _op(mesh, S.nm, seed=21, rho=True, source=True, inflow=True)
    odd = _zodd(N)
    rng = np.random.default_rng(22)
    u = rng.standard_normal((op.nc, S.nm))
    ue = np.where(odd[None, :], 0.0, u)
    uo = np.where(odd[None, :], u, 0.0)
    opo = op.replace(inflow=np.where(odd[None, :], op.inflow, 0.0), source=None)
    ope = op.replace(inflow=np.where(odd[None, :], 0.0, op.inflow))
    full = pn.pn_step(op, S, u, 0.01)
    even_only = pn.pn_step(ope, S, ue, 0.01)
    odd_only = pn.pn_step(opo, S, uo, 0.01)
    scale = np.abs(full).max()
    # the quadrature and eigen-decomposition leave rounding-level entries outside the pattern
    assert np.abs(even_only[:, odd]).max() < 1e-14 * scale
    assert np.abs(odd_only[:, ~odd]).max() < 1e-14 * scale
    assert np.abs(full - even_only - odd_only).max() < 1e-13 * np.abs(full).max()
