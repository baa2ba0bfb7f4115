"""P_N solver step with the A^+/A^- upwind flux (Sec. 3.1 P_N closure, Sec. 4.3) --
TEST INFRASTRUCTURE, plain numpy in FP64.

The P_N closure expands psi in the real spherical harmonics m (degree <= N, the ordering
and normalisation of :mod:`oracle.moments`), which turns the transport equation into the
linear moment system

    d_t u + A_1 d_x (u / rho) + A_2 d_y (u / rho) + Sigma_t u = Sigma u + q,
    A_l = int m m^T Omega_l dOmega,   Sigma = diag(sigma_s sigma_l(j)),

in two space dimensions (A_3 d_z drops out).  Each A_l is split into its positive and
negative semidefinite parts A_l = A_l^+ + A_l^- (eigen-decomposition), and the upwind flux
over the face i -> j with outward normal n (times the face length) is, per Sec. 4.3,

    F(u_i, u_j) = sum_l (A_l^+ u_i/rho_i + A_l^- u_j/rho_j) n_l H(n_l)
                        + (A_l^- u_i/rho_i + A_l^+ u_j/rho_j) n_l (1 - H(n_l)),

H the Heaviside function (H(0) = 0; the term carries the factor n_l = 0 there anyway).  One
explicit Euler step is then (Sec. 4.2 with this flux)

    u_i' = u_i - dt/A_i sum_j F(u_i, u_j)
           + dt (-alpha_t sigma_t,i u_i + alpha_s sigma_s,i sigma_l(j) u_i + q_i e_0 sqrt(4 pi)),

the isotropic source q_i projected on the moments (int q m_0 dOmega = sqrt(4 pi) q).  Boundary
faces use a ghost state u_j/rho_j: the given ghost moments times inflow_scale (Dirichlet;
zero when none are given) or the cell's own u_i/rho_i (Neumann), as the S_N step does.

The integrals A_l are taken with a product rule that is exact for the polynomial degree
2N+1 of m m^T Omega_l (Gauss-Legendre in mu with N+2 nodes times 2N+4 equally spaced
azimuths), so they carry rounding only.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

from .moments import real_sh, sigma_diagonal


def sphere_rule(N: int):
    """(omega [Q][3], w [Q]) exact for spherical polynomials of degree <= 2N+3."""
    x, wl = np.polynomial.legendre.leggauss(N + 2)
    nphi = 2 * N + 4
    phi = (np.arange(nphi) + 0.5) * 2.0 * np.pi / nphi
    mu = np.repeat(x, nphi)
    ph = np.tile(phi, x.size)
    w = np.repeat(wl, nphi) * (2.0 * np.pi / nphi)
    s = np.sqrt(1.0 - mu * mu)
    return np.stack([s * np.sin(ph), s * np.cos(ph), mu], axis=1), w


def flux_jacobians(N: int):
    """(A_x, A_y, A_z), each [(N+1)^2][(N+1)^2]: A_l = int m m^T Omega_l (P_N closure)."""
    omega, w = sphere_rule(N)
    m = real_sh(omega, N)
    return tuple(m.T @ ((w * omega[:, l])[:, None] * m) for l in range(3))


def split(A: np.ndarray):
    """(A^+, A^-): the positive and negative semidefinite parts of the symmetric A (Sec. 4.3)."""
    lam, V = np.linalg.eigh(0.5 * (A + A.T))
    return (V * np.maximum(lam, 0.0)) @ V.T, (V * np.minimum(lam, 0.0)) @ V.T


def project_isotropic_source(nm: int) -> np.ndarray:
    """Moments of a unit isotropic source: int m_j dOmega = sqrt(4 pi) on m_0, zero else."""
    e = np.zeros(nm)
    e[0] = math.sqrt(4.0 * math.pi)
    return e


class PNSystem:
    """The degree-N moment system: Jacobians, their splits and the scattering diagonal."""

    def __init__(self, N: int, sigma_l: Optional[np.ndarray] = None):
        self.N = int(N)
        self.nm = (self.N + 1) ** 2
        self.Ax, self.Ay, self.Az = flux_jacobians(self.N)
        self.Axp, self.Axm = split(self.Ax)
        self.Ayp, self.Aym = split(self.Ay)
        sl = np.zeros(self.N + 1)
        sl[0] = 1.0                                   # isotropic scattering by default
        if sigma_l is not None:
            given = np.asarray(sigma_l, dtype=np.float64)
            sl[:min(given.size, sl.size)] = given[:sl.size]
        self.sigma_l = sl
        self.sig = sigma_diagonal(sl)


def pn_step(op, pn: PNSystem, u: np.ndarray, dt: float, alpha_t: float = 1.0,
            alpha_s: float = 1.0, inflow_scale: float = 1.0,
            cells: Optional[np.ndarray] = None) -> np.ndarray:
    """One explicit Euler P_N step of every cell (or of ``cells``): u [nc][nm] -> [nc][nm] (or
    [len(cells)][nm]).  ``op`` is an :class:`oracle.OracleProblem` whose ``inflow`` holds the
    ghost moments [nbfaces][nm] (u/rho units) and whose ``source`` is the isotropic q_i."""
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(op.nc, pn.nm)
    sel = np.arange(op.nc) if cells is None else np.asarray(cells, dtype=np.int64)
    rho = op.rho if op.rho is not None else np.ones(op.nc)
    up = u / rho[:, None]                                  # u / rho of every cell
    ui = up[sel]
    flux = np.zeros((sel.size, pn.nm))
    for f in range(op.mf):
        j = op.face_nbr[sel, f].astype(np.int64)
        n = op.face_normal[sel, f]                         # [k][2]
        used = j != np.iinfo(np.int32).min
        uj = np.zeros_like(ui)
        inner = used & (j >= 0)
        uj[inner] = up[j[inner]]
        bnd = used & (j < 0)
        if op.neumann:
            uj[bnd] = ui[bnd]
        elif op.inflow is not None:
            uj[bnd] = op.inflow.reshape(-1, pn.nm)[-1 - j[bnd]] * inflow_scale
        for l, (Ap, Am) in enumerate(((pn.Axp, pn.Axm), (pn.Ayp, pn.Aym))):
            nl = n[:, l:l + 1]
            H = (nl > 0.0).astype(np.float64)
            F = ((ui @ Ap.T + uj @ Am.T) * nl * H + (ui @ Am.T + uj @ Ap.T) * nl * (1.0 - H))
            flux += np.where(used[:, None], F, 0.0)
    src = op.source[sel] if op.source is not None else np.zeros(sel.size)
    R = (-alpha_t * op.sigma_t[sel, None] * u[sel]
         + alpha_s * op.sigma_s[sel, None] * pn.sig[None, :] * u[sel]
         + src[:, None] * project_isotropic_source(pn.nm)[None, :])
    return u[sel] - dt / op.area[sel, None] * flux + dt * R


def pn_rollout(op, pn: PNSystem, u0: np.ndarray, dt: float, nsteps: int, **kw) -> np.ndarray:
    """``nsteps`` explicit P_N steps from u0."""
    u = np.ascontiguousarray(u0, dtype=np.float64).reshape(op.nc, pn.nm)
    for _ in range(nsteps):
        u = pn_step(op, pn, u, dt, **kw)
    return u


def pn_cfl_dt(op, pn: PNSystem, cfl: float) -> float:
    """dt = cfl min_i A_i rho_i / sum_f (|n_x| rho(A_x) + |n_y| rho(A_y)), rho(.) the spectral
    radius: the forward-Euler limit of the upwind scheme."""
    rx = float(np.max(np.abs(np.linalg.eigvalsh(pn.Ax)))) if pn.N > 0 else 0.0
    ry = float(np.max(np.abs(np.linalg.eigvalsh(pn.Ay)))) if pn.N > 0 else 0.0
    used = op.face_nbr != np.iinfo(np.int32).min
    s = np.sum(np.where(used, np.abs(op.face_normal[..., 0]) * rx
                        + np.abs(op.face_normal[..., 1]) * ry, 0.0), axis=1)
    rho = op.rho if op.rho is not None else np.ones(op.nc)
    s = np.where(s > 0.0, s, np.inf)
    return float(cfl * np.min(op.area * rho / s))
