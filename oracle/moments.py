"""Moment-projected scattering O Sigma M of the S_N equations (eq. SNEqns2, Sec. 3.1) --
TEST INFRASTRUCTURE, plain numpy in FP64.

The real spherical harmonics m_l^k (Sec. 3.1, moment equations) are built from the
normalised complex harmonics
    Y_l^k = sqrt((2l+1)/(4 pi) (l-k)!/(l+k)!) e^{i k phi} P_l^k(mu)
with the associated Legendre functions P_l^k (Condon-Shortley phase, three-term recurrence
in l).  Taking the real and imaginary parts as the section's combinations prescribe gives
    m_l^0 = Y_l^0,  m_l^k = (-1)^k sqrt(2) Re Y_l^k,  m_l^{-k} = (-1)^k sqrt(2) Im Y_l^k  (k > 0),
ordered (m_0^0, m_1^-1, m_1^0, m_1^1, ..., m_N^N).  O[q][j] = m_j(Omega_q) maps moments to
ordinates, M[j][q] = w_q m_j(Omega_q) ordinates to moments, and Sigma is diagonal with the
kernel's Legendre moments sigma_l = 2 pi int P_l(mu) k(mu) dmu on every moment of degree l.

The directions follow the paper's parametrisation Omega = (sqrt(1-mu^2) sin phi,
sqrt(1-mu^2) cos phi, mu), so mu = Omega_z and phi = atan2(Omega_x, Omega_y).
"""
from __future__ import annotations

import math

import numpy as np


def assoc_legendre(N: int, mu: np.ndarray) -> np.ndarray:
    """P_l^k(mu) for 0 <= k <= l <= N (Condon-Shortley phase): array [N+1][N+1][len(mu)]."""
    mu = np.asarray(mu, dtype=np.float64)
    s = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    P = np.zeros((N + 1, N + 1) + mu.shape)
    P[0, 0] = 1.0
    for k in range(1, N + 1):                   # P_k^k = -(2k-1) s P_{k-1}^{k-1}
        P[k, k] = -(2 * k - 1) * s * P[k - 1, k - 1]
    for k in range(0, N):                       # P_{k+1}^k = (2k+1) mu P_k^k
        P[k + 1, k] = (2 * k + 1) * mu * P[k, k]
    for k in range(0, N + 1):
        for l in range(k + 2, N + 1):           # (l-k) P_l^k = (2l-1) mu P_{l-1}^k - (l+k-1) P_{l-2}^k
            P[l, k] = ((2 * l - 1) * mu * P[l - 1, k] - (l + k - 1) * P[l - 2, k]) / (l - k)
    return P


def real_sh(omega: np.ndarray, N: int) -> np.ndarray:
    """m_j(Omega_q), j = l^2 + l + k: array [Q][(N+1)^2]."""
    omega = np.asarray(omega, dtype=np.float64).reshape(-1, 3)
    mu = omega[:, 2]
    phi = np.arctan2(omega[:, 0], omega[:, 1])
    P = assoc_legendre(N, mu)
    out = np.zeros((omega.shape[0], (N + 1) ** 2))
    for l in range(N + 1):
        for k in range(0, l + 1):
            norm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - k) /
                             math.factorial(l + k))
            if k == 0:
                out[:, l * l + l] = norm * P[l, 0]
            else:
                c = (-1) ** k * math.sqrt(2.0) * norm * P[l, k]
                out[:, l * l + l + k] = c * np.cos(k * phi)
                out[:, l * l + l - k] = c * np.sin(k * phi)
    return out


def moment_matrices(omega: np.ndarray, w: np.ndarray, N: int):
    """(O, M): O [Q][(N+1)^2] = m(Omega_q), M [(N+1)^2][Q] = w_q m(Omega_q)."""
    O = real_sh(omega, N)
    M = (np.asarray(w, dtype=np.float64)[:, None] * O).T.copy()
    return O, M


def sigma_diagonal(sigma_l: np.ndarray) -> np.ndarray:
    """The diagonal of Sigma: sigma_l repeated on the 2l+1 moments of degree l."""
    sigma_l = np.asarray(sigma_l, dtype=np.float64)
    return np.concatenate([np.full(2 * l + 1, sigma_l[l]) for l in range(sigma_l.size)])


def moment_scattering(omega: np.ndarray, w: np.ndarray, sigma_l: np.ndarray,
                      psi: np.ndarray) -> np.ndarray:
    """S = O Sigma M psi for every cell (rows of psi): the right-hand side of eq. SNEqns2
    without the per-cell cross section."""
    N = np.asarray(sigma_l).size - 1
    O, M = moment_matrices(omega, w, N)
    u = np.asarray(psi, dtype=np.float64) @ M.T            # moments per cell
    return (u * sigma_diagonal(sigma_l)[None, :]) @ O.T


def moment_kernel(omega: np.ndarray, w: np.ndarray, sigma_l: np.ndarray) -> np.ndarray:
    """The same operator as a dense kernel in the oracle's convention
    S_q = sum_p K[q][p] w_p psi_p:  K[q][p] = sum_j m_j(Omega_q) sigma_j m_j(Omega_p)."""
    N = np.asarray(sigma_l).size - 1
    O = real_sh(omega, N)
    return (O * sigma_diagonal(sigma_l)[None, :]) @ O.T
