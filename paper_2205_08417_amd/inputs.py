"""Seeded synthetic inputs for the S_N step: meshes, quadrature, kernels, materials, time steps.

This module builds the *problem data* that the paper's solver takes as given -- an
unstructured cell-centred triangle grid (Sec. 4.1), a product quadrature on the unit
sphere (Sec. 3.2, eq. spherical-coordinatesProduct), scattering kernels, cross sections,
sources and boundary inflow -- and nothing of the step itself.  It holds no streaming,
scattering or update arithmetic, so both the FP64 oracle and the HIP library can consume
its output without sharing any code of the method.

Everything is FP64 NumPy and fully determined by the seeds given here.

Layout conventions shared by every consumer:

* ``face_nbr[c, f]``   int32: ``>= 0`` neighbour cell; ``-1 - b`` boundary face ``b``;
                        ``INT32_MIN`` for an unused slot (quadrilateral padding).
* ``face_normal[c, f]`` FP64 (2,): outward unit normal times face length, ``n_{i,j}`` of
                        Sec. 4.1.  For an interior face the neighbour's copy is the exact
                        bitwise negation (both are formed from the same coordinate
                        differences).
* ``omega[q]``          FP64 (3,): ``(sqrt(1-mu^2) sin phi, sqrt(1-mu^2) cos phi, mu)``.
* ``K[q, p]``           dense scattering kernel; the scattering source is
                        ``S_q = sum_p K[q, p] w_p psi_p`` (eq. SNEqns).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional

import numpy as np

INT32_MIN = np.iinfo(np.int32).min
FOUR_PI = 4.0 * math.pi


# ----------------------------------------------------------------------------------------
# Quadrature (Sec. 3.2, product rule)
# ----------------------------------------------------------------------------------------

def product_quadrature(n_polar: int, n_azimuth: int):
    """Product rule: Gauss-Legendre in mu times equally spaced azimuths.

    Azimuths are ``phi_l = l * dphi`` for ``l = 1..n_azimuth`` with ``dphi = 2 pi / n_azimuth``
    as the paper writes them, weights ``2 pi w^G_k / n_azimuth``.  Ordinates are numbered
    zero-based ``q = k * n_azimuth + (l - 1)``: polar index outer, azimuth inner.

    Returns ``(omega[nq, 3], w[nq])`` in FP64.
    """
    if n_polar < 1 or n_azimuth < 1:
        raise ValueError("quadrature orders must be positive")
    mu, wg = np.polynomial.legendre.leggauss(n_polar)
    dphi = 2.0 * math.pi / n_azimuth
    phi = dphi * np.arange(1, n_azimuth + 1, dtype=np.float64)
    MU = np.repeat(mu, n_azimuth)
    PHI = np.tile(phi, n_polar)
    st = np.sqrt(1.0 - MU * MU)
    omega = np.stack([st * np.sin(PHI), st * np.cos(PHI), MU], axis=1)
    w = np.repeat(2.0 * math.pi * wg / n_azimuth, n_azimuth)
    return np.ascontiguousarray(omega), np.ascontiguousarray(w)


# ----------------------------------------------------------------------------------------
# Meshes (Sec. 4.1)
# ----------------------------------------------------------------------------------------

@dataclasses.dataclass
class Mesh:
    points: np.ndarray        # [nv, 2]
    cells: np.ndarray         # [nc, mf] vertex ids, counter-clockwise
    face_nbr: np.ndarray      # [nc, mf] int32
    face_normal: np.ndarray   # [nc, mf, 2] FP64
    area: np.ndarray          # [nc] FP64
    centroid: np.ndarray      # [nc, 2] FP64
    bface_cell: np.ndarray    # [nbf] owning cell of boundary face b
    bface_mid: np.ndarray     # [nbf, 2] midpoint of boundary face b
    face_mid: Optional[np.ndarray] = None   # [nc, mf, 2] midpoint of every face slot, seen
                                            # from its cell (unwrapped on periodic meshes)

    @property
    def ncells(self) -> int:
        return int(self.area.shape[0])

    @property
    def max_faces(self) -> int:
        return int(self.face_nbr.shape[1])

    @property
    def nbfaces(self) -> int:
        return int(self.bface_cell.shape[0])


def _faces_from_triangles(points: np.ndarray, tris: np.ndarray, nbrs: np.ndarray) -> Mesh:
    """Per-cell face arrays of a CCW triangle list; ``nbrs[c, k]`` = neighbour opposite vertex k."""
    tris = np.asarray(tris, dtype=np.int64)
    p = points[tris]                                    # [nc, 3, 2]
    d1 = p[:, 1] - p[:, 0]
    d2 = p[:, 2] - p[:, 0]
    cross = d1[:, 0] * d2[:, 1] - d1[:, 1] * d2[:, 0]
    flip = cross < 0
    if np.any(flip):                                     # make every triangle CCW
        tris = tris.copy()
        nbrs = nbrs.copy()
        tris[flip, 1], tris[flip, 2] = tris[flip, 2].copy(), tris[flip, 1].copy()
        nbrs[flip, 1], nbrs[flip, 2] = nbrs[flip, 2].copy(), nbrs[flip, 1].copy()
        p = points[tris]
        d1 = p[:, 1] - p[:, 0]
        d2 = p[:, 2] - p[:, 0]
        cross = d1[:, 0] * d2[:, 1] - d1[:, 1] * d2[:, 0]
    nc = tris.shape[0]
    area = 0.5 * cross
    centroid = p.mean(axis=1)
    normal = np.empty((nc, 3, 2))
    for k in range(3):                                   # face k is the edge opposite vertex k
        a = p[:, (k + 1) % 3]
        b = p[:, (k + 2) % 3]
        normal[:, k, 0] = b[:, 1] - a[:, 1]
        normal[:, k, 1] = -(b[:, 0] - a[:, 0])
    face_nbr = np.asarray(nbrs, dtype=np.int64).copy()
    bc, bf = np.nonzero(face_nbr < 0)                    # row-major order -> boundary ids
    nbf = bc.shape[0]
    face_nbr[bc, bf] = -1 - np.arange(nbf)
    mids = 0.5 * (p[bc, (bf + 1) % 3] + p[bc, (bf + 2) % 3])
    fmid = np.stack([0.5 * (p[:, (k + 1) % 3] + p[:, (k + 2) % 3]) for k in range(3)], axis=1)
    return Mesh(points=points, cells=tris, face_nbr=face_nbr.astype(np.int32),
                face_normal=normal, area=area, centroid=centroid,
                bface_cell=bc.astype(np.int64), bface_mid=mids, face_mid=fmid)


def jittered_delaunay_mesh(n: int, lo: float, hi: float, seed: int, jitter: float = 0.25,
                           line_every: Optional[int] = None) -> Mesh:
    """Delaunay triangulation of an ``n x n`` grid of points on ``[lo, hi]^2``.

    Interior points move uniformly by up to ``jitter * h`` per coordinate; points on the
    boundary only slide along their edge; corners stay fixed.  With ``line_every = m`` the
    grid lines with index divisible by ``m`` keep their coordinate, so material interfaces on
    those lines are followed closely.  A jittered grid in general position gives exactly
    ``2 n^2 - 4 (n - 1) - 2`` triangles, which is asserted.
    """
    from scipy.spatial import Delaunay

    if n < 2:
        raise ValueError("need at least 2 points per side")
    rng = np.random.default_rng(seed)
    h = (hi - lo) / (n - 1)
    g = lo + h * np.arange(n, dtype=np.float64)
    g[-1] = hi
    X, Y = np.meshgrid(g, g, indexing="ij")
    jx = rng.uniform(-jitter, jitter, (n, n)) * h
    jy = rng.uniform(-jitter, jitter, (n, n)) * h
    idx = np.arange(n)
    if line_every:
        keep = (idx % line_every) == 0
        jx[keep, :] = 0.0
        jy[:, keep] = 0.0
    jx[[0, -1], :] = 0.0
    jy[:, [0, -1]] = 0.0
    pts = np.stack([X + jx, Y + jy], axis=-1).reshape(-1, 2)
    tri = Delaunay(pts)
    expect = 2 * n * n - 4 * (n - 1) - 2
    if tri.simplices.shape[0] != expect or len(tri.coplanar):
        raise RuntimeError(f"degenerate triangulation: {tri.simplices.shape[0]} != {expect}")
    mesh = _faces_from_triangles(pts, tri.simplices, tri.neighbors)
    if np.min(mesh.area) <= 1e-6 * h * h:
        raise RuntimeError("sliver triangle in the jittered mesh")
    return mesh


def four_triangle_mesh() -> Mesh:
    """The unit square cut by both diagonals: bottom, right, top, left triangles (area 1/4)."""
    pts = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0], [0.5, 0.5]])
    tris = np.array([[0, 1, 4], [1, 2, 4], [2, 3, 4], [3, 0, 4]])
    nbrs = np.array([[1, 3, -1], [2, 0, -1], [3, 1, -1], [0, 2, -1]])
    return _faces_from_triangles(pts, tris, nbrs)


def periodic_mesh(n: int, length: float = 1.0, diagonal_flip: bool = True) -> Mesh:
    """``n x n`` squares on a torus of side ``length``, each cut into two triangles.

    Every face is interior (no boundary).  Normals come from integer grid displacements
    scaled by ``h``, so each face's two copies are exact negations.  With
    ``diagonal_flip`` the diagonal alternates direction like a checkerboard.
    """
    if n < 3:
        raise ValueError("periodic mesh needs n >= 3 (smaller tori alias distinct edges)")
    h = length / n
    cells = []
    lverts = []   # local integer vertex coordinates per triangle (unwrapped)

    def sq(i, j):
        return (i % n) * n + (j % n)

    for i in range(n):
        for j in range(n):
            v00, v10, v11, v01 = (i, j), (i + 1, j), (i + 1, j + 1), (i, j + 1)
            if diagonal_flip and (i + j) % 2:
                lverts.append((v00, v10, v01))
                lverts.append((v10, v11, v01))
            else:
                lverts.append((v00, v10, v11))
                lverts.append((v00, v11, v01))
    lverts = np.array(lverts, dtype=np.int64)                 # [nc, 3, 2]
    nc = lverts.shape[0]
    # neighbour search: key each edge by its wrapped, sorted vertex pair
    def vid(v):
        return (v[..., 0] % n) * n + (v[..., 1] % n)
    edge_owner = {}
    face_nbr = np.full((nc, 3), -1, dtype=np.int64)
    for c in range(nc):
        for k in range(3):
            a = vid(lverts[c, (k + 1) % 3])
            b = vid(lverts[c, (k + 2) % 3])
            key = (min(a, b), max(a, b))
            # two triangles of a 2x2-or-larger torus share at most one edge per key
            if key in edge_owner:
                oc, ok = edge_owner.pop(key)
                face_nbr[c, k] = oc
                face_nbr[oc, ok] = c
            else:
                edge_owner[key] = (c, k)
    if edge_owner:
        raise RuntimeError("unmatched periodic edges")
    normal = np.empty((nc, 3, 2))
    for k in range(3):
        a = lverts[:, (k + 1) % 3]
        b = lverts[:, (k + 2) % 3]
        normal[:, k, 0] = (b[:, 1] - a[:, 1]) * h
        normal[:, k, 1] = -(b[:, 0] - a[:, 0]) * h
    d1 = (lverts[:, 1] - lverts[:, 0]) * h
    d2 = (lverts[:, 2] - lverts[:, 0]) * h
    area = 0.5 * (d1[:, 0] * d2[:, 1] - d1[:, 1] * d2[:, 0])
    centroid = lverts.mean(axis=1) * h
    fmid = np.stack([0.5 * (lverts[:, (k + 1) % 3] + lverts[:, (k + 2) % 3]) * h
                     for k in range(3)], axis=1)
    pts = np.array([[i * h, j * h] for i in range(n) for j in range(n)])
    cells = np.stack([vid(lverts[:, k]) for k in range(3)], axis=1)
    return Mesh(points=pts, cells=cells, face_nbr=face_nbr.astype(np.int32), face_normal=normal,
                area=area, centroid=centroid, bface_cell=np.zeros(0, np.int64),
                bface_mid=np.zeros((0, 2)), face_mid=fmid)


def quad_grid_mesh(nx: int, ny: int, lo=(0.0, 0.0), hi=(1.0, 1.0), periodic_x: bool = False,
                   periodic_y: bool = False) -> Mesh:
    """Structured ``nx x ny`` grid of rectangles (quadrilateral cells, four faces each).

    Face f of a cell is its CCW edge ``v_f -> v_{f+1}`` (bottom, right, top, left).  With
    ``periodic_x`` / ``periodic_y`` the grid wraps around in that direction (face midpoints
    stay in the cell's own frame); the remaining boundary faces are numbered as usual.
    """
    xs = np.linspace(lo[0], hi[0], nx + 1)
    ys = np.linspace(lo[1], hi[1], ny + 1)
    nc = nx * ny
    cid = lambda i, j: j * nx + i
    face_nbr = np.empty((nc, 4), dtype=np.int64)
    normal = np.empty((nc, 4, 2))
    fmid = np.empty((nc, 4, 2))
    area = np.empty(nc)
    centroid = np.empty((nc, 2))
    cells = np.empty((nc, 4), dtype=np.int64)
    bcell, bmid = [], []
    for j in range(ny):
        for i in range(nx):
            c = cid(i, j)
            v = [(xs[i], ys[j]), (xs[i + 1], ys[j]), (xs[i + 1], ys[j + 1]), (xs[i], ys[j + 1])]
            cells[c] = [j * (nx + 1) + i, j * (nx + 1) + i + 1, (j + 1) * (nx + 1) + i + 1,
                        (j + 1) * (nx + 1) + i]
            nb = [cid(i, j - 1) if j > 0 else (cid(i, ny - 1) if periodic_y else -1),
                  cid(i + 1, j) if i < nx - 1 else (cid(0, j) if periodic_x else -1),
                  cid(i, j + 1) if j < ny - 1 else (cid(i, 0) if periodic_y else -1),
                  cid(i - 1, j) if i > 0 else (cid(nx - 1, j) if periodic_x else -1)]
            for f in range(4):
                a, b = v[f], v[(f + 1) % 4]
                normal[c, f] = (b[1] - a[1], -(b[0] - a[0]))
                fmid[c, f] = (0.5 * (a[0] + b[0]), 0.5 * (a[1] + b[1]))
                face_nbr[c, f] = nb[f]
            area[c] = (xs[i + 1] - xs[i]) * (ys[j + 1] - ys[j])
            centroid[c] = (0.5 * (xs[i] + xs[i + 1]), 0.5 * (ys[j] + ys[j + 1]))
    bc, bf = np.nonzero(face_nbr < 0)
    face_nbr[bc, bf] = -1 - np.arange(bc.shape[0])
    pts = np.array([(x, y) for y in ys for x in xs])
    mids = np.array([0.5 * (np.array(pts[cells[c, f]]) + np.array(pts[cells[c, (f + 1) % 4]]))
                     for c, f in zip(bc, bf)]).reshape(-1, 2)
    return Mesh(points=pts, cells=cells, face_nbr=face_nbr.astype(np.int32),
                face_normal=normal, area=area, centroid=centroid,
                bface_cell=bc.astype(np.int64), bface_mid=mids, face_mid=fmid)


def pad_faces(mesh: Mesh, max_faces: int = 4) -> Mesh:
    """Same mesh with unused face slots (``INT32_MIN``, zero normal) appended per cell."""
    nc, mf = mesh.face_nbr.shape
    if max_faces < mf:
        raise ValueError("cannot drop faces")
    nbr = np.full((nc, max_faces), INT32_MIN, dtype=np.int32)
    nbr[:, :mf] = mesh.face_nbr
    nrm = np.zeros((nc, max_faces, 2))
    nrm[:, :mf] = mesh.face_normal
    mid = None
    if mesh.face_mid is not None:
        mid = np.zeros((nc, max_faces, 2))
        mid[:, :mf] = mesh.face_mid
    return dataclasses.replace(mesh, face_nbr=nbr, face_normal=nrm, face_mid=mid)


# ----------------------------------------------------------------------------------------
# Scattering kernels (eq. SNEqns; total = scattering cross section, Sec. 2)
# ----------------------------------------------------------------------------------------

def hg_legendre_moments(g: float, N: int) -> np.ndarray:
    """Legendre moments ``2 pi int P_l(mu) k_HG(mu) dmu = g^l`` (l = 0..N) of the
    Henyey-Greenstein kernel normalised to ``int k dOmega = 1``: the diagonal entries of the
    moment-projected scattering (eq. SNEqns2) for HG scattering."""
    return float(g) ** np.arange(N + 1, dtype=np.float64)


def isotropic_kernel(nq: int) -> np.ndarray:
    """Dense ``K = 1/(4 pi)``: the isotropic kernel written as a matrix."""
    return np.full((nq, nq), 1.0 / FOUR_PI)


def henyey_greenstein_kernel(omega: np.ndarray, w: np.ndarray, g: float,
                             normalise: bool = True) -> np.ndarray:
    """HG kernel ``k(mu) = (1 - g^2) / (4 pi (1 + g^2 - 2 g mu)^{3/2})`` at ``mu = Omega_q . Omega_p``.

    With ``normalise`` every column is divided by its quadrature integral so that
    ``sum_q w_q K[q, p] = 1`` exactly: scattering then conserves particles on the discrete
    sphere.  Column scaling leaves ``K`` non-symmetric.
    """
    mu = np.clip(omega @ omega.T, -1.0, 1.0)
    K = (1.0 - g * g) / (FOUR_PI * np.power(1.0 + g * g - 2.0 * g * mu, 1.5))
    if normalise:
        col = w @ K                                   # col[p] = sum_q w_q K[q, p]
        K = K / col[None, :]
    return np.ascontiguousarray(K)


# ----------------------------------------------------------------------------------------
# Time step (explicit Euler, CFL rule)
# ----------------------------------------------------------------------------------------

def cfl_dt(mesh: Mesh, omega: np.ndarray, cfl: float, rho: Optional[np.ndarray] = None) -> float:
    """``dt = cfl * min_i A_i rho_i / max_q sum_f (Omega_q . n_if)^+``.

    The bound keeps the streaming part of the explicit update a convex combination.
    """
    ox, oy = omega[:, 0], omega[:, 1]
    out = np.empty(mesh.ncells)
    for c0 in range(0, mesh.ncells, 4096):              # chunks bound the [c, f, q] temporary
        n = mesh.face_normal[c0:c0 + 4096]
        s = n[:, :, 0, None] * ox[None, None, :] + n[:, :, 1, None] * oy[None, None, :]
        valid = (mesh.face_nbr[c0:c0 + 4096] != INT32_MIN)[:, :, None]
        out[c0:c0 + 4096] = np.where(valid, np.maximum(s, 0.0), 0.0).sum(axis=1).max(axis=1)
    r = np.ones(mesh.ncells) if rho is None else rho
    return float(cfl * np.min(mesh.area * r / out))


def pn_cfl_dt(mesh: Mesh, cfl: float, rho: Optional[np.ndarray] = None) -> float:
    """``dt = cfl * min_i A_i rho_i / sum_f (|n_x| + |n_y|)``: a step bound for the P_N
    system, whose flux Jacobians have spectral radius below one."""
    valid = mesh.face_nbr != INT32_MIN
    s = np.sum(np.where(valid, np.abs(mesh.face_normal[..., 0]) + np.abs(mesh.face_normal[..., 1]),
                        0.0), axis=1)
    r = np.ones(mesh.ncells) if rho is None else rho
    return float(cfl * np.min(mesh.area * r / s))


# ----------------------------------------------------------------------------------------
# CSD energy <-> pseudo-time for the synthetic stopping power S(E) = 2 E^-0.3 (Sec. 2)
# ----------------------------------------------------------------------------------------

def stopping_power(E):
    return 2.0 * np.power(E, -0.3)


def csd_pseudo_time(E, e_max: float = 20.0):
    """``E~(E) = int_E^{Emax} dE'/S(E') = (Emax^1.3 - E^1.3) / 2.6`` for ``S = 2 E^-0.3``."""
    return (e_max ** 1.3 - np.power(E, 1.3)) / 2.6


def csd_energy(t, e_max: float = 20.0):
    """Inverse of :func:`csd_pseudo_time`."""
    return np.power(e_max ** 1.3 - 2.6 * np.asarray(t, dtype=np.float64), 1.0 / 1.3)


# ----------------------------------------------------------------------------------------
# Problems
# ----------------------------------------------------------------------------------------

@dataclasses.dataclass
class Problem:
    name: str
    mesh: Mesh
    omega: np.ndarray
    w: np.ndarray
    K: Optional[np.ndarray]          # None: isotropic
    sigma_t: np.ndarray
    sigma_s: np.ndarray
    rho: Optional[np.ndarray]        # None: rho = 1
    source: Optional[np.ndarray]     # per-cell isotropic source q_i (angular density)
    inflow: Optional[np.ndarray]     # [nbf, nq] ghost u = psi/rho on inflow faces, None: vacuum
    psi0: np.ndarray                 # [nc, nq]
    dt: float
    nsteps: int
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def ncells(self):
        return self.mesh.ncells

    @property
    def nq(self):
        return int(self.w.shape[0])


def checkerboard_absorbers():
    """Unit squares ``[i, i+1] x [j, j+1]`` of the 7x7 lattice that absorb.

    Reading of the layout: 1 <= i, j <= 5 with i + j even, minus the source square (3, 3)
    and the square above it (3, 5), which leaves the opening towards the top.
    """
    out = []
    for i in range(1, 6):
        for j in range(1, 6):
            if (i + j) % 2 == 0 and (i, j) not in ((3, 3), (3, 5)):
                out.append((i, j))
    return out


def _in_squares(xy: np.ndarray, squares) -> np.ndarray:
    m = np.zeros(xy.shape[0], dtype=bool)
    for i, j in squares:
        m |= (xy[:, 0] > i) & (xy[:, 0] < i + 1) & (xy[:, 1] > j) & (xy[:, 1] < j + 1)
    return m


def linesource(n_side: int, n_polar: int, n_azimuth: int, seed: int, nsteps: int,
               hg_g: Optional[float] = None, width: float = 0.03, cfl: float = 0.5) -> Problem:
    """Line-source-like case on ``[-1.5, 1.5]^2``: isotropic Gaussian pulse at the origin.

    ``sigma_s = 1``, ``sigma_a = 0``, vacuum boundary; the pulse
    ``(2 pi width^2)^-1 exp(-|x|^2 / (2 width^2))`` is sampled at cell centroids and is the
    same for every ordinate.  ``hg_g`` switches to a column-normalised HG kernel.
    """
    mesh = jittered_delaunay_mesh(n_side, -1.5, 1.5, seed)
    omega, w = product_quadrature(n_polar, n_azimuth)
    nc, nq = mesh.ncells, w.shape[0]
    r2 = np.sum(mesh.centroid ** 2, axis=1)
    pulse = np.exp(-r2 / (2 * width * width)) / (2 * math.pi * width * width)
    psi0 = np.repeat(pulse[:, None], nq, axis=1)
    K = None if hg_g is None else henyey_greenstein_kernel(omega, w, hg_g)
    return Problem(name="linesource", mesh=mesh, omega=omega, w=w, K=K,
                   sigma_t=np.ones(nc), sigma_s=np.ones(nc), rho=None, source=None,
                   inflow=None, psi0=np.ascontiguousarray(psi0),
                   dt=cfl_dt(mesh, omega, cfl), nsteps=nsteps,
                   meta={"hg_g": hg_g, "cfl": cfl, "seed": seed, "n_side": n_side})


def checkerboard(n_side: int, n_polar: int, n_azimuth: int, seed: int, nsteps: int,
                 cfl: float = 0.5) -> Problem:
    """Checkerboard lattice on ``[0, 7]^2`` (Sec. 7.2) with the absorber reading above.

    Absorbers: ``sigma_s = 0``, ``sigma_t = 10``; background ``sigma_s = sigma_t = 1``;
    isotropic source ``q = 1`` in ``[3, 4]^2``; vacuum boundary; ``psi0 = 0``.
    Materials are assigned by centroid.  Grid lines on integers are kept straight when the
    spacing allows.
    """
    line_every = (n_side - 1) // 7 if (n_side - 1) % 7 == 0 else None
    mesh = jittered_delaunay_mesh(n_side, 0.0, 7.0, seed, line_every=line_every)
    omega, w = product_quadrature(n_polar, n_azimuth)
    nc, nq = mesh.ncells, w.shape[0]
    absorb = _in_squares(mesh.centroid, checkerboard_absorbers())
    src = _in_squares(mesh.centroid, [(3, 3)])
    sigma_s = np.where(absorb, 0.0, 1.0)
    sigma_t = np.where(absorb, 10.0, 1.0)
    source = np.where(src, 1.0, 0.0)
    return Problem(name="checkerboard", mesh=mesh, omega=omega, w=w, K=None,
                   sigma_t=sigma_t, sigma_s=sigma_s, rho=None, source=source, inflow=None,
                   psi0=np.zeros((nc, nq)), dt=cfl_dt(mesh, omega, cfl), nsteps=nsteps,
                   meta={"cfl": cfl, "seed": seed, "n_side": n_side,
                         "detector": [5.0, 6.0, 3.0, 4.0]})


def region_mask(mesh: Mesh, box) -> np.ndarray:
    """Cells whose centroid lies in the box ``[x0, x1] x [y0, y1]``."""
    x0, x1, y0, y1 = box
    c = mesh.centroid
    return (c[:, 0] >= x0) & (c[:, 0] <= x1) & (c[:, 1] >= y0) & (c[:, 1] <= y1)


def csd_phantom(n_side: int, n_polar: int, n_azimuth: int, seed: int, nsteps: Optional[int],
                hg_g: float = 0.95, rho_air: float = 0.001, cfl: float = 0.5,
                e_max: float = 20.0, e_min: float = 0.1) -> Problem:
    """Water phantom ``[0, 10]^2`` cm with a bone insert and an air cavity, electron beam on top.

    Densities: water 1, bone 1.85 in ``[5.5, 7.5] x [4, 6]``, air ``rho_air`` in the disc of
    radius 0.75 at (4, 7).  Water cross sections ``Sigma_t = Sigma_s = 1``/cm with a
    column-normalised HG kernel; only ``1/rho`` enters the streaming (eq.
    BoltzmannCSDTrafo).  The beam enters through the top edge ``y = 10`` as the ghost
    ``u_b = S(E) G_x G_Omega G_E`` with ``G_x = exp(-(x-5)^2/(2 0.25^2))``,
    ``G_Omega = exp(-(Omega_y+1)^2/(2 0.1^2))`` and ``G_E = exp(-(E-20)^2/(2 0.5^2))``;
    the stored inflow is ``G_x G_Omega`` and each step scales it by ``S(E_n) G_E(E_n)``.
    ``nsteps=None`` runs the whole energy range ``e_max -> e_min``.
    """
    mesh = jittered_delaunay_mesh(n_side, 0.0, 10.0, seed)
    omega, w = product_quadrature(n_polar, n_azimuth)
    nc, nq = mesh.ncells, w.shape[0]
    c = mesh.centroid
    rho = np.ones(nc)
    rho[region_mask(mesh, (5.5, 7.5, 4.0, 6.0))] = 1.85
    air = (c[:, 0] - 4.0) ** 2 + (c[:, 1] - 7.0) ** 2 <= 0.75 ** 2
    rho[air] = rho_air
    K = henyey_greenstein_kernel(omega, w, hg_g)
    top = np.abs(mesh.bface_mid[:, 1] - 10.0) < 1e-12
    gx = np.where(top, np.exp(-(mesh.bface_mid[:, 0] - 5.0) ** 2 / (2 * 0.25 ** 2)), 0.0)
    gom = np.exp(-(omega[:, 1] + 1.0) ** 2 / (2 * 0.1 ** 2))
    inflow = np.ascontiguousarray(gx[:, None] * gom[None, :])
    dt = cfl_dt(mesh, omega, cfl, rho)
    t_end = float(csd_pseudo_time(e_min, e_max))
    if nsteps is None:
        nsteps = int(math.ceil(t_end / dt))
        dt = t_end / nsteps
    t = dt * np.arange(nsteps)
    E = csd_energy(t, e_max)
    SE = stopping_power(E)
    gE = np.exp(-(E - e_max) ** 2 / (2 * 0.5 ** 2))
    target = region_mask(mesh, (4.5, 5.5, 2.0, 3.0))
    organ = region_mask(mesh, (6.0, 7.0, 2.0, 3.0))
    return Problem(name="csd", mesh=mesh, omega=omega, w=w, K=K,
                   sigma_t=np.ones(nc), sigma_s=np.ones(nc), rho=rho, source=None,
                   inflow=inflow, psi0=np.zeros((nc, nq)), dt=dt, nsteps=nsteps,
                   meta={"energy": E, "inflow_scale": SE * gE, "dose_coeff": dt * SE,
                         "target": target, "organ": organ, "hg_g": hg_g, "seed": seed,
                         "n_side": n_side, "rho_air": rho_air})


# ----------------------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------------------

WORKLOADS: Dict[str, dict] = {
    # FP64 line source: 45x45 points -> 3 872 triangles, 8x8 = 64 ordinates, 100 steps
    "linesource_s8": dict(kind="linesource", n_side=45, n_polar=8, n_azimuth=8,
                          seed=1001, nsteps=100),
    # FP32 isotropic checkerboard: 316x316 points -> 198 450 triangles, 256 ordinates
    "checkerboard_s16": dict(kind="checkerboard", n_side=316, n_polar=16, n_azimuth=16,
                             seed=1002, nsteps=1000),
    # anisotropic HG g=0.9 line source: 225x225 -> 100 352 triangles, 1024 ordinates
    "linesource_hg_s32": dict(kind="linesource", n_side=225, n_polar=32, n_azimuth=32,
                              seed=1003, nsteps=200, hg_g=0.9),
    # adjoint checkerboard: 162x162 -> 51 842 triangles, 256 ordinates, 400 steps
    "checkerboard_adjoint_s16": dict(kind="checkerboard", n_side=162, n_polar=16,
                                     n_azimuth=16, seed=1004, nsteps=400),
    # CSD dose phantom: 388x388 -> 299 538 triangles, 16x32 = 512 ordinates, 500 steps
    "csd_phantom_s512": dict(kind="csd", n_side=388, n_polar=16, n_azimuth=32,
                             seed=1005, nsteps=500, hg_g=0.95),
}


def build(name: str, **over) -> Problem:
    """Build a named workload; keyword overrides change sizes (e.g. ``n_side=30``)."""
    spec = dict(WORKLOADS[name])
    spec.update(over)
    kind = spec.pop("kind")
    if kind == "linesource":
        return linesource(**spec)
    if kind == "checkerboard":
        return checkerboard(**spec)
    if kind == "csd":
        return csd_phantom(**spec)
    raise KeyError(kind)


def pn_checkerboard(n_side: int = 316, degree: int = 5, seed: int = 1002, cfl: float = 0.5,
                    nsteps: int = 1000) -> dict:
    """The checkerboard lattice (mesh and materials of :func:`checkerboard`) for a P_N
    solver of the given degree (Sec. 7.2 runs P_5): zero initial moments, vacuum boundary,
    isotropic scattering.  316 x 316 points give the 198 450 triangles of the S_N case."""
    P = checkerboard(n_side, 2, 2, seed, nsteps, cfl)
    nm = (degree + 1) ** 2
    return dict(name=f"checkerboard_p{degree}", mesh=P.mesh, degree=degree,
                sigma_t=P.sigma_t, sigma_s=P.sigma_s, source=P.source,
                u0=np.zeros((P.ncells, nm)), dt=pn_cfl_dt(P.mesh, cfl), nsteps=nsteps)


def random_moments(nc: int, nm: int, seed: int) -> np.ndarray:
    """Signed moments (standard normal, FP64), [nc][nm]."""
    return np.random.default_rng(seed).standard_normal((nc, nm))


def random_state(nc: int, nq: int, seed: int, decades: float = 6.0) -> np.ndarray:
    """Positive state spanning ``decades`` orders of magnitude (log-uniform), FP64."""
    rng = np.random.default_rng(seed)
    return np.power(10.0, -decades * rng.random((nc, nq)))
