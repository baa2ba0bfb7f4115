"""ctypes front end of ``sn_oracle.c`` plus plain rollout / gradient drivers (FP64, host).

TEST INFRASTRUCTURE: see the package docstring.  The drivers are literal loops over the
paper's explicit time iteration (Alg. "Execution of the solver", one Runge-Kutta stage for
explicit Euler); the adjoint drivers walk the same loop backwards with the exact
transpose of each step.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Callable, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sn_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_lp = ctypes.POINTER(ctypes.c_int64)


def build_oracle(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP over independent cells / ordinates)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_oracle()
        L = ctypes.CDLL(_LIB)
        L.oracle_version.restype = ctypes.c_int
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_num_threads.restype = ctypes.c_int
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        L.oracle_step.restype = ctypes.c_int
        L.oracle_step.argtypes = [ctypes.c_int64, ctypes.c_int32, _ip, _dp, _dp, ctypes.c_int32,
                                  _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_double,
                                  ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, _dp, _dp, ctypes.c_int64, _lp]
        L.oracle_adjoint_step.restype = ctypes.c_int
        L.oracle_adjoint_step.argtypes = [ctypes.c_int64, ctypes.c_int32, _ip, _dp, _dp,
                                          ctypes.c_int32, _dp, _dp, _dp, _dp, _dp, _dp,
                                          ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, _dp, _dp, _dp, _dp, _dp, _dp]
        L.oracle_mass.restype = ctypes.c_double
        L.oracle_mass.argtypes = [ctypes.c_int64, _dp, ctypes.c_int32, _dp, _dp]
        L.oracle_scalar_flux.restype = ctypes.c_int
        L.oracle_scalar_flux.argtypes = [ctypes.c_int64, ctypes.c_int32, _dp, _dp, _dp]
        L.oracle_dose_accumulate.restype = ctypes.c_int
        L.oracle_dose_accumulate.argtypes = [ctypes.c_int64, ctypes.c_int32, _dp, _dp, _dp,
                                             ctypes.c_double, _dp]
        L.oracle_limited_gradient.restype = ctypes.c_int
        L.oracle_limited_gradient.argtypes = [ctypes.c_int64, ctypes.c_int32, _ip, _dp, _dp, _dp,
                                              _dp, ctypes.c_int32, _dp, _dp, ctypes.c_double,
                                              ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                              _dp, _dp, _dp]
        L.oracle_step2.restype = ctypes.c_int
        L.oracle_step2.argtypes = [ctypes.c_int64, ctypes.c_int32, _ip, _dp, _dp, _dp, _dp,
                                   ctypes.c_int32, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                   ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                   ctypes.c_double, _dp, _dp]
        _lib = L
    return _lib


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


class OracleProblem:
    """The arrays one step needs, converted once to contiguous FP64 / int32."""

    def __init__(self, face_nbr, face_normal, area, omega, w, sigma_t, sigma_s, K=None,
                 rho=None, source=None, inflow=None, neumann=False, face_mid=None,
                 centroid=None):
        self.face_nbr = np.ascontiguousarray(face_nbr, dtype=np.int32)
        self.nc, self.mf = self.face_nbr.shape
        self.face_normal = _f64(face_normal).reshape(self.nc, self.mf, 2)
        self.face_mid = None if face_mid is None else _f64(face_mid).reshape(self.nc, self.mf, 2)
        self.centroid = None if centroid is None else _f64(centroid).reshape(self.nc, 2)
        self.area = _f64(area)
        self.omega = _f64(omega).reshape(-1, 3)
        self.w = _f64(w)
        self.nq = int(self.w.shape[0])
        self.K = _f64(K)
        self.sigma_t = _f64(sigma_t)
        self.sigma_s = _f64(sigma_s)
        self.rho = _f64(rho)
        self.source = _f64(source)
        self.inflow = _f64(inflow)
        self.neumann = bool(neumann)

    @classmethod
    def from_problem(cls, P, **over):
        kw = dict(face_nbr=P.mesh.face_nbr, face_normal=P.mesh.face_normal, area=P.mesh.area,
                  omega=P.omega, w=P.w, sigma_t=P.sigma_t, sigma_s=P.sigma_s, K=P.K, rho=P.rho,
                  source=P.source, inflow=P.inflow, face_mid=P.mesh.face_mid,
                  centroid=P.mesh.centroid)
        kw.update(over)
        return cls(**kw)

    def replace(self, **over):
        kw = dict(face_nbr=self.face_nbr, face_normal=self.face_normal, area=self.area,
                  omega=self.omega, w=self.w, sigma_t=self.sigma_t, sigma_s=self.sigma_s,
                  K=self.K, rho=self.rho, source=self.source, inflow=self.inflow,
                  neumann=self.neumann, face_mid=self.face_mid, centroid=self.centroid)
        kw.update(over)
        return OracleProblem(**kw)


def step(op: OracleProblem, psi: np.ndarray, dt: float, alpha_t: float = 1.0,
         alpha_s: float = 1.0, inflow_scale: float = 1.0, cells: Optional[np.ndarray] = None):
    """One explicit Euler S_N step (Sec. 4.2 with eq. upwind1stOrder2 and eq. SNEqns)."""
    psi = _f64(psi).reshape(op.nc, op.nq)
    if cells is None:
        out = np.empty((op.nc, op.nq))
        sel, nsel = None, 0
    else:
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.empty((cells.shape[0], op.nq))
        sel, nsel = cells.ctypes.data_as(_lp), cells.shape[0]
    rc = lib().oracle_step(op.nc, op.mf, op.face_nbr.ctypes.data_as(_ip), _d(op.face_normal),
                           _d(op.area), op.nq, _d(op.omega), _d(op.w), _d(op.K),
                           _d(op.sigma_t), _d(op.sigma_s), _d(op.rho), _d(op.source),
                           _d(op.inflow), float(inflow_scale), int(op.neumann), float(dt),
                           float(alpha_t), float(alpha_s), _d(psi), _d(out), nsel, sel)
    if rc != 0:
        raise ValueError("oracle_step rejected its arguments")
    return out


def adjoint_step(op: OracleProblem, psi_n: np.ndarray, lam_np1: np.ndarray, dt: float,
                 alpha_t: float = 1.0, alpha_s: float = 1.0, g_sigma_t=None, g_sigma_s=None,
                 g_rho=None):
    """Exact transpose of :func:`step` applied to ``lam_np1``; gradients accumulate in place."""
    psi_n = _f64(psi_n).reshape(op.nc, op.nq)
    lam_np1 = _f64(lam_np1).reshape(op.nc, op.nq)
    out = np.empty((op.nc, op.nq))
    rc = lib().oracle_adjoint_step(op.nc, op.mf, op.face_nbr.ctypes.data_as(_ip),
                                   _d(op.face_normal), _d(op.area), op.nq, _d(op.omega),
                                   _d(op.w), _d(op.K), _d(op.sigma_t), _d(op.sigma_s),
                                   _d(op.rho), int(op.neumann), float(dt), float(alpha_t),
                                   float(alpha_s), _d(psi_n), _d(lam_np1), _d(out),
                                   _d(g_sigma_t), _d(g_sigma_s), _d(g_rho))
    if rc != 0:
        raise ValueError("oracle_adjoint_step rejected its arguments")
    return out


_LIMITERS = {"barth-jespersen": 0, "venkatakrishnan": 1}


def limited_gradient(op: OracleProblem, psi: np.ndarray, inflow_scale: float = 1.0,
                     limiter: str = "barth-jespersen", vk_k: float = 1.0):
    """Psi_i grad(u_i) per cell and ordinate (Green-Gauss + the Barth-Jespersen or the
    Venkatakrishnan limiter, Sec. 4.2 second order schemes): returns (gx, gy), each [nc][nq].

    Venkatakrishnan (the limiter the section names next to Barth-Jespersen, in the form of
    its cited paper): per face, with d2 = grad u_i . r_if and d1 = u_max - u_i (d2 > 0) or
    u_min - u_i (d2 < 0), phi = ((d1^2 + eps^2) d2 + 2 d2^2 d1) / (d1^2 + 2 d2^2 + d1 d2 +
    eps^2) / d2, Psi_i = min over faces; eps^2 = (vk_k sqrt(A_i))^3."""
    psi = _f64(psi).reshape(op.nc, op.nq)
    if op.face_mid is None or op.centroid is None:
        raise ValueError("the second-order scheme needs face midpoints and centroids")
    gx = np.empty((op.nc, op.nq))
    gy = np.empty((op.nc, op.nq))
    rc = lib().oracle_limited_gradient(op.nc, op.mf, op.face_nbr.ctypes.data_as(_ip),
                                       _d(op.face_normal), _d(op.face_mid), _d(op.centroid),
                                       _d(op.area), op.nq, _d(op.rho), _d(op.inflow),
                                       float(inflow_scale), int(op.neumann), _LIMITERS[limiter],
                                       float(vk_k), _d(psi), _d(gx), _d(gy))
    if rc != 0:
        raise ValueError("oracle_limited_gradient rejected its arguments")
    return gx, gy


def step2(op: OracleProblem, psi: np.ndarray, dt: float, alpha_t: float = 1.0,
          alpha_s: float = 1.0, inflow_scale: float = 1.0, limiter: str = "barth-jespersen",
          vk_k: float = 1.0) -> np.ndarray:
    """One Heun step of the second-order scheme (Sec. 4.2): (psi + L(L(psi))) / 2, with the
    limiter of :func:`limited_gradient`."""
    psi = _f64(psi).reshape(op.nc, op.nq)
    if op.face_mid is None or op.centroid is None:
        raise ValueError("the second-order scheme needs face midpoints and centroids")
    out = np.empty((op.nc, op.nq))
    rc = lib().oracle_step2(op.nc, op.mf, op.face_nbr.ctypes.data_as(_ip), _d(op.face_normal),
                            _d(op.face_mid), _d(op.centroid), _d(op.area), op.nq, _d(op.omega),
                            _d(op.w), _d(op.K), _d(op.sigma_t), _d(op.sigma_s), _d(op.rho),
                            _d(op.source), _d(op.inflow), float(inflow_scale), int(op.neumann),
                            float(dt), float(alpha_t), float(alpha_s), _LIMITERS[limiter],
                            float(vk_k), _d(psi), _d(out))
    if rc != 0:
        raise ValueError(f"oracle_step2 failed ({rc})")
    return out


def mass(op: OracleProblem, psi) -> float:
    """Total mass sum_i A_i sum_q w_q psi_iq (solver log quantity, Sec. 5.1)."""
    psi = _f64(psi).reshape(op.nc, op.nq)
    return float(lib().oracle_mass(op.nc, _d(op.area), op.nq, _d(op.w), _d(psi)))


def scalar_flux(op: OracleProblem, psi) -> np.ndarray:
    """Psi_i = sum_q w_q psi_iq (Sec. 7.2)."""
    psi = _f64(psi).reshape(op.nc, op.nq)
    out = np.empty(op.nc)
    lib().oracle_scalar_flux(op.nc, op.nq, _d(op.w), _d(psi), _d(out))
    return out


def dose_accumulate(op: OracleProblem, psi, coeff: float, dose: np.ndarray) -> np.ndarray:
    """D_i += coeff / rho_i sum_q w_q psi_iq (dose integral of Sec. 2, left endpoint)."""
    psi = _f64(psi).reshape(op.nc, op.nq)
    assert dose.dtype == np.float64 and dose.flags.c_contiguous
    lib().oracle_dose_accumulate(op.nc, op.nq, _d(op.w), _d(psi), _d(op.rho), float(coeff),
                                 _d(dose))
    return dose


# ----------------------------------------------------------------------------------------
# Rollouts (the time loop of the solver algorithm, explicit Euler: one stage per step)
# ----------------------------------------------------------------------------------------

def rollout(op: OracleProblem, psi0, dt: float, nsteps: int, alpha_t=None, alpha_s=None,
            inflow_scale=None, dose_coeff=None, keep_states: bool = False):
    """Run ``nsteps`` explicit steps.  Per-step sequences may be given for ``alpha_t``,
    ``alpha_s``, ``inflow_scale`` and ``dose_coeff`` (the dose adds ``dose_coeff[n]`` times the
    density-weighted scalar flux of the state *entering* step n).

    Returns ``(psi_N, dose or None, states or None)``; ``states[n]`` is psi^n for n < N.
    """
    psi = _f64(psi0).reshape(op.nc, op.nq).copy()
    dose = np.zeros(op.nc) if dose_coeff is not None else None
    states = [] if keep_states else None
    for n in range(nsteps):
        at = 1.0 if alpha_t is None else float(alpha_t[n])
        as_ = 1.0 if alpha_s is None else float(alpha_s[n])
        isc = 1.0 if inflow_scale is None else float(inflow_scale[n])
        if keep_states:
            states.append(psi)
        if dose is not None:
            dose_accumulate(op, psi, float(dose_coeff[n]), dose)
        psi = step(op, psi, dt, at, as_, isc)
    return psi, dose, states


def rollout_gradient(op: OracleProblem, psi0, dt: float, nsteps: int,
                     dJ_dpsiN: Optional[np.ndarray] = None, dJ_ddose: Optional[np.ndarray] = None,
                     alpha_t=None, alpha_s=None, inflow_scale=None, dose_coeff=None,
                     ckpt_every: Optional[int] = None):
    """Reverse pass of :func:`rollout` for a functional J(psi^N, D) that is linear in its
    arguments with the given partial derivatives.  Returns a dict with ``psi0``,
    ``sigma_t``, ``sigma_s`` and (when ``op.rho`` is given) ``rho`` gradients.

    Recurrence: lam^N = dJ/dpsi^N; lam^n = T_n^T lam^{n+1} + dJ/dpsi^n, where the dose term
    of step n gives dJ/dpsi^n_iq = coeff_n w_q (dJ/dD_i) / rho_i, and the explicit density
    derivative of D_i = (1/rho_i) sum_n coeff_n phi_i^n is -D_i/rho_i (dJ/dD_i).

    ``ckpt_every``: None keeps every state psi^n of the forward pass; an integer K keeps only
    psi^{kK} and, walking the segments backwards, steps each one forward again from its
    stored state before the adjoint steps need it (the memory of a long run is then about
    (N/K + K) states instead of N).  The states, and so the result, are the same either way.
    """
    nc, nq = op.nc, op.nq

    def scalars(n):
        return (1.0 if alpha_t is None else float(alpha_t[n]),
                1.0 if alpha_s is None else float(alpha_s[n]),
                1.0 if inflow_scale is None else float(inflow_scale[n]))

    if ckpt_every is None:
        _, dose, states = rollout(op, psi0, dt, nsteps, alpha_t, alpha_s, inflow_scale,
                                  dose_coeff, keep_states=True)
        K = max(nsteps, 1)
        kept = {0: None}
    else:
        if ckpt_every < 1:
            raise ValueError("ckpt_every must be >= 1")
        K = int(ckpt_every)
        # forward pass keeping psi^n for n = 0, K, 2K, ... (and the dose)
        psi = _f64(psi0).reshape(nc, nq).copy()
        dose = np.zeros(nc) if dose_coeff is not None else None
        kept = {}
        for n in range(nsteps):
            at, as_, isc = scalars(n)
            if n % K == 0:
                kept[n] = psi
            if dose is not None:
                dose_accumulate(op, psi, float(dose_coeff[n]), dose)
            psi = step(op, psi, dt, at, as_, isc)
        states = None
    lam = np.zeros((nc, nq)) if dJ_dpsiN is None else _f64(dJ_dpsiN).reshape(nc, nq).copy()
    g_t = np.zeros(nc)
    g_s = np.zeros(nc)
    g_r = np.zeros(nc) if op.rho is not None else None
    rho = op.rho if op.rho is not None else np.ones(nc)
    for n0 in sorted(kept, reverse=True):
        n1 = min(n0 + K, nsteps)
        if states is None:
            seg = [kept[n0]]
            for n in range(n0, n1 - 1):
                at, as_, isc = scalars(n)
                seg.append(step(op, seg[-1], dt, at, as_, isc))
        else:
            seg = states[n0:n1]
        for n in range(n1 - 1, n0 - 1, -1):
            at, as_, _ = scalars(n)
            lam = adjoint_step(op, seg[n - n0], lam, dt, at, as_, g_t, g_s, g_r)
            if dJ_ddose is not None and dose_coeff is not None:
                lam += float(dose_coeff[n]) * op.w[None, :] * (dJ_ddose / rho)[:, None]
    if g_r is not None and dJ_ddose is not None and dose is not None:
        g_r += -dose / rho * dJ_ddose
    return {"psi0": lam, "sigma_t": g_t, "sigma_s": g_s, "rho": g_r, "dose": dose}


def num_threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().oracle_num_threads())


def set_num_threads(n: int) -> int:
    """Sets the OpenMP thread count of the oracle's parallel loops; returns the previous."""
    return int(lib().oracle_set_num_threads(int(n)))


def rel_l2(x, ref) -> float:
    """||x - ref||_2 / ||ref||_2 over all entries."""
    x = np.asarray(x, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    nr = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / (nr if nr > 0 else 1.0))


# ----------------------------------------------------------------------------------------
# IMEX step (Sec. 4.2): implicit linear collision operator, explicit streaming and source
# ----------------------------------------------------------------------------------------

def step_imex(op: OracleProblem, psi: np.ndarray, dt: float, alpha_t: float = 1.0,
              alpha_s: float = 1.0, inflow_scale: float = 1.0,
              cells: Optional[np.ndarray] = None) -> np.ndarray:
    """(I - dt R_i) psi_i^{n+1} = psi_i^n - dt/A_i sum_j F_up + dt q_i per cell, with the
    linear collision operator R_i psi = -alpha_t sigma_t,i psi + alpha_s sigma_s,i S(psi)
    (S the scattering source of eq. SNEqns) taken implicitly and the source q explicitly.

    The right-hand side is the explicit step with the collision term switched off; the
    per-cell system (a I - c K~) psi = b, a = 1 + dt alpha_t sigma_t, c = dt alpha_s sigma_s,
    K~[q][p] = K[q][p] w_p (K = 1/(4 pi) when isotropic), is solved with numpy's LU solver.
    ``cells``: only those cells' rows, in that order.
    """
    zero = np.zeros(op.nc)
    b = step(op.replace(sigma_t=zero, sigma_s=zero), psi, dt, alpha_t, alpha_s, inflow_scale,
             cells=cells)
    K = op.K if op.K is not None else np.full((op.nq, op.nq), 1.0 / (4.0 * np.pi))
    Kw = K * op.w[None, :]
    idx = np.arange(op.nc) if cells is None else np.asarray(cells, dtype=np.int64)
    a = 1.0 + dt * alpha_t * op.sigma_t[idx]
    c = dt * alpha_s * op.sigma_s[idx]
    out = np.empty_like(b)
    eye = np.eye(op.nq)
    for start in range(0, b.shape[0], 256):                # batches of cells
        sl = slice(start, min(b.shape[0], start + 256))
        A = a[sl, None, None] * eye[None] - c[sl, None, None] * Kw[None]
        out[sl] = np.linalg.solve(A, b[sl][..., None])[..., 0]
    return out
