"""Torch-facing layer over the libsnrt C ABI: problem upload, stepping, rollouts.

PyTorch supplies device memory and streams only; every step of the S_N path runs in the
HIP kernels behind ``snrt``.  States live on the device in the library's internal cell
order (a Hilbert renumbering); :meth:`Solver.to_internal` / :meth:`Solver.to_user` move
between that order and the user's with the library's own permute kernel.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np
import torch

from . import snrt
from .inputs import Problem

_PREC = {"fp32": snrt.SNRT_FP32, "bf16x3": snrt.SNRT_BF16X3, "bf16x2": snrt.SNRT_BF16X2,
         "bf16x1": snrt.SNRT_BF16X1, "fp16x3": snrt.SNRT_FP16X3}


def _require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("the S_N library needs a HIP device; none is visible")


class Solver:
    """Device-resident S_N problem: mesh / quadrature / scattering handles and materials.

    ``precision`` selects the dense scattering product (``fp32``, ``bf16x3``, ``bf16x2``,
    ``bf16x1``, ``fp16x3``); isotropic problems ignore it.  ``moments`` (Legendre moments sigma_0..sigma_N of the
    scattering kernel) selects the moment-projected scattering O Sigma M instead of ``P.K``.  ``fp64`` additionally uploads FP64 copies of the
    materials for the FP64 parity template (:meth:`step_f64`).
    """

    def __init__(self, P: Problem, device: str = "cuda", precision: str = "fp32",
                 reorder: bool = True, fp64: bool = False,
                 moments: Optional[Sequence[float]] = None):
        _require_gpu()
        self.P = P
        self.device = torch.device(device)
        self.nc, self.nq = P.ncells, P.nq
        m = P.mesh
        flags = snrt.SNRT_REORDER_HILBERT if reorder else snrt.SNRT_NO_REORDER
        with torch.cuda.device(self.device):
            self.mesh = snrt.snrt_mesh_create(m.face_nbr, m.face_normal, m.area, m.centroid,
                                              m.nbfaces, flags)
            self.quad = snrt.snrt_quad_create(P.omega, P.w)
            self.is_moments = moments is not None
            if moments is not None:
                # moment-projected scattering O Sigma M (eq. SNEqns2) with Legendre moments
                self.scatter = snrt.snrt_scatter_moments(self.quad, moments, _PREC[precision])
            elif P.K is None:
                self.scatter = snrt.snrt_scatter_isotropic(self.quad)
            else:
                self.scatter = snrt.snrt_scatter_dense(self.quad, P.K, _PREC[precision])
            self.ws_bytes = snrt.snrt_workspace_size(self.mesh, self.quad, self.scatter)
            if m.face_mid is not None:
                snrt.snrt_mesh_set_face_midpoints(self.mesh, m.face_mid)
        self.perm = snrt.snrt_mesh_permutation(self.mesh)
        self.ws2 = {}   # second-order workspaces by element type, allocated on first use
        self.ws = (torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
                   if self.ws_bytes else None)
        self.mats32 = self._materials(torch.float32)
        self.mats64 = self._materials(torch.float64) if fp64 else None

    # ------------------------------------------------------------------ layout helpers
    def _materials(self, dtype):
        P = self.P
        r = {"sigma_t": self.cells_to_internal(P.sigma_t, dtype),
             "sigma_s": self.cells_to_internal(P.sigma_s, dtype),
             "inv_rho": None if P.rho is None else self.cells_to_internal(1.0 / P.rho, dtype),
             "source": None if P.source is None else self.cells_to_internal(P.source, dtype),
             "inflow": None if P.inflow is None else
             torch.as_tensor(P.inflow, dtype=dtype).to(self.device).contiguous()}
        return r

    def to_internal(self, x, dtype=torch.float32) -> torch.Tensor:
        """[nc, ...] user-order array or tensor -> device tensor in internal order."""
        src = torch.as_tensor(np.asarray(x) if not torch.is_tensor(x) else x, dtype=dtype)
        src = src.to(self.device).contiguous()
        out = torch.empty_like(src)
        row = src[0].numel() * src.element_size() if src.shape[0] else 4
        snrt.snrt_permute(self.mesh, 0, src, out, row)
        return out

    def to_user(self, x: torch.Tensor) -> torch.Tensor:
        """Device tensor in internal order -> device tensor in user order."""
        x = x.contiguous()
        out = torch.empty_like(x)
        row = x[0].numel() * x.element_size() if x.shape[0] else 4
        snrt.snrt_permute(self.mesh, 1, x, out, row)
        return out

    def cells_to_internal(self, a, dtype=torch.float32) -> torch.Tensor:
        return self.to_internal(np.asarray(a).reshape(self.nc, 1), dtype).reshape(self.nc)

    def initial_state(self, dtype=torch.float32) -> torch.Tensor:
        return self.to_internal(self.P.psi0, dtype)

    # ------------------------------------------------------------------ steps
    def args(self, dt=None, alpha_t=1.0, alpha_s=1.0, inflow_scale=1.0, fp64=False,
             mats=None, boundary=snrt.SNRT_BC_DIRICHLET):
        M = mats or (self.mats64 if fp64 else self.mats32)
        return snrt.step_args(M["sigma_t"], M["sigma_s"], self.P.dt if dt is None else dt,
                              inv_rho=M["inv_rho"], source=M["source"], inflow=M["inflow"],
                              inflow_scale=inflow_scale, alpha_t=alpha_t, alpha_s=alpha_s,
                              boundary=boundary)

    def step(self, psi_in, psi_out, args=None, **kw):
        snrt.snrt_step(self.mesh, self.quad, self.scatter, args or self.args(**kw), psi_in,
                       psi_out, self.ws, self.ws_bytes)

    def step_f64(self, psi_in, psi_out, args=None, **kw):
        if self.mats64 is None:
            self.mats64 = self._materials(torch.float64)
        kw["fp64"] = True
        snrt.snrt_step_f64(self.mesh, self.quad, self.scatter, args or self.args(**kw), psi_in,
                           psi_out, self.ws, self.ws_bytes)

    def _ws2(self, fp64: bool):
        if fp64 not in self.ws2:
            n = snrt.snrt_step2_workspace_size(self.mesh, self.quad, self.scatter, fp64)
            self.ws2[fp64] = (torch.empty(max(n, 16), dtype=torch.uint8, device=self.device), n)
        return self.ws2[fp64]

    @property
    def is_dense(self) -> bool:
        return self.P.K is not None and not self.is_moments

    def prepare_implicit(self):
        """Set up the dense kernel's implicit form (snrt_scatter_prepare_implicit, once) and
        grow the workspace to what the dense IMEX step needs."""
        if getattr(self, "_implicit_ready", False):
            return
        with torch.cuda.device(self.device):
            snrt.snrt_scatter_prepare_implicit(self.scatter)
            n = snrt.snrt_workspace_size(self.mesh, self.quad, self.scatter)
        if n > self.ws_bytes:
            self.ws = torch.empty(n, dtype=torch.uint8, device=self.device)
            self.ws_bytes = n
        self._implicit_ready = True

    def _imex_fn(self, fp64: bool):
        """The IMEX entry point for this scattering form, as fn(mesh, quad, scatter, args,
        psi_in, psi_out, ws, ws_bytes, stream)."""
        if self.is_moments:
            return snrt.snrt_step_imex_moments_f64 if fp64 else snrt.snrt_step_imex_moments
        if self.is_dense:
            self.prepare_implicit()
            return snrt.snrt_step_imex_dense_f64 if fp64 else snrt.snrt_step_imex_dense
        fn = snrt.snrt_step_imex_f64 if fp64 else snrt.snrt_step_imex
        return lambda m, q, sc, args, a, b, ws_, n_, st=None: fn(m, q, sc, args, a, b, st)

    def step_imex(self, psi_in, psi_out, args=None, **kw):
        """One IMEX step: implicit collision (isotropic, dense or moment-projected
        scattering), explicit streaming and source."""
        args = args or self.args(**kw)
        fn = self._imex_fn(False)
        fn(self.mesh, self.quad, self.scatter, args, psi_in, psi_out, self.ws, self.ws_bytes)

    def step_imex_f64(self, psi_in, psi_out, args=None, **kw):
        if self.mats64 is None:
            self.mats64 = self._materials(torch.float64)
        kw["fp64"] = True
        args = args or self.args(**kw)
        fn = self._imex_fn(True)
        fn(self.mesh, self.quad, self.scatter, args, psi_in, psi_out, self.ws, self.ws_bytes)

    def step2(self, psi_in, psi_out, args=None, limiter="barth-jespersen", vk_k=1.0, **kw):
        """One Heun step of the second-order scheme (limited linear reconstruction);
        ``limiter`` is "barth-jespersen" or "venkatakrishnan" (with its K = ``vk_k``)."""
        ws, n = self._ws2(False)
        snrt.snrt_step2_limited(self.mesh, self.quad, self.scatter, args or self.args(**kw),
                                snrt.limiter(limiter, vk_k), psi_in, psi_out, ws, n)

    def step2_f64(self, psi_in, psi_out, args=None, limiter="barth-jespersen", vk_k=1.0, **kw):
        if self.mats64 is None:
            self.mats64 = self._materials(torch.float64)
        kw["fp64"] = True
        ws, n = self._ws2(True)
        snrt.snrt_step2_limited_f64(self.mesh, self.quad, self.scatter, args or self.args(**kw),
                                    snrt.limiter(limiter, vk_k), psi_in, psi_out, ws, n)

    def adjoint_step(self, psi_n, lam_np1, lam_n, g_sigma_t=None, g_sigma_s=None, g_rho=None,
                     args=None, **kw):
        snrt.snrt_step_adjoint(self.mesh, self.quad, self.scatter, args or self.args(**kw),
                               psi_n, lam_np1, lam_n, g_sigma_t, g_sigma_s, g_rho, self.ws,
                               self.ws_bytes)

    def adjoint_step_f64(self, psi_n, lam_np1, lam_n, g_sigma_t=None, g_sigma_s=None,
                         g_rho=None, args=None, **kw):
        if self.mats64 is None:
            self.mats64 = self._materials(torch.float64)
        kw["fp64"] = True
        snrt.snrt_step_adjoint_f64(self.mesh, self.quad, self.scatter, args or self.args(**kw),
                                   psi_n, lam_np1, lam_n, g_sigma_t, g_sigma_s, g_rho, self.ws,
                                   self.ws_bytes)

    def rollout(self, psi0: torch.Tensor, nsteps: int, fp64: bool = False,
                alpha_t: Optional[Sequence[float]] = None,
                alpha_s: Optional[Sequence[float]] = None,
                inflow_scale: Optional[Sequence[float]] = None,
                dose_coeff: Optional[Sequence[float]] = None,
                dose: Optional[torch.Tensor] = None, order: int = 1, imex: bool = False,
                limiter: str = "barth-jespersen", vk_k: float = 1.0):
        """Advance ``nsteps`` explicit steps (ping-pong buffers).  Returns ``(psi, dose)``;
        the dose (FP64, internal order) adds ``dose_coeff[n]`` times the density-weighted
        scalar flux of the state entering step n.  ``limiter`` and ``vk_k`` choose the slope
        limiter of the second-order scheme (``order=2``)."""
        if fp64 and dose_coeff is not None:
            raise ValueError("the dose accumulation runs on FP32 states")
        a = psi0.clone()
        b = torch.empty_like(a)
        if dose_coeff is not None and dose is None:
            dose = torch.zeros(self.nc, dtype=torch.float64, device=self.device)
        if fp64 and self.mats64 is None:
            self.mats64 = self._materials(torch.float64)
        if imex:
            step = self._imex_fn(fp64)
            ws = self.ws.data_ptr() if self.ws is not None else None
            ws_bytes = self.ws_bytes
        elif order == 2:
            fn2 = snrt.snrt_step2_limited_f64 if fp64 else snrt.snrt_step2_limited
            lim = snrt.limiter(limiter, vk_k)
            step = lambda m, q, sc, args, a, b, ws_, n_, st: fn2(m, q, sc, args, lim, a, b,  # noqa
                                                                  ws_, n_, st)
            w2, ws_bytes = self._ws2(fp64)
            ws = w2.data_ptr()
        elif order == 1:
            step = snrt.snrt_step_f64 if fp64 else snrt.snrt_step
            ws = self.ws.data_ptr() if self.ws is not None else None
            ws_bytes = self.ws_bytes
        else:
            raise ValueError("order is 1 (explicit Euler, first-order flux) or 2 (Heun, "
                             "limited linear reconstruction)")
        stream = torch.cuda.current_stream().cuda_stream
        if order == 1 and not imex:
            # the whole explicit Euler loop in one library call (snrt_rollout)
            sched = snrt.schedule(alpha_t, alpha_s, inflow_scale, dose_coeff)
            base = self.args(fp64=fp64)
            if fp64:
                snrt.snrt_rollout_f64(self.mesh, self.quad, self.scatter, base, sched, nsteps,
                                      a, b, None, 1, ws, ws_bytes, stream)
            else:
                snrt.snrt_rollout(self.mesh, self.quad, self.scatter, base, sched, nsteps, a, b,
                                  None, 1, dose if dose_coeff is not None else None, ws,
                                  ws_bytes, stream)
            return a, dose
        pa, pb = a.data_ptr(), b.data_ptr()
        cache = {}
        for n in range(nsteps):
            key = (1.0 if alpha_t is None else float(alpha_t[n]),
                   1.0 if alpha_s is None else float(alpha_s[n]),
                   1.0 if inflow_scale is None else float(inflow_scale[n]))
            if key not in cache:
                cache[key] = self.args(alpha_t=key[0], alpha_s=key[1], inflow_scale=key[2],
                                       fp64=fp64)
            if dose_coeff is not None:
                snrt.snrt_dose_accumulate(self.mesh, self.quad, pa, self.mats32["inv_rho"],
                                          float(dose_coeff[n]), dose, stream)
            step(self.mesh, self.quad, self.scatter, cache[key], pa, pb, ws, ws_bytes, stream)
            pa, pb = pb, pa
        return (a if pa == a.data_ptr() else b), dose

    # ------------------------------------------------------------------ reductions
    def mass(self, psi: torch.Tensor) -> float:
        out = torch.empty(1, dtype=torch.float64, device=self.device)
        snrt.snrt_mass(self.mesh, self.quad, psi, out)
        return float(out.item())

    def scalar_flux(self, psi: torch.Tensor) -> torch.Tensor:
        phi = torch.empty(self.nc, dtype=torch.float32, device=self.device)
        snrt.snrt_scalar_flux(self.mesh, self.quad, psi, phi)
        return phi

    def close(self):
        for fn, h in ((snrt.snrt_scatter_destroy, "scatter"), (snrt.snrt_quad_destroy, "quad"),
                      (snrt.snrt_mesh_destroy, "mesh")):
            v = getattr(self, h, None)
            if v:
                fn(v)
                setattr(self, h, None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------------------------------
# Differentiable rollout: hand-written adjoint steps with checkpoint-and-recompute
# ------------------------------------------------------------------------------------------

def _seq(x, n, default=1.0):
    return [default] * n if x is None else [float(v) for v in x]


class SNRollout(torch.autograd.Function):
    """``nsteps`` explicit S_N steps as one differentiable operation.

    Inputs (device tensors, internal cell order): ``psi0`` [nc, nq] (FP32, or FP64 for the
    parity template), per-cell ``sigma_t``, ``sigma_s`` and optional density ``rho``.  The
    forward pass (one ``snrt_rollout`` call) keeps the state every ``ckpt_every`` steps; the
    backward pass (one ``snrt_rollout_adjoint`` call) recomputes each segment from its
    checkpoint (bit-identical: the kernels are deterministic) and walks it backwards with the
    library's adjoint step:

        lam^N = dJ/dpsi^N,  lam^n = T_n^T lam^{n+1} + dJ/dpsi^n,
        dJ/dsigma_t, dJ/dsigma_s, dJ/drho accumulated by the adjoint kernel per step.

    With ``dose_coeff`` the dose D_i += coeff_n (1/rho_i) phi_i(psi^n) is accumulated before
    every step n (FP64) and returned as a second output; its adjoint adds
    coeff_n w_q (dJ/dD_i)/rho_i to lam^n and -D_i/rho_i dJ/dD_i to dJ/drho_i.
    """

    @staticmethod
    def forward(ctx, psi0, sigma_t, sigma_s, rho, solver, nsteps, ckpt_every, alpha_t, alpha_s,
                inflow_scale, dose_coeff):
        S = solver
        fp64 = psi0.dtype == torch.float64
        if fp64 and dose_coeff is not None:
            raise ValueError("the dose accumulation runs on FP32 states")
        if ckpt_every < 1:
            raise ValueError("ckpt_every must be >= 1")
        inv_rho = None if rho is None else torch.reciprocal(rho.detach()).contiguous()
        st, ss = sigma_t.detach().contiguous(), sigma_s.detach().contiguous()
        M = S.mats64 if fp64 else S.mats32
        if M is None:
            S.mats64 = S._materials(torch.float64)
            M = S.mats64
        # the step arguments over the differentiable materials; the per-step scalars come
        # from the schedule
        base = snrt.step_args(st, ss, S.P.dt, inv_rho=inv_rho, source=M["source"],
                              inflow=M["inflow"])
        sched = snrt.schedule(_seq(alpha_t, nsteps), _seq(alpha_s, nsteps),
                              _seq(inflow_scale, nsteps),
                              None if dose_coeff is None else _seq(dose_coeff, nsteps))
        stream = torch.cuda.current_stream().cuda_stream
        ws = S.ws.data_ptr() if S.ws is not None else None
        a = psi0.detach().contiguous().clone()
        b = torch.empty_like(a)
        dose = (torch.zeros(S.nc, dtype=torch.float64, device=a.device)
                if dose_coeff is not None else None)
        # one allocation holds every checkpoint; the library's rollout writes each
        # checkpointed state into its slot directly
        n_ck = (nsteps + ckpt_every - 1) // ckpt_every
        ck_store = torch.empty((max(n_ck, 1),) + tuple(a.shape), dtype=a.dtype, device=a.device)
        if fp64:
            snrt.snrt_rollout_f64(S.mesh, S.quad, S.scatter, base, sched, nsteps, a, b, ck_store,
                                  ckpt_every, ws, S.ws_bytes, stream)
        else:
            snrt.snrt_rollout(S.mesh, S.quad, S.scatter, base, sched, nsteps, a, b, ck_store,
                              ckpt_every, dose, ws, S.ws_bytes, stream)
        ctx.S, ctx.fp64, ctx.nsteps, ctx.K = S, fp64, nsteps, ckpt_every
        ctx.base, ctx.sched, ctx.ck_store = base, sched, ck_store
        ctx.stream, ctx.ws = stream, ws
        ctx.has_rho, ctx.has_dose = rho is not None, dose_coeff is not None
        ctx.save_for_backward(st, ss, inv_rho if inv_rho is not None else st,
                              dose if dose is not None else st)
        if dose is not None:
            return a, dose
        return a

    @staticmethod
    def backward(ctx, g_psi, g_dose=None):
        S, fp64, N, K = ctx.S, ctx.fp64, ctx.nsteps, ctx.K
        st, ss, inv_rho, dose = ctx.saved_tensors
        if not ctx.has_rho:
            inv_rho = None
        if not ctx.has_dose:
            dose = None
        dt = torch.float64 if fp64 else torch.float32
        dev = st.device
        lam = (torch.zeros((S.nc, S.nq), dtype=dt, device=dev) if g_psi is None
               else g_psi.to(dt).contiguous().clone())
        tmp = torch.empty_like(lam)
        # the reverse pass accumulates the gradients in FP64 (one small contribution per step)
        f64 = torch.float64
        g_t = torch.zeros(S.nc, dtype=f64, device=dev)
        g_s = torch.zeros(S.nc, dtype=f64, device=dev)
        g_r = torch.zeros(S.nc, dtype=f64, device=dev) if inv_rho is not None else None
        gd = None if (g_dose is None or dose is None) else g_dose.to(torch.float64).contiguous()
        seg = (torch.empty((K - 1,) + tuple(lam.shape), dtype=lam.dtype, device=dev)
               if K > 1 else None)
        if fp64:
            snrt.snrt_rollout_adjoint_f64(S.mesh, S.quad, S.scatter, ctx.base, ctx.sched, N,
                                          ctx.ck_store, K, seg, lam, tmp, g_t, g_s, g_r, ctx.ws,
                                          S.ws_bytes, ctx.stream)
        else:
            snrt.snrt_rollout_adjoint(S.mesh, S.quad, S.scatter, ctx.base, ctx.sched, N,
                                      ctx.ck_store, K, seg, lam, tmp, g_t, g_s, g_r, gd, dose,
                                      ctx.ws, S.ws_bytes, ctx.stream)
        g_t, g_s = g_t.to(st.dtype), g_s.to(ss.dtype)
        if g_r is not None:
            g_r = g_r.to(inv_rho.dtype)
        return (lam, g_t, g_s, g_r, None, None, None, None, None, None, None)


def differentiable_rollout(solver: Solver, psi0, nsteps, sigma_t=None, sigma_s=None, rho=None,
                           ckpt_every: int = 20, alpha_t=None, alpha_s=None, inflow_scale=None,
                           dose_coeff=None):
    """Convenience wrapper of :class:`SNRollout`; materials default to the problem's."""
    fp64 = psi0.dtype == torch.float64
    if fp64 and solver.mats64 is None:
        solver.mats64 = solver._materials(torch.float64)
    M = solver.mats64 if fp64 else solver.mats32
    sigma_t = M["sigma_t"] if sigma_t is None else sigma_t
    sigma_s = M["sigma_s"] if sigma_s is None else sigma_s
    return SNRollout.apply(psi0, sigma_t, sigma_s, rho, solver, int(nsteps), int(ckpt_every),
                           alpha_t, alpha_s, inflow_scale, dose_coeff)
