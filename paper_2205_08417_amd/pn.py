"""Torch-facing layer over the P_N entry points of libsnrt (Sec. 3.1 P_N closure, Sec. 4.3).

PyTorch supplies device memory and streams only; the step runs in the library's HIP
kernels.  States live on the device in the library's tiled moment layout (cells in the
mesh's internal order, 64-cell tiles, moment-major inside a tile); :meth:`PNSolver.to_tiled`
and :meth:`PNSolver.to_user` convert from and to the user's [ncells][nmoments] rows with
the library's own layout kernel.
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np
import torch

from . import snrt
from .inputs import Mesh


class PNSolver:
    """Device-resident P_N problem of degree ``degree`` on ``mesh``.

    Materials are per cell in user order: ``sigma_t``, ``sigma_s``, optional ``rho`` and the
    isotropic ``source`` q_i.  ``sigma_l`` are the scattering kernel's Legendre moments
    (None: isotropic).  ``ghost`` holds Dirichlet ghost moments [nbfaces][nmoments] in u/rho
    units (None: vacuum); ``neumann`` makes every boundary face copy the cell's own state.
    """

    def __init__(self, mesh: Mesh, degree: int, sigma_t, sigma_s, dt: float,
                 sigma_l: Optional[Sequence[float]] = None, rho=None, source=None, ghost=None,
                 neumann: bool = False, device: str = "cuda", reorder: bool = True):
        if not torch.cuda.is_available():
            raise RuntimeError("the P_N step needs a HIP device; none is visible")
        self.device = torch.device(device)
        self.nc = mesh.ncells
        self.dt = float(dt)
        self.neumann = bool(neumann)
        flags = snrt.SNRT_REORDER_HILBERT if reorder else snrt.SNRT_NO_REORDER
        with torch.cuda.device(self.device):
            self.mesh = snrt.snrt_mesh_create(mesh.face_nbr, mesh.face_normal, mesh.area,
                                              mesh.centroid, mesh.nbfaces, flags)
            self.pn = snrt.snrt_pn_create(degree, sigma_l)
        self.degree, self.nm = snrt.snrt_pn_info(self.pn)
        self.elems = snrt.snrt_pn_state_elems(self.mesh, self.pn)
        self._host = {"sigma_t": sigma_t, "sigma_s": sigma_s,
                      "inv_rho": None if rho is None else 1.0 / np.asarray(rho, dtype=np.float64),
                      "source": source, "ghost": ghost}
        self.mats = {torch.float32: self._materials(torch.float32)}

    # ------------------------------------------------------------------ layout helpers
    def _cells(self, a, dtype) -> torch.Tensor:
        src = torch.as_tensor(np.asarray(a, dtype=np.float64).reshape(self.nc, 1), dtype=dtype)
        src = src.to(self.device).contiguous()
        out = torch.empty_like(src)
        snrt.snrt_permute(self.mesh, 0, src, out, src.element_size())
        return out.reshape(self.nc)

    def _materials(self, dtype):
        h = self._host
        g = h["ghost"]
        return {"sigma_t": self._cells(h["sigma_t"], dtype),
                "sigma_s": self._cells(h["sigma_s"], dtype),
                "inv_rho": None if h["inv_rho"] is None else self._cells(h["inv_rho"], dtype),
                "source": None if h["source"] is None else self._cells(h["source"], dtype),
                "ghost": None if g is None else
                torch.as_tensor(np.asarray(g, dtype=np.float64), dtype=dtype)
                .to(self.device).contiguous()}

    def new_state(self, dtype=torch.float32) -> torch.Tensor:
        """An uninitialised device state in the tiled layout."""
        return torch.empty(self.elems, dtype=dtype, device=self.device)

    def to_tiled(self, u_user, dtype=torch.float32) -> torch.Tensor:
        """[ncells][nmoments] user-order moments -> device state in the tiled layout."""
        src = torch.as_tensor(np.asarray(u_user) if not torch.is_tensor(u_user) else u_user,
                              dtype=dtype).to(self.device).contiguous()
        if tuple(src.shape) != (self.nc, self.nm):
            raise ValueError(f"expected [{self.nc}, {self.nm}] moments, got {tuple(src.shape)}")
        out = torch.zeros(self.elems, dtype=dtype, device=self.device)
        snrt.snrt_pn_layout(self.mesh, self.pn, 0, src.element_size(), src, out)
        return out

    def to_user(self, u: torch.Tensor) -> torch.Tensor:
        """Tiled device state -> [ncells][nmoments] in user order."""
        out = torch.empty((self.nc, self.nm), dtype=u.dtype, device=self.device)
        snrt.snrt_pn_layout(self.mesh, self.pn, 1, u.element_size(), u, out)
        return out

    # ------------------------------------------------------------------ steps
    def args(self, dtype=torch.float32, dt=None, alpha_t=1.0, alpha_s=1.0, inflow_scale=1.0):
        if dtype not in self.mats:
            self.mats[dtype] = self._materials(dtype)
        M = self.mats[dtype]
        return snrt.step_args(M["sigma_t"], M["sigma_s"], self.dt if dt is None else dt,
                              inv_rho=M["inv_rho"], source=M["source"], inflow=M["ghost"],
                              inflow_scale=inflow_scale, alpha_t=alpha_t, alpha_s=alpha_s,
                              boundary=snrt.SNRT_BC_NEUMANN if self.neumann
                              else snrt.SNRT_BC_DIRICHLET)

    def step(self, u_in: torch.Tensor, u_out: torch.Tensor, args=None, **kw) -> None:
        if u_in.dtype == torch.float64:
            snrt.snrt_pn_step_f64(self.mesh, self.pn, args or self.args(torch.float64, **kw),
                                  u_in, u_out)
        else:
            snrt.snrt_pn_step(self.mesh, self.pn, args or self.args(torch.float32, **kw),
                              u_in, u_out)

    def rollout(self, u0: torch.Tensor, nsteps: int, **kw) -> torch.Tensor:
        """``nsteps`` steps from the tiled state u0 (ping-pong buffers); returns the last."""
        a = u0.clone()
        b = torch.empty_like(a)
        args = self.args(u0.dtype, **kw)
        for _ in range(nsteps):
            self.step(a, b, args)
            a, b = b, a
        return a

    def close(self):
        if getattr(self, "pn", None):
            snrt.snrt_pn_destroy(self.pn)
            self.pn = None
        if getattr(self, "mesh", None):
            snrt.snrt_mesh_destroy(self.mesh)
            self.mesh = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
