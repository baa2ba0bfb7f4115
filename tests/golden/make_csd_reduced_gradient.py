"""Writes csd_reduced_gradient.npz: the FP64 oracle's dose and dose-functional gradients for
the reduced CSD dose workload (the full 20 -> 0.1 MeV energy range).

Workload: phantom of 51 x 51 jittered points on [0, 10]^2 cm (5 000 triangles, seed 1005),
8 x 8 product quadrature (64 ordinates), column-normalised Henyey-Greenstein kernel g = 0.95,
densities water 1 / bone 1.85 / air raised to 0.05, beam inflow scaled by S(E_n) G_E(E_n),
explicit steps at CFL 0.5 in pseudo-time from E = 20 to E = 0.1 MeV, the FP64 dose
accumulated before every step.  Functional J = sum_T A_i D_i - sum_O A_i D_i over the target
[4.5, 5.5] x [2, 3] and the organ [6, 7] x [2, 3].

Only the oracle and the seeded input generators are called.  Run from the repository root:
    python tests/golden/make_csd_reduced_gradient.py
"""
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as o                      # noqa: E402
from paper_2205_08417_amd import inputs as I        # noqa: E402

OUT = os.path.join(HERE, "csd_reduced_gradient.npz")
SPEC = dict(n_side=51, n_polar=8, n_azimuth=8, nsteps=None, rho_air=0.05)
CKPT = 126


def problem():
    return I.build("csd_phantom_s512", **SPEC)


def functional_weights(P):
    T = P.meta["target"].astype(float)
    O = P.meta["organ"].astype(float)
    return P.mesh.area * (T - O)


def input_digest(P) -> str:
    """Hash of the arrays that define the run (mesh, materials, inflow, schedule)."""
    h = hashlib.sha256()
    for a in (P.mesh.face_nbr, P.mesh.face_normal, P.mesh.area, P.rho, P.K, P.inflow,
              np.asarray(P.meta["inflow_scale"]), np.asarray(P.meta["dose_coeff"]),
              np.asarray([P.dt, P.nsteps], dtype=np.float64)):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def main():
    P = problem()
    print(f"{P.ncells} cells x {P.nq} ordinates, {P.nsteps} steps, dt = {P.dt:.6e}, "
          f"{o.num_threads()} threads", flush=True)
    t0 = time.time()
    g = o.rollout_gradient(o.OracleProblem.from_problem(P), P.psi0, P.dt, P.nsteps,
                           dJ_ddose=functional_weights(P),
                           inflow_scale=np.asarray(P.meta["inflow_scale"]),
                           dose_coeff=np.asarray(P.meta["dose_coeff"]), ckpt_every=CKPT)
    print(f"oracle reverse pass: {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(OUT, dose=g["dose"], g_rho=g["rho"], g_sigma_t=g["sigma_t"],
                        g_sigma_s=g["sigma_s"], digest=np.array(input_digest(P)),
                        nsteps=np.array(P.nsteps), ncells=np.array(P.ncells))
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
