"""Shared helpers of the GPU parity tests (inputs from the seeded generators only)."""
import numpy as np

from paper_2205_08417_amd import inputs as I


def small_problem(mesh, npol=4, naz=8, seed=0, K=None, rho=False, source=False, inflow=False,
                  sigma=(0.5, 2.0), scatter=(0.0, 1.0), nsteps=10, cfl=0.4, omega_w=None):
    """Random materials on a given mesh; a positive random initial state."""
    rng = np.random.default_rng(seed)
    if omega_w is None:
        omega, w = I.product_quadrature(npol, naz)
    else:
        omega, w = omega_w
    nc, nq = mesh.ncells, w.size
    r = rng.uniform(0.5, 2.0, nc) if rho else None
    return I.Problem(name="random", mesh=mesh, omega=omega, w=w, K=K,
                     sigma_t=rng.uniform(*sigma, nc), sigma_s=rng.uniform(*scatter, nc), rho=r,
                     source=rng.uniform(0, 1, nc) if source else None,
                     inflow=rng.uniform(0, 1, (mesh.nbfaces, nq)) if inflow else None,
                     psi0=rng.uniform(0, 1, (nc, nq)), dt=I.cfl_dt(mesh, omega, cfl, r),
                     nsteps=nsteps)


def rel_l2(x, ref):
    x = np.asarray(x, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    n = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / (n if n > 0 else 1.0))
