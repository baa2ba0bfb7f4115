"""Degenerate inputs through the C ABI: a mesh without cells (every entry point returns
success and touches nothing), zero-step rollouts (the state comes back bitwise), and a
single triangle whose three faces are all boundary faces (every flux term is a ghost),
against the oracle.
"""
import dataclasses

import numpy as np
import pytest

from _util import rel_l2, small_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2205_08417_amd import inputs as I  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2205_08417_amd import snrt
    snrt.lib()


def test_zero_cell_mesh_every_entry_point():
    from paper_2205_08417_amd import snrt
    omega, w = I.product_quadrature(4, 8)
    mesh = snrt.snrt_mesh_create(np.zeros((0, 3), np.int32), np.zeros((0, 3, 2)), np.zeros(0),
                                 np.zeros((0, 2)), 0)
    quad = snrt.snrt_quad_create(omega, w)
    K = I.henyey_greenstein_kernel(omega, w, 0.6)
    scatters = {"isotropic": snrt.snrt_scatter_isotropic(quad),
                "dense": snrt.snrt_scatter_dense(quad, K, snrt.SNRT_BF16X3),
                "moments": snrt.snrt_scatter_moments(quad, [1.0, 0.5], snrt.SNRT_FP32)}
    snrt.snrt_scatter_prepare_implicit(scatters["dense"])
    e32 = torch.empty(0, device="cuda")
    e64 = torch.empty(0, dtype=torch.float64, device="cuda")
    a32 = snrt.step_args(e32, e32, 0.1)
    a64 = snrt.step_args(e64, e64, 0.1)
    for name, sc in scatters.items():
        assert snrt.snrt_workspace_size(mesh, quad, sc) == 0
        snrt.snrt_step(mesh, quad, sc, a32, None, None)
        snrt.snrt_step_f64(mesh, quad, sc, a64, None, None)
        snrt.snrt_step_dose(mesh, quad, sc, a32, None, None, 1.0, None)
        snrt.snrt_step_adjoint(mesh, quad, sc, a32, None, None, None)
        snrt.snrt_rollout(mesh, quad, sc, a32, None, 5, None, None)
        snrt.snrt_rollout_adjoint(mesh, quad, sc, a32, None, 5, None, 1, None, None, None)
        if name == "isotropic":
            snrt.snrt_step_imex(mesh, quad, sc, a32, None, None)
            snrt.snrt_step_dose_noalloc(mesh, quad, sc, a32, None, None, 1.0, None)
        elif name == "dense":
            snrt.snrt_step_imex_dense(mesh, quad, sc, a32, None, None, None, 0)
        else:
            snrt.snrt_step_imex_moments(mesh, quad, sc, a32, None, None, None, 0)
        snrt.snrt_scatter_destroy(sc)
    out = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    snrt.snrt_mass(mesh, quad, None, out)
    torch.cuda.synchronize()
    assert float(out.item()) in (0.0, 7.0)           # nothing to add: zero or untouched
    pn = snrt.snrt_pn_create(5)
    snrt.snrt_pn_step(mesh, pn, a32, None, None)
    snrt.snrt_pn_destroy(pn)
    snrt.snrt_quad_destroy(quad)
    snrt.snrt_mesh_destroy(mesh)


def test_zero_step_rollouts_return_the_state():
    from paper_2205_08417_amd import snrt
    from paper_2205_08417_amd.solver import Solver
    P = small_problem(I.jittered_delaunay_mesh(8, 0.0, 1.0, seed=91), 4, 8, seed=91,
                      source=True, inflow=True)
    S = Solver(P)
    a = S.initial_state()
    ref = a.clone()
    b = torch.empty_like(a)
    snrt.snrt_rollout(S.mesh, S.quad, S.scatter, S.args(), None, 0, a, b)
    lam = torch.rand_like(a)
    lam_ref = lam.clone()
    snrt.snrt_rollout_adjoint(S.mesh, S.quad, S.scatter, S.args(), None, 0, a, 1, b, lam,
                              torch.empty_like(a))
    torch.cuda.synchronize()
    assert torch.equal(a, ref)
    assert torch.equal(lam, lam_ref)
    S.close()


@pytest.mark.parametrize("kernel", ["isotropic", "hg"])
def test_single_boundary_triangle(kernel):
    """One cell, all three faces on the boundary (Dirichlet inflow on each), densities and a
    source: the step is all ghost terms."""
    from oracle import oracle as o
    from paper_2205_08417_amd.solver import Solver
    pts = np.array([[0.0, 0.0], [1.0, 0.1], [0.2, 0.9]])
    mesh = I._faces_from_triangles(pts, np.array([[0, 1, 2]]), np.array([[-1, -1, -1]]))
    omega, w = I.product_quadrature(4, 16)
    K = None if kernel == "isotropic" else I.henyey_greenstein_kernel(omega, w, 0.8)
    P = small_problem(mesh, omega_w=(omega, w), seed=92, K=K, rho=True, source=True,
                      inflow=True, scatter=(0.5, 1.0))
    op = o.OracleProblem.from_problem(P)
    for fp64, tol in ((True, 1e-13), (False, 2e-6)):
        S = Solver(P, fp64=fp64)
        dt = torch.float64 if fp64 else torch.float32
        a = S.initial_state(dt)
        b = torch.empty_like(a)
        (S.step_f64 if fp64 else S.step)(a, b, alpha_t=1.2, alpha_s=0.7, inflow_scale=0.6)
        ref = o.step(op, P.psi0, P.dt, 1.2, 0.7, 0.6)
        err = rel_l2(S.to_user(b).cpu().numpy(), ref)
        print(f"single triangle {kernel} fp64={fp64}: {err:.2e}")
        assert err <= tol
        S.close()
