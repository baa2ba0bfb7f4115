"""snrt_step_dose_noalloc (the fused dose step whose dose partials live in the library's static
device scratch) against snrt_step_dose, through the C ABI: two calls in a row, the second on
a smaller problem, each bitwise equal in the new state and the dose; and its refusals (dense
scattering, more cells than the scratch holds) before any launch."""
import ctypes

import numpy as np
import pytest

from _util import small_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2205_08417_amd import inputs as I  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2205_08417_amd import snrt
    snrt.lib()


def _both(P, coeff, seed):
    """(noalloc state, noalloc dose), (workspace state, workspace dose) from one input."""
    from paper_2205_08417_amd import snrt
    from paper_2205_08417_amd.solver import Solver
    S = Solver(P)
    print(f"noalloc vs workspace dose step: {P.ncells} cells x {P.nq} ordinates", flush=True)
    rng = np.random.default_rng(seed)
    psi = S.to_internal(rng.uniform(0.0, 1.0, (P.ncells, P.nq)))
    dose0 = torch.tensor(rng.uniform(0.0, 1.0, P.ncells), dtype=torch.float64, device="cuda")
    args = S.args()
    out_a, out_b = torch.empty_like(psi), torch.empty_like(psi)
    dose_a, dose_b = dose0.clone(), dose0.clone()
    snrt.snrt_step_dose_noalloc(S.mesh, S.quad, S.scatter, args, psi, out_a, coeff, dose_a)
    ws = torch.empty(max(S.ws_bytes, 16), dtype=torch.uint8, device="cuda")
    snrt.snrt_step_dose(S.mesh, S.quad, S.scatter, args, psi, out_b, coeff, dose_b, ws,
                        S.ws_bytes)
    torch.cuda.synchronize()
    S.close()
    return (out_a.cpu(), dose_a.cpu()), (out_b.cpu(), dose_b.cpu())


def test_noalloc_dose_step_matches_workspace_version_twice():
    big = small_problem(I.jittered_delaunay_mesh(60, 0.0, 1.0, seed=71), npol=16, naz=16,
                        rho=True, source=True, inflow=True, seed=71)
    small = small_problem(I.jittered_delaunay_mesh(17, 0.0, 1.0, seed=72), npol=8, naz=8,
                          rho=True, seed=72)
    assert small.ncells < big.ncells
    for P, coeff, seed in ((big, 0.37, 1), (small, 1.9, 2)):
        (sa, da), (sb, db) = _both(P, coeff, seed)
        assert torch.equal(sa, sb)
        assert torch.equal(da, db)
        assert float(torch.max(torch.abs(da))) > 0.0


def test_noalloc_refuses_dense_and_oversize_meshes():
    from paper_2205_08417_amd import snrt
    from paper_2205_08417_amd.solver import Solver
    omega, w = I.product_quadrature(16, 16)
    P = small_problem(I.jittered_delaunay_mesh(8, 0.0, 1.0, seed=73), omega_w=(omega, w),
                      K=I.henyey_greenstein_kernel(omega, w, 0.5), seed=73)
    S = Solver(P)
    psi = S.initial_state()
    out = torch.empty_like(psi)
    dose = torch.zeros(P.ncells, dtype=torch.float64, device="cuda")
    with pytest.raises(snrt.SnrtError, match="product workspace"):
        snrt.snrt_step_dose_noalloc(S.mesh, S.quad, S.scatter, S.args(), psi, out, 1.0, dose)
    S.close()
    # one cell more than the scratch holds: refused before any array is touched
    m = I.quad_grid_mesh(1025, 1024)
    assert m.ncells > 1 << 20
    mesh = snrt.snrt_mesh_create(m.face_nbr, m.face_normal, m.area, None, m.nbfaces,
                                 snrt.SNRT_NO_REORDER)
    quad = snrt.snrt_quad_create(*I.product_quadrature(1, 2))
    iso = snrt.snrt_scatter_isotropic(quad)
    L = snrt.lib()
    args = snrt.StepArgs()
    st = L.snrt_step_dose_noalloc(mesh, quad, iso, ctypes.byref(args), None, None, 1.0, None,
                                  None)
    assert st == snrt.SNRT_E_UNSUPPORTED
    assert "static scratch" in snrt.snrt_last_error()
    snrt.snrt_scatter_destroy(iso)
    snrt.snrt_quad_destroy(quad)
    snrt.snrt_mesh_destroy(mesh)
