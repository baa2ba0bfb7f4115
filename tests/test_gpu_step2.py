"""GPU parity of the second-order step (limited linear reconstruction + Heun) against the
FP64 oracle's ``step2``.

All calls go through the C ABI.  Tolerances as for the first-order step: the FP64 template
follows the same arithmetic up to reassociation (1e-12 relative L2 over the run); FP32 holds
1e-5.  The limiter's branch on the sign of the reconstructed increment is continuous in its
inputs except at exact ties, which the FP64 template reproduces and which FP32 rounding only
moves by amounts covered by the FP32 tolerance.
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


def _solver(P, **kw):
    from paper_2205_08417_amd.solver import Solver
    return Solver(P, **kw)


def _oracle2(P, nsteps, neumann=False, inflow_scale=1.0, **lim):
    from oracle import oracle as o
    op = o.OracleProblem.from_problem(P, neumann=neumann)
    psi = P.psi0
    for _ in range(nsteps):
        psi = o.step2(op, psi, P.dt, inflow_scale=inflow_scale, **lim)
    return psi


def _gpu2(P, nsteps, fp64=False, lim=None, **kw):
    S = _solver(P, fp64=fp64, **kw)
    psi, _ = S.rollout(S.initial_state(torch.float64 if fp64 else torch.float32), nsteps,
                       fp64=fp64, order=2, **(lim or {}))
    out = S.to_user(psi).cpu().numpy()
    S.close()
    return out


@pytest.mark.parametrize("rho,source,inflow", [(False, False, False), (True, True, True),
                                               (False, True, True)])
def test_delaunay_isotropic_fp64_and_fp32(rho, source, inflow):
    P = small_problem(I.jittered_delaunay_mesh(13, 0.0, 1.0, seed=21), 4, 16, seed=21, rho=rho,
                      source=source, inflow=inflow, scatter=(0.3, 1.5))
    ref = _oracle2(P, 12)
    e64 = rel_l2(_gpu2(P, 12, fp64=True), ref)
    e32 = rel_l2(_gpu2(P, 12), ref)
    print(f"step2 isotropic rho={rho}: fp64 {e64:.2e} fp32 {e32:.2e}")
    assert e64 <= 1e-12
    assert e32 <= 1e-5


def test_linesource_fp32_50_steps():
    """The line-source pulse (3 872 cells x 64 ordinates): steep gradients keep the limiter
    busy on every step."""
    P = I.build("linesource_s8", nsteps=50)
    ref = _oracle2(P, 50)
    err = rel_l2(_gpu2(P, 50), ref)
    print(f"step2 line source 50 steps: {err:.2e}")
    assert err <= 1e-5


def test_quadrilateral_and_padded_meshes():
    for mesh in (I.quad_grid_mesh(11, 8), I.pad_faces(I.jittered_delaunay_mesh(9, 0.0, 1.0,
                                                                               seed=22), 4)):
        P = small_problem(mesh, 4, 16, seed=22, rho=True, source=True, inflow=True)
        ref = _oracle2(P, 6)
        assert rel_l2(_gpu2(P, 6, fp64=True), ref) <= 1e-12
        assert rel_l2(_gpu2(P, 6), ref) <= 1e-5


def test_neumann_and_inflow_scale():
    from paper_2205_08417_amd import snrt
    P = small_problem(I.jittered_delaunay_mesh(10, 0.0, 1.0, seed=23), 4, 16, seed=23, rho=True,
                      inflow=True)
    for neumann, isc in ((True, 1.0), (False, 0.4)):
        ref = _oracle2(P, 1, neumann=neumann, inflow_scale=isc)
        S = _solver(P, fp64=True)
        a = S.initial_state(torch.float64)
        b = torch.empty_like(a)
        S.step2_f64(a, b, boundary=snrt.SNRT_BC_NEUMANN if neumann else snrt.SNRT_BC_DIRICHLET,
                    inflow_scale=isc)
        assert rel_l2(S.to_user(b).cpu().numpy(), ref) <= 1e-13
        S.close()


@pytest.mark.parametrize("nq_shape,precision,tol", [((16, 16), "fp32", 1e-5),
                                                     ((16, 16), "bf16x3", 1e-4),
                                                     ((16, 32), "fp32", 1e-5),
                                                     ((16, 32), "bf16x3", 1e-4)])
def test_dense_hg(nq_shape, precision, tol):
    """HG g=0.8: 256 ordinates (whole rows per wave) and 512 ordinates (rows cut into
    256-ordinate items in both kernels)."""
    omega, w = I.product_quadrature(*nq_shape)
    K = I.henyey_greenstein_kernel(omega, w, 0.8)
    P = small_problem(I.jittered_delaunay_mesh(12, 0.0, 1.0, seed=24), omega_w=(omega, w), K=K,
                      seed=24, rho=True, inflow=True, scatter=(0.5, 1.5))
    ref = _oracle2(P, 5)
    S = _solver(P, precision=precision)
    psi, _ = S.rollout(S.initial_state(), 5, order=2)
    err = rel_l2(S.to_user(psi).cpu().numpy(), ref)
    S.close()
    print(f"step2 dense {nq_shape} {precision}: {err:.2e}")
    assert err <= tol
    if precision == "fp32":
        assert rel_l2(_gpu2(P, 5, fp64=True), ref) <= 1e-12


def test_full_size_checkerboard_one_step():
    """198 450 cells x 256 ordinates from a rough state: the launch shape of a benchmark run."""
    P = I.build("checkerboard_s16")
    P = dataclasses.replace(P, psi0=I.random_state(P.ncells, P.nq, seed=25, decades=3))
    ref = _oracle2(P, 1)
    err = rel_l2(_gpu2(P, 1), ref)
    print(f"step2 full-size checkerboard: {err:.2e}")
    assert err <= 1e-6


@pytest.mark.parametrize("vk_k", [0.0, 0.3, 5.0])
def test_venkatakrishnan_fp64_and_fp32(vk_k):
    """Venkatakrishnan's limiter (eps^2 = (K sqrt(A_i))^3): K = 0 (no threshold), a small K
    and a K at which eps is comparable to the variation of the data."""
    P = small_problem(I.jittered_delaunay_mesh(13, 0.0, 1.0, seed=27), 4, 16, seed=27, rho=True,
                      source=True, inflow=True, scatter=(0.3, 1.5))
    lim = dict(limiter="venkatakrishnan", vk_k=vk_k)
    ref = _oracle2(P, 12, **lim)
    e64 = rel_l2(_gpu2(P, 12, fp64=True, lim=lim), ref)
    e32 = rel_l2(_gpu2(P, 12, lim=lim), ref)
    print(f"step2 venkatakrishnan K={vk_k}: fp64 {e64:.2e} fp32 {e32:.2e}")
    assert e64 <= 1e-12
    assert e32 <= 1e-5
    # and it is not the Barth-Jespersen step
    assert rel_l2(_oracle2(P, 12), ref) > 1e-6


def test_venkatakrishnan_quadrilateral_padded_and_neumann():
    from paper_2205_08417_amd import snrt
    lim = dict(limiter="venkatakrishnan", vk_k=1.0)
    for mesh in (I.quad_grid_mesh(11, 8), I.pad_faces(I.jittered_delaunay_mesh(9, 0.0, 1.0,
                                                                               seed=28), 4)):
        P = small_problem(mesh, 4, 16, seed=28, rho=True, source=True, inflow=True)
        ref = _oracle2(P, 6, **lim)
        assert rel_l2(_gpu2(P, 6, fp64=True, lim=lim), ref) <= 1e-12
        assert rel_l2(_gpu2(P, 6, lim=lim), ref) <= 1e-5
        ref = _oracle2(P, 1, neumann=True, **lim)
        S = _solver(P, fp64=True)
        a = S.initial_state(torch.float64)
        b = torch.empty_like(a)
        S.step2_f64(a, b, boundary=snrt.SNRT_BC_NEUMANN, **lim)
        assert rel_l2(S.to_user(b).cpu().numpy(), ref) <= 1e-13
        S.close()


def test_venkatakrishnan_linesource_and_dense():
    """The line-source pulse over 30 FP32 steps, and dense HG scattering (512 ordinates, rows
    cut into 256-ordinate items) with the limiter."""
    lim = dict(limiter="venkatakrishnan", vk_k=0.5)
    P = I.build("linesource_s8", nsteps=30)
    err = rel_l2(_gpu2(P, 30, lim=lim), _oracle2(P, 30, **lim))
    print(f"step2 venkatakrishnan line source: {err:.2e}")
    assert err <= 1e-5
    omega, w = I.product_quadrature(16, 32)
    K = I.henyey_greenstein_kernel(omega, w, 0.8)
    P = small_problem(I.jittered_delaunay_mesh(12, 0.0, 1.0, seed=29), omega_w=(omega, w), K=K,
                      seed=29, rho=True, inflow=True, scatter=(0.5, 1.5))
    ref = _oracle2(P, 4, **lim)
    assert rel_l2(_gpu2(P, 4, lim=lim), ref) <= 1e-5
    assert rel_l2(_gpu2(P, 4, fp64=True, lim=lim), ref) <= 1e-12


def test_limiter_arguments_are_checked():
    from paper_2205_08417_amd import snrt
    P = small_problem(I.jittered_delaunay_mesh(8, 0.0, 1.0, seed=30), 4, 16, seed=30)
    S = _solver(P)
    psi = S.initial_state()
    out = torch.empty_like(psi)
    ws, n = S._ws2(False)
    bad = [snrt.Limiter(2, 0, 1.0), snrt.Limiter(1, 1, 1.0), snrt.Limiter(1, 0, -1.0),
           snrt.Limiter(1, 0, float("nan")), snrt.Limiter(1, 0, float("inf"))]
    for lim in bad:
        with pytest.raises(snrt.SnrtError) as ei:
            snrt.snrt_step2_limited(S.mesh, S.quad, S.scatter, S.args(), lim, psi, out, ws, n)
        assert ei.value.status == snrt.SNRT_E_ARG
    # NULL and an explicit Barth-Jespersen selector are the plain second-order step
    ref = torch.empty_like(psi)
    snrt.snrt_step2(S.mesh, S.quad, S.scatter, S.args(), psi, ref, ws, n)
    for lim in (None, snrt.limiter("barth-jespersen", 7.0)):
        snrt.snrt_step2_limited(S.mesh, S.quad, S.scatter, S.args(), lim, psi, out, ws, n)
        assert torch.equal(out, ref)
    with pytest.raises(ValueError):
        snrt.limiter("minmod")
    S.close()


def test_renumbering_is_bitwise_invisible():
    P = I.build("checkerboard_s16", n_side=40, nsteps=10)
    assert np.array_equal(_gpu2(P, 10, reorder=True), _gpu2(P, 10, reorder=False))


def test_needs_midpoints_and_workspace():
    from paper_2205_08417_amd import snrt
    P = small_problem(I.jittered_delaunay_mesh(8, 0.0, 1.0, seed=26), 4, 16, seed=26)
    S = _solver(P)
    psi = S.initial_state()
    out = torch.empty_like(psi)
    ws, n = S._ws2(False)
    with pytest.raises(snrt.SnrtError) as ei:
        snrt.snrt_step2(S.mesh, S.quad, S.scatter, S.args(), psi, out, ws, n - 4)
    assert "workspace" in str(ei.value)
    m = P.mesh
    bare = snrt.snrt_mesh_create(m.face_nbr, m.face_normal, m.area, m.centroid, m.nbfaces)
    with pytest.raises(snrt.SnrtError) as ei:
        snrt.snrt_step2(bare, S.quad, S.scatter, S.args(), psi, out, ws, n)
    assert "snrt_mesh_set_face_midpoints" in str(ei.value)
    nocen = snrt.snrt_mesh_create(m.face_nbr, m.face_normal, m.area, None, m.nbfaces,
                                  snrt.SNRT_NO_REORDER)
    with pytest.raises(snrt.SnrtError) as ei:
        snrt.snrt_mesh_set_face_midpoints(nocen, m.face_mid)
    assert ei.value.status == snrt.SNRT_E_ARG
    snrt.snrt_mesh_destroy(bare)
    snrt.snrt_mesh_destroy(nocen)
    S.close()
