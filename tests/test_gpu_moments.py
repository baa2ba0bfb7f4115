"""GPU parity of moment-projected scattering O Sigma M (eq. SNEqns2) against the oracle,
which applies the same operator as the dense kernel sum_j m_j(Omega_q) sigma_j m_j(Omega_p)
built from its own (pinned) spherical harmonics.

Tolerances as for dense scattering: FP64 template 1e-12, FP32 1e-5, BF16 hi+lo 1e-4.
"""
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


def _oracle_problem(P, sigma_l, **kw):
    from oracle import moments as mo
    from oracle import oracle as o
    return o.OracleProblem.from_problem(P, K=mo.moment_kernel(P.omega, P.w, sigma_l), **kw)


def _problem(npol, naz, seed, **kw):
    omega, w = I.product_quadrature(npol, naz)
    return small_problem(I.jittered_delaunay_mesh(12, 0.0, 1.0, seed=seed), omega_w=(omega, w),
                         seed=seed, scatter=(0.5, 1.5), **kw)


@pytest.mark.parametrize("npol,naz,N,precision,tol", [
    (8, 8, 4, "fp32", 1e-5), (16, 16, 8, "fp32", 1e-5), (16, 16, 8, "bf16x3", 1e-4),
    (16, 32, 8, "fp32", 1e-5), (16, 32, 8, "bf16x3", 1e-4), (16, 16, 15, "bf16x3", 1e-4)])
def test_moment_rollout_vs_oracle(npol, naz, N, precision, tol):
    from oracle import oracle as o
    P = _problem(npol, naz, seed=31 + N, rho=True, inflow=True, source=True)
    sig = I.hg_legendre_moments(0.85, N)
    op = _oracle_problem(P, sig)
    ref = o.rollout(op, P.psi0, P.dt, 10)[0]
    S = _solver(P, precision=precision, moments=sig)
    psi, _ = S.rollout(S.initial_state(), 10)
    err = rel_l2(S.to_user(psi).cpu().numpy(), ref)
    print(f"moments N={N} nq={npol * naz} {precision}: {err:.2e}")
    assert err <= tol
    if precision == "fp32":
        psi64, _ = S.rollout(S.initial_state(torch.float64), 10, fp64=True)
        assert rel_l2(S.to_user(psi64).cpu().numpy(), ref) <= 1e-12
    S.close()


def test_isotropic_moment_set_equals_isotropic_path():
    P = _problem(8, 8, seed=40, inflow=True)
    S1 = _solver(P, moments=[1.0])
    S2 = _solver(P)
    a, _ = S1.rollout(S1.initial_state(torch.float64), 5, fp64=True)
    b, _ = S2.rollout(S2.initial_state(torch.float64), 5, fp64=True)
    assert rel_l2(S1.to_user(a).cpu().numpy(), S2.to_user(b).cpu().numpy()) <= 1e-13


@pytest.mark.parametrize("fp64,tol", [(True, 1e-12), (False, 1e-5)])
def test_adjoint_step_with_moments(fp64, tol):
    from oracle import oracle as o
    P = _problem(16, 16, seed=41, rho=True)
    sig = I.hg_legendre_moments(0.7, 6)
    op = _oracle_problem(P, sig)
    rng = np.random.default_rng(3)
    lam = rng.standard_normal((P.ncells, P.nq))
    gt, gs, gr = np.zeros(P.ncells), np.zeros(P.ncells), np.zeros(P.ncells)
    ref = o.adjoint_step(op, P.psi0, lam, P.dt, 1.1, 0.9, gt, gs, gr)
    S = _solver(P, fp64=fp64, moments=sig)
    dt = torch.float64 if fp64 else torch.float32
    psi = S.to_internal(P.psi0, dt)
    l1 = S.to_internal(lam, dt)
    l0 = torch.empty_like(l1)
    g = [torch.zeros(P.ncells, dtype=dt, device="cuda") for _ in range(3)]
    fn = S.adjoint_step_f64 if fp64 else S.adjoint_step
    fn(psi, l1, l0, g[0], g[1], g[2], alpha_t=1.1, alpha_s=0.9)
    assert rel_l2(S.to_user(l0).cpu().numpy(), ref) <= tol
    for gg, rr in zip(g, (gt, gs, gr)):
        got = S.to_user(gg.reshape(S.nc, 1)).cpu().numpy().ravel()
        assert rel_l2(got, rr) <= tol
    S.close()


def test_second_order_step_with_moments():
    from oracle import oracle as o
    P = _problem(16, 16, seed=42, inflow=True)
    sig = I.hg_legendre_moments(0.8, 8)
    ref = o.step2(_oracle_problem(P, sig), P.psi0, P.dt)
    for precision, tol in (("fp32", 1e-5), ("bf16x3", 1e-4)):
        S = _solver(P, precision=precision, moments=sig)
        a = S.initial_state()
        b = torch.empty_like(a)
        S.step2(a, b)
        assert rel_l2(S.to_user(b).cpu().numpy(), ref) <= tol
        S.close()


def test_full_size_line_source_moments_sampled():
    """100 352 cells x 1024 ordinates, HG g=0.9 to degree 8 (81 moments), BF16 hi+lo, in the
    benchmark's launch shape; one step from the pulse, sampled cells checked one by one."""
    from oracle import oracle as o
    P = I.build("linesource_hg_s32")
    sig = I.hg_legendre_moments(0.9, 8)
    S = _solver(P, precision="bf16x3", moments=sig)
    psi, _ = S.rollout(S.initial_state(), 1)
    out = S.to_user(psi).cpu().numpy()
    S.close()
    rng = np.random.default_rng(1)
    hot = np.nonzero(np.sum(P.mesh.centroid ** 2, axis=1) < 0.01)[0]
    cells = np.unique(np.concatenate([hot[:100], rng.choice(P.ncells, 100, False)]))
    ref = o.step(_oracle_problem(P, sig), P.psi0, P.dt, cells=cells)
    err = rel_l2(out[cells], ref)
    print(f"moments full-size sampled: {err:.2e}")
    assert err <= 1e-4


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-6), ("bf16x3", 1e-5), ("fp16x3", 1e-6)])
@pytest.mark.parametrize("transpose", [0, 1])
def test_scatter_apply_moment_form(precision, tol, transpose):
    """snrt_scatter_apply of the moment form (with its workspace) against the equivalent
    dense kernel built by the oracle's own harmonics; the transposed product too.  A
    workspace is required."""
    from oracle import moments as mo
    from paper_2205_08417_amd import snrt
    P = _problem(16, 16, seed=43)
    sig = I.hg_legendre_moments(0.8, 6)
    S = _solver(P, moments=sig, precision=precision)
    rng = np.random.default_rng(44)
    x = torch.tensor(rng.uniform(0.0, 1.0, (P.ncells, P.nq)), dtype=torch.float32, device="cuda")
    out = torch.empty_like(x)
    with pytest.raises(snrt.SnrtError) as ei:
        snrt.snrt_scatter_apply(S.mesh, S.quad, S.scatter, x, out, transpose)
    assert ei.value.status == snrt.SNRT_E_ARG
    snrt.snrt_scatter_apply(S.mesh, S.quad, S.scatter, x, out, transpose, S.ws, S.ws_bytes)
    Kd = mo.moment_kernel(P.omega, P.w, sig)
    B = P.w[:, None] * Kd.T                      # S = Psi B, B[p][q] = w_p K[q][p]
    xs = x.cpu().numpy().astype(np.float64)
    ref = xs @ (B if transpose == 0 else B.T)
    err = rel_l2(out.cpu().numpy(), ref)
    print(f"moment-form product {precision} transpose={transpose}: {err:.2e}")
    assert err <= tol
    S.close()
