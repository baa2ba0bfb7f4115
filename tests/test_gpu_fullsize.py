"""GPU parity at full workload sizes and on the kernels' wide-row paths, against the FP64 oracle.

- The transposed step on the full adjoint checkerboard (51 842 cells x 256 ordinates, the
  persistent pipelined kernel in the launch shape the benchmark times): the adjoint state
  and all three gradient contributions element by element.
- The one-launch dense transposed step on the full CSD phantom (299 538 x 512, BF16 hi+lo):
  the adjoint state and the three gradients of every cell.
- The wide-row adjoint kernel (more than 32 bytes of a row per lane: FP32 at 1024
  ordinates, FP64 at 512), isotropic and dense, with density and both boundary modes.
- A 40-step differentiable rollout on the full adjoint mesh (checkpoints every 20) against
  the oracle's reverse pass, and central differences of the full 400-step workload on 20
  seeded cells per cross section (FP64 template for the differences).
- The mixed-precision products over 200 steps at 1024 ordinates against the oracle.
- The reduced CSD dose workload over its whole energy range (5 000 cells, 64 ordinates,
  15 812 steps, checkpoints every 20) with the mixed-precision products: dose and the
  gradient of the target-minus-organ dose functional w.r.t. density against the oracle's
  values stored by tests/golden/make_csd_reduced_gradient.py.

Element-wise bounds are |x - ref| <= rtol |ref| + atol with atol a small fraction of the
largest |ref| (the floor covers entries that are sums of terms of both signs); the worst
entry is printed.
"""
import numpy as np
import pytest

from _util import rel_l2

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


def _cells_user(S, x):
    return S.to_user(x.reshape(S.nc, -1)).cpu().numpy().reshape(S.nc, -1).squeeze(-1)


def check_elementwise(name, x, ref, rtol, atol_frac):
    x = np.asarray(x, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    atol = atol_frac * float(np.max(np.abs(ref)))
    err = np.abs(x - ref)
    excess = err - (rtol * np.abs(ref) + atol)
    k = int(np.argmax(excess))
    print(f"{name}: rel-L2 {rel_l2(x, ref):.2e}, max|err|/max|ref| "
          f"{float(np.max(err)) / max(float(np.max(np.abs(ref))), 1e-300):.2e}, worst entry {k}: "
          f"{x[k]:.6e} vs {ref[k]:.6e}")
    assert excess[k] <= 0.0, name


def _detector_weights(P):
    region = I.region_mask(P.mesh, P.meta["detector"])
    return (region * P.mesh.area)[:, None] * P.w[None, :]


# ------------------------------------------------------------------ one transposed step

@pytest.mark.parametrize("signed,neumann", [(False, False), (True, True)])
def test_adjoint_step_full_size_elementwise(signed, neumann):
    """Full adjoint checkerboard with a random density: lam_n, g_sigma_t, g_sigma_s, g_rho of
    one snrt_step_adjoint against oracle.adjoint_step.  Positive states and adjoint states
    make the gradient sums free of cancellation (relative bound only); the signed case has
    a floor."""
    from oracle import oracle as o
    from paper_2205_08417_amd import snrt
    P = I.build("checkerboard_adjoint_s16")
    rng = np.random.default_rng(11)
    P.rho = rng.uniform(0.5, 2.0, P.ncells)
    P.source = None
    psi = I.random_state(P.ncells, P.nq, seed=12, decades=3)
    lam = (rng.standard_normal((P.ncells, P.nq)) if signed
           else rng.uniform(0.5, 1.5, (P.ncells, P.nq)))
    at, as_ = 1.1, 0.9
    print(f"full adjoint step: {P.ncells} cells x {P.nq} ordinates, signed={signed}, "
          f"neumann={neumann}", flush=True)
    op = o.OracleProblem.from_problem(P, neumann=neumann)
    gt, gs, gr = np.zeros(P.ncells), np.zeros(P.ncells), np.zeros(P.ncells)
    ref = o.adjoint_step(op, psi, lam, P.dt, at, as_, gt, gs, gr)
    S = _solver(P)
    bc = snrt.SNRT_BC_NEUMANN if neumann else snrt.SNRT_BC_DIRICHLET
    p = S.to_internal(psi)
    l1 = S.to_internal(lam)
    l0 = torch.empty_like(l1)
    g = [torch.zeros(P.ncells, dtype=torch.float32, device="cuda") for _ in range(3)]
    S.adjoint_step(p, l1, l0, g[0], g[1], g[2], alpha_t=at, alpha_s=as_, boundary=bc)
    check_elementwise("lam_n", S.to_user(l0).cpu().numpy(), ref, 1e-5, 1e-6)
    grad_rtol, grad_floor = (1e-5, 1e-6) if signed else (1e-5, 0.0)
    check_elementwise("g_sigma_t", _cells_user(S, g[0]), gt, grad_rtol, grad_floor)
    check_elementwise("g_sigma_s", _cells_user(S, g[1]), gs, grad_rtol, grad_floor)
    check_elementwise("g_rho", _cells_user(S, g[2]), gr, 1e-5, 1e-6)
    S.close()


def test_csd_transposed_step_full_size_one_launch():
    """The dense transposed step at the full CSD phantom's size (299 538 cells x 512
    ordinates, HG g = 0.95, densities, BF16 hi+lo) in the form the dose-gradient benchmark
    runs it: one launch of the transposed product whose tiles update lam_n (256 x 256 tiles
    and the last round's smaller ones), and the fold of the gradient pieces.  Every element
    of lam_n and every cell's three gradients against oracle.adjoint_step over the whole
    mesh.  Positive states and adjoint states: no cancellation in the gradient sums."""
    from oracle import oracle as o
    P = I.build("csd_phantom_s512")
    rng = np.random.default_rng(21)
    P.source = None
    psi = I.random_state(P.ncells, P.nq, seed=22, decades=3)
    lam = rng.uniform(0.5, 1.5, (P.ncells, P.nq))
    # the device's FP32 inputs, so that only the step's own arithmetic differs
    psi = psi.astype(np.float32).astype(np.float64)
    lam = lam.astype(np.float32).astype(np.float64)
    at, as_ = 1.1, 0.9
    S = _solver(P, precision="bf16x3")
    print(f"CSD transposed step: {P.ncells} cells x {P.nq} ordinates, BF16x3", flush=True)
    p = S.to_internal(psi)
    l1 = S.to_internal(lam)
    l0 = torch.empty_like(l1)
    g = [torch.zeros(P.ncells, dtype=torch.float32, device="cuda") for _ in range(3)]
    S.adjoint_step(p, l1, l0, g[0], g[1], g[2], alpha_t=at, alpha_s=as_)
    torch.cuda.synchronize()
    got = S.to_user(l0).cpu().numpy()
    gg = [_cells_user(S, x) for x in g]
    S.close()
    del p, l1, l0, g
    print("oracle transposed step over the whole mesh", flush=True)
    op = o.OracleProblem.from_problem(P)
    gt, gs, gr = np.zeros(P.ncells), np.zeros(P.ncells), np.zeros(P.ncells)
    ref = o.adjoint_step(op, psi, lam, P.dt, at, as_, gt, gs, gr)
    check_elementwise("lam_n", got, ref, 1e-5, 1e-6)
    check_elementwise("g_sigma_t", gg[0], gt, 1e-5, 0.0)
    check_elementwise("g_sigma_s", gg[1], gs, 1e-5, 1e-7)
    check_elementwise("g_rho", gg[2], gr, 1e-5, 1e-6)


@pytest.mark.parametrize("fp64,nq,dense,rho,neumann", [
    (False, 1024, False, True, False),
    (False, 1024, True, True, False),
    (False, 1024, False, False, True),
    (True, 512, True, True, False),
    (True, 512, False, True, True),
])
def test_adjoint_wide_rows_vs_oracle(fp64, nq, dense, rho, neumann):
    """The one-wave-per-cell adjoint kernel of wide rows, on a 12 x 12-point mesh (222
    cells, a ragged last block), element by element."""
    from oracle import oracle as o
    from paper_2205_08417_amd import snrt
    from _util import small_problem
    npol, naz = (32, 32) if nq == 1024 else (16, 32)
    omega, w = I.product_quadrature(npol, naz)
    K = I.henyey_greenstein_kernel(omega, w, 0.8) if dense else None
    P = small_problem(I.jittered_delaunay_mesh(12, 0.0, 1.0, seed=61), omega_w=(omega, w), K=K,
                      rho=rho, seed=61, scatter=(0.2, 1.0))
    rng = np.random.default_rng(62)
    lam = rng.standard_normal((P.ncells, P.nq))
    print(f"wide adjoint: fp64={fp64} nq={nq} dense={dense} rho={rho} neumann={neumann}",
          flush=True)
    op = o.OracleProblem.from_problem(P, neumann=neumann)
    gt, gs = np.zeros(P.ncells), np.zeros(P.ncells)
    gr = np.zeros(P.ncells) if rho else None
    ref = o.adjoint_step(op, P.psi0, lam, P.dt, 1.2, 0.8, gt, gs, gr)
    S = _solver(P, fp64=fp64)
    dt = torch.float64 if fp64 else torch.float32
    psi = S.to_internal(P.psi0, dt)
    l1 = S.to_internal(lam, dt)
    l0 = torch.empty_like(l1)
    g = [torch.zeros(P.ncells, dtype=dt, device="cuda") for _ in range(3)]
    fn = S.adjoint_step_f64 if fp64 else S.adjoint_step
    bc = snrt.SNRT_BC_NEUMANN if neumann else snrt.SNRT_BC_DIRICHLET
    fn(psi, l1, l0, g[0], g[1], g[2] if rho else None, alpha_t=1.2, alpha_s=0.8, boundary=bc)
    rtol, floor = (1e-12, 1e-13) if fp64 else (1e-5, 1e-6)
    check_elementwise("lam_n", S.to_user(l0).cpu().numpy(), ref, rtol, floor)
    check_elementwise("g_sigma_t", _cells_user(S, g[0]), gt, rtol, floor)
    check_elementwise("g_sigma_s", _cells_user(S, g[1]), gs, rtol, floor)
    if rho:
        check_elementwise("g_rho", _cells_user(S, g[2]), gr, rtol, floor)
    S.close()


# ------------------------------------------------------------------ differentiable rollouts

def _gpu_gradients(S, P, nsteps, ckpt, fp64=False):
    from paper_2205_08417_amd.solver import differentiable_rollout
    dt = torch.float64 if fp64 else torch.float32
    psi0 = S.to_internal(P.psi0, dt).requires_grad_(True)
    st = S.cells_to_internal(P.sigma_t, dt).requires_grad_(True)
    ss = S.cells_to_internal(P.sigma_s, dt).requires_grad_(True)
    W = S.to_internal(_detector_weights(P), dt)
    psiN = differentiable_rollout(S, psi0, nsteps, st, ss, ckpt_every=ckpt)
    J = torch.sum(W * psiN)
    J.backward()
    return {"J": float(J), "psi0": S.to_user(psi0.grad).cpu().numpy(),
            "sigma_t": _cells_user(S, st.grad), "sigma_s": _cells_user(S, ss.grad)}


def test_rollout_gradient_full_size_40_steps_vs_oracle():
    """Full adjoint mesh (51 842 x 256), 40 steps from a random state, checkpoints every 20;
    J = integrated scalar flux over [5,6] x [3,4]: every gradient against the oracle's
    reverse pass (rel-L2 <= 1e-4 and element-wise)."""
    from oracle import oracle as o
    P = I.build("checkerboard_adjoint_s16", nsteps=40)
    P.psi0 = I.random_state(P.ncells, P.nq, seed=13, decades=2)
    print(f"full-size 40-step gradient: {P.ncells} x {P.nq}", flush=True)
    ref = o.rollout_gradient(o.OracleProblem.from_problem(P), P.psi0, P.dt, 40,
                             dJ_dpsiN=_detector_weights(P), ckpt_every=20)
    S = _solver(P)
    g = _gpu_gradients(S, P, 40, 20)
    S.close()
    for k in ("sigma_t", "sigma_s", "psi0"):
        assert rel_l2(g[k], ref[k]) <= 1e-4, k
        check_elementwise(f"gradient {k}", g[k], ref[k], 1e-4, 1e-5)


def test_central_fd_full_workload_400_steps():
    """The full adjoint workload (51 842 x 256, 400 steps from the empty state, source in
    the centre square, checkpoints every 20): the FP32 gradients of J w.r.t. sigma_t and
    sigma_s on 20 seeded cells each (drawn among |g| >= 1e-3 max|g|) against central
    differences h = 1e-4 max(|theta|, 1) of the FP64 template, and the FP64 adjoint
    gradients against the same differences."""
    from paper_2205_08417_amd import snrt
    P = I.build("checkerboard_adjoint_s16")
    n = P.nsteps
    print(f"full-size FD: {P.ncells} x {P.nq}, {n} steps", flush=True)
    S = _solver(P, fp64=True)
    g32 = _gpu_gradients(S, P, n, 20)
    g64 = _gpu_gradients(S, P, n, 20, fp64=True)
    W = S.to_internal(_detector_weights(P), torch.float64)
    psi0 = S.to_internal(P.psi0, torch.float64)
    tmp = torch.empty_like(psi0)
    M = S.mats64

    def J(attr, cell, h):
        arr = getattr(P, attr).copy()
        arr[cell] += h
        t = S.cells_to_internal(arr, torch.float64)
        mats = dict(M)
        mats[attr] = t
        psi = psi0.clone()
        snrt.snrt_rollout_f64(S.mesh, S.quad, S.scatter, S.args(mats=mats), None, n, psi, tmp,
                              None, 1, S.ws, S.ws_bytes)
        return float(torch.sum(W * psi))

    rng = np.random.default_rng(17)
    for attr in ("sigma_t", "sigma_s"):
        gg = g64[attr]
        cand = np.nonzero(np.abs(gg) >= 1e-3 * np.max(np.abs(gg)))[0]
        cells = rng.choice(cand, min(20, cand.size), replace=False)
        worst32 = worst64 = 0.0
        for c in cells:
            h = 1e-4 * max(abs(getattr(P, attr)[c]), 1.0)
            fd = (J(attr, c, h) - J(attr, c, -h)) / (2 * h)
            e32 = abs(g32[attr][c] - fd) / abs(fd)
            e64 = abs(g64[attr][c] - fd) / abs(fd)
            worst32, worst64 = max(worst32, e32), max(worst64, e64)
            assert e32 <= 1e-4, (attr, c, g32[attr][c], fd)
            assert e64 <= 1e-6, (attr, c, g64[attr][c], fd)
        print(f"{attr}: {cells.size} cells, worst relative difference to FD: FP32 gradient "
              f"{worst32:.2e}, FP64 gradient {worst64:.2e}")
    S.close()


# ------------------------------------------------------------------ mixed precision, 200 steps

@pytest.fixture(scope="module")
def linesource_1024():
    """HG g=0.9 line source on 18 x 18 points (578 cells: two full 256-row product tiles and
    a ragged tail), 32 x 32 = 1024 ordinates, 200 steps; the oracle's final state."""
    from oracle import oracle as o
    P = I.build("linesource_hg_s32", n_side=18, nsteps=200)
    print(f"oracle: line source {P.ncells} x {P.nq}, 200 steps", flush=True)
    ref = o.rollout(o.OracleProblem.from_problem(P), P.psi0, P.dt, 200)[0]
    return P, ref


@pytest.mark.parametrize("precision,tol", [("bf16x3", 1e-4), ("bf16x2", 1e-3),
                                           ("fp16x3", 1e-4), ("fp32", 1e-5)])
def test_mixed_precision_1024_ordinates_200_steps(linesource_1024, precision, tol):
    """Error of the whole 200-step run at 1024 ordinates against the FP64 oracle: rel-L2 and
    max|err| / max|ref| within the product's bound (hi+lo BF16 at 1e-3, the three-product
    form expected near 1e-6)."""
    P, ref = linesource_1024
    S = _solver(P, precision=precision)
    psi, _ = S.rollout(S.initial_state(), 200)
    out = S.to_user(psi).cpu().numpy()
    S.close()
    err = rel_l2(out, ref)
    mx = float(np.max(np.abs(out - ref)) / np.max(np.abs(ref)))
    print(f"{precision} 1024 ordinates, 200 steps: rel-L2 {err:.2e}, max-abs/max-ref {mx:.2e}")
    assert err <= tol and mx <= tol


# ------------------------------------------------------------------ CSD dose gradient

@pytest.mark.parametrize("precision", ["bf16x3", "fp16x3", "fp32"])
def test_csd_reduced_dose_gradient_full_energy_range(precision):
    """The reduced CSD workload from 20 MeV to 0.1 MeV: GPU dose (FP64 accumulation) and
    the density gradient of J = sum_T A D - sum_O A D through the differentiable rollout
    (checkpoints every 20 steps, the mixed-precision product forward and transposed) against
    the oracle's reverse pass: dose rel-L2 <= 1e-4, gradient rel-L2 <= 1e-4 and element-wise
    within 1e-3 relative above a floor of 1e-4 max|g|."""
    import importlib.util
    import os
    from paper_2205_08417_amd.solver import differentiable_rollout
    here = os.path.dirname(os.path.abspath(__file__))
    spec = importlib.util.spec_from_file_location(
        "make_csd", os.path.join(here, "golden", "make_csd_reduced_gradient.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    P = gen.problem()
    ref = np.load(os.path.join(here, "golden", "csd_reduced_gradient.npz"))
    assert str(ref["digest"]) == gen.input_digest(P), "inputs differ from the stored run"
    n = P.nsteps
    print(f"CSD reduced: {P.ncells} x {P.nq}, {n} steps, {precision}", flush=True)
    S = _solver(P, precision=precision)
    psi0 = S.initial_state()
    r = S.cells_to_internal(P.rho).requires_grad_(True)
    psiN, dose = differentiable_rollout(S, psi0, n, rho=r, ckpt_every=20,
                                        inflow_scale=np.asarray(P.meta["inflow_scale"]),
                                        dose_coeff=np.asarray(P.meta["dose_coeff"]))
    w_d = S.cells_to_internal(gen.functional_weights(P), torch.float64)
    J = torch.sum(w_d * dose)
    J.backward()
    d = _cells_user(S, dose.detach())
    g = _cells_user(S, r.grad)
    S.close()
    e_d, e_g = rel_l2(d, ref["dose"]), rel_l2(g, ref["g_rho"])
    print(f"{precision}: dose rel-L2 {e_d:.2e}, density gradient rel-L2 {e_g:.2e}")
    assert e_d <= 1e-4 and e_g <= 1e-4
    check_elementwise(f"{precision} density gradient", g, ref["g_rho"], 1e-3, 1e-4)
