"""GPU tests of the one-launch dense step: the low-precision scattering product whose tiles
run the transport update (Sec. 4.2 explicit step, eq. SNEqns / SNEqns2) on the cells and
ordinates they hold, instead of writing S for a second kernel; with the dose of the input
state (Sec. 2) fused as well for snrt_step_dose.

snrt_step and snrt_step_dose take this path for triangles with nq % 256 == 0 and a BF16 /
FP16 product.  A child process with SNRT_STEP_FUSED=0 (read once per process) computes the
same steps with two launches (the product, then the step kernel); the states must agree
bit for bit, the doses to FP64 rounding, and both with the FP64 oracle to the product's
precision.  The launch shapes cover full 256 x 256 tiles with a ragged last row tile, the
last-round 64 x 128 and 64 x 256 tiles of larger meshes, a single cell, 256 / 512 / 1024
ordinates, densities, sources, Dirichlet inflow, Neumann and vacuum boundaries, and the
moment form (moments, then the fused second product).
"""
import os
import subprocess
import sys
import tempfile

import numpy as np
import pytest

from _util import rel_l2, small_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2205_08417_amd import inputs as I  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# one-step error bounds against the FP64 oracle from a uniform random state
TOL = {"bf16x3": 1e-5, "bf16x2": 1e-3, "bf16x1": 1e-2, "fp16x3": 1e-5}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2205_08417_amd import snrt
    snrt.lib()


def _plan(M, nq):
    """The product's block plan for M rows and nq columns (the library's policy): the rows of
    the 256-row tiles and the width of the last-round tiles (0: none)."""
    cu = torch.cuda.get_device_properties(0).multi_processor_count
    tiles = -(-M // 256) * (nq // 256)
    rem = tiles % cu
    level = tiles > cu and rem != 0 and cu % 8 == 0
    eighth = level and rem * 8 <= cu
    quarter = not eighth and level and rem * 4 <= cu
    rows1 = min(((tiles - rem) // (nq // 256)) * 256, M)
    if eighth:
        return rows1, 128
    if quarter:
        return rows1, 256
    return M, 0


def _case(name, seed):
    """(problem, solver kwargs, boundary) for a named case."""
    if name == "single-cell":
        pts = np.array([[0.0, 0.0], [1.0, 0.1], [0.2, 0.9]])
        mesh = I._faces_from_triangles(pts, np.array([[0, 1, 2]]), np.array([[-1, -1, -1]]))
        npol, naz, rho, src, inflow, bc = 16, 16, True, True, True, "dirichlet"
    else:
        n, npol, naz, rho, src, inflow, bc = {
            "256-ragged": (40, 16, 16, True, True, True, "dirichlet"),
            "512-neumann": (20, 16, 32, False, True, False, "neumann"),
            "1024-vacuum": (14, 32, 32, True, False, False, "vacuum"),
            "256-eighth": (183, 16, 16, False, True, True, "dirichlet"),
            "256-quarter": (196, 16, 16, True, False, True, "dirichlet"),
            "moments-256": (30, 16, 16, True, True, True, "dirichlet"),
            "moments-512": (16, 16, 32, False, False, False, "neumann"),
        }[name]
        mesh = I.jittered_delaunay_mesh(n, 0.0, 1.0, seed=seed)
    omega, w = I.product_quadrature(npol, naz)
    kw = {}
    K = None
    if name.startswith("moments"):
        kw["moments"] = I.hg_legendre_moments(0.8, 5)
    else:
        K = I.henyey_greenstein_kernel(omega, w, 0.85)
    P = small_problem(mesh, omega_w=(omega, w), K=K, seed=seed, rho=rho, source=src,
                      inflow=inflow, scatter=(0.5, 2.0))
    return P, kw, bc


def _oracle_problem(P, kw, neumann):
    from oracle import moments as mo
    from oracle import oracle as o
    if "moments" in kw:
        return o.OracleProblem.from_problem(
            P, K=mo.moment_kernel(P.omega, P.w, kw["moments"]), neumann=neumann)
    return o.OracleProblem.from_problem(P, neumann=neumann)


CASES = ["single-cell", "256-ragged", "512-neumann", "1024-vacuum", "256-eighth",
         "256-quarter", "moments-256", "moments-512"]
PRECISIONS = ["bf16x3", "bf16x2", "bf16x1", "fp16x3"]


def _skip(name, precision):
    return name in ("256-eighth", "256-quarter") and precision not in ("bf16x3", "fp16x3")


def _one_step(name, precision):
    """The step and the dose of every cell (user order) through snrt_step and snrt_step_dose,
    in whichever form this process runs the dense step."""
    from paper_2205_08417_amd import snrt
    from paper_2205_08417_amd.solver import Solver
    P, kw, bc = _case(name, 17)
    boundary = snrt.SNRT_BC_NEUMANN if bc == "neumann" else snrt.SNRT_BC_DIRICHLET
    S = Solver(P, precision=precision, **kw)
    args = S.args(alpha_t=1.1, alpha_s=0.9, inflow_scale=0.6, boundary=boundary)
    psi = S.initial_state()
    out = torch.empty_like(psi)
    out_d = torch.empty_like(psi)
    dose = torch.full((S.nc,), 0.25, dtype=torch.float64, device="cuda")
    snrt.snrt_step(S.mesh, S.quad, S.scatter, args, psi, out, S.ws, S.ws_bytes)
    snrt.snrt_step_dose(S.mesh, S.quad, S.scatter, args, psi, out_d, 0.37, dose, S.ws,
                        S.ws_bytes)
    torch.cuda.synchronize()
    res = (S.to_user(out).cpu().numpy(), S.to_user(out_d).cpu().numpy(),
           S.to_user(dose.reshape(-1, 1)).cpu().numpy().ravel(), S.perm.copy(), S.nc, S.nq)
    S.close()
    return P, kw, bc, res


def _one_adjoint(name, precision):
    """One transposed step (snrt_step_adjoint) from a seeded adjoint state, with the three
    per-cell gradients accumulated onto nonzero values, in whichever form this process runs
    it: lam_n and the gradients in user order."""
    from paper_2205_08417_amd import snrt
    from paper_2205_08417_amd.solver import Solver
    P, kw, bc = _case(name, 17)
    boundary = snrt.SNRT_BC_NEUMANN if bc == "neumann" else snrt.SNRT_BC_DIRICHLET
    S = Solver(P, precision=precision, **kw)
    lam = np.random.default_rng(29).standard_normal((P.ncells, S.nq))
    # small starting values: the FP32 rounding of g0 + increment stays far below the
    # increments (1e-2 to 1 here)
    g0 = 1e-3 * np.random.default_rng(30).standard_normal((3, P.ncells))
    psi = S.initial_state()
    l1 = S.to_internal(lam)
    l0 = torch.empty_like(l1)
    g = [S.cells_to_internal(g0[i]).contiguous() for i in range(3)]
    S.adjoint_step(psi, l1, l0, g[0], g[1], g[2] if P.rho is not None else None,
                   alpha_t=1.2, alpha_s=0.8, boundary=boundary)
    torch.cuda.synchronize()
    res = (S.to_user(l0).cpu().numpy(),
           np.stack([S.to_user(x.reshape(-1, 1)).cpu().numpy().ravel() for x in g]))
    S.close()
    return P, kw, bc, lam, g0, res


@pytest.fixture(scope="module")
def two_launch():
    """Every case's step and dose from a child process that runs the two launches."""
    script = (
        "import sys, numpy as np\n"
        f"sys.path.insert(0, {ROOT!r}); sys.path.insert(0, {os.path.join(ROOT, 'tests')!r})\n"
        "import test_gpu_step_fused as T\n"
        "out = sys.argv[1]\n"
        "for name in T.CASES:\n"
        "    for prec in T.PRECISIONS:\n"
        "        if T._skip(name, prec):\n"
        "            continue\n"
        "        print(f'two-launch {name} {prec}', flush=True)\n"
        "        _, _, _, r = T._one_step(name, prec)\n"
        "        np.save(f'{out}/{name}-{prec}-step.npy', r[0])\n"
        "        np.save(f'{out}/{name}-{prec}-dose-step.npy', r[1])\n"
        "        np.save(f'{out}/{name}-{prec}-dose.npy', r[2])\n"
        "        _, _, _, _, _, a = T._one_adjoint(name, prec)\n"
        "        np.save(f'{out}/{name}-{prec}-adj.npy', a[0])\n"
        "        np.save(f'{out}/{name}-{prec}-adj-grad.npy', a[1])\n")
    env = dict(os.environ, SNRT_STEP_FUSED="0")
    with tempfile.TemporaryDirectory() as tmp:
        print("child: two-launch steps of every case", flush=True)
        r = subprocess.run([sys.executable, "-c", script, tmp], env=env, capture_output=True,
                           text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-3000:]
        yield tmp


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("name", CASES)
def test_fused_step_equals_two_launch_step_and_oracle(two_launch, name, precision):
    from oracle import oracle as o
    if _skip(name, precision):
        pytest.skip("the last-round tile shapes are covered by two precisions")
    P, kw, bc, (out, out_d, dose, perm, nc, nq) = _one_step(name, precision)
    rows1, tail = _plan(nc, nq)
    print(f"{name} {precision}: {nc} cells x {nq} ordinates, 256-row tiles up to row "
          f"{rows1}, last-round tiles {'64x%d' % tail if tail else 'none'}", flush=True)
    if name == "256-eighth":
        assert tail == 128
    if name == "256-quarter":
        assert tail == 256
    ref = np.load(os.path.join(two_launch, f"{name}-{precision}-step.npy"))
    ref_d = np.load(os.path.join(two_launch, f"{name}-{precision}-dose-step.npy"))
    ref_dose = np.load(os.path.join(two_launch, f"{name}-{precision}-dose.npy"))
    for got, want, what in ((out, ref, "snrt_step"), (out_d, ref_d, "snrt_step_dose")):
        if not np.array_equal(got, want):
            bad = np.argwhere(got != want)
            print(f"  {what}: {bad.shape[0]} elements differ, max "
                  f"{np.abs(got - want).max():.3e}; first {bad[:6].tolist()}", flush=True)
        assert np.array_equal(got, want), f"{what}: one launch must equal two launches"
    assert np.array_equal(out, out_d)
    derr = float(np.max(np.abs(dose - ref_dose)) / np.max(np.abs(ref_dose)))
    print(f"  dose vs two-launch dose: {derr:.2e}")
    assert derr <= 1e-14
    # the oracle on sampled cells: every row of a small mesh, else cells of the full tiles
    # and of the last-round tiles (internal order: the last rows)
    if nc <= 4000:
        cells = np.arange(nc)
    else:
        rng = np.random.default_rng(3)
        inner = perm[rng.choice(min(rows1, nc), 80, replace=False)]
        last = perm[rows1 + rng.choice(nc - rows1, 80, replace=False)] if rows1 < nc \
            else perm[-80:]
        cells = np.unique(np.concatenate([inner, last, perm[-1:]]))
    op = _oracle_problem(P, kw, bc == "neumann")
    want = o.step(op, P.psi0, P.dt, 1.1, 0.9, 0.6, cells=cells)
    err = rel_l2(out[cells], want)
    worst = float(np.max(np.abs(out[cells] - want)) / np.max(np.abs(want)))
    print(f"  vs oracle on {cells.size} cells: rel-L2 {err:.2e}, max {worst:.2e}")
    assert err <= TOL[precision]
    assert worst <= 10 * TOL[precision]
    # the dose of the input state against the oracle's (FP32 copies of psi and 1/rho, as on
    # the device)
    op32 = _oracle_problem(P, kw, bc == "neumann")
    if P.rho is not None:
        op32 = op32.replace(rho=1.0 / (1.0 / P.rho).astype(np.float32).astype(np.float64))
    psi32 = P.psi0.astype(np.float32).astype(np.float64)
    dref = o.dose_accumulate(op32, psi32, 0.37, np.full(nc, 0.25))
    dose_err = rel_l2(dose, dref)
    print(f"  dose vs oracle: {dose_err:.2e}")
    assert dose_err <= 1e-12


@pytest.mark.parametrize("precision", PRECISIONS)
@pytest.mark.parametrize("name", CASES)
def test_fused_adjoint_equals_two_launch_adjoint_and_oracle(two_launch, name, precision):
    """The transposed step in one launch (G = Lambda B^T formed tile by tile, the adjoint
    update on the tile's cells, per-piece gradient sums folded by a second small kernel):
    lam_n bit for bit against the two launches; the gradients to FP32 rounding of their
    sums (128-ordinate pieces here, whole rows there); both against the oracle's transposed
    step to the product's precision."""
    from oracle import oracle as o
    if _skip(name, precision):
        pytest.skip("the last-round tile shapes are covered by two precisions")
    P, kw, bc, lam, g0, (out, grad) = _one_adjoint(name, precision)
    nc = P.ncells
    ref = np.load(os.path.join(two_launch, f"{name}-{precision}-adj.npy"))
    ref_g = np.load(os.path.join(two_launch, f"{name}-{precision}-adj-grad.npy"))
    if not np.array_equal(out, ref):
        bad = np.argwhere(out != ref)
        print(f"  lam_n: {bad.shape[0]} elements differ, max {np.abs(out - ref).max():.3e}; "
              f"first {bad[:6].tolist()}", flush=True)
    assert np.array_equal(out, ref), "one launch must equal two launches"
    nr = 3 if P.rho is not None else 2
    for i, what in enumerate(("sigma_t", "sigma_s", "rho")[:nr]):
        d = grad[i] - g0[i]
        dr = ref_g[i] - g0[i]
        err = float(np.max(np.abs(d - dr)) / np.max(np.abs(dr)))
        print(f"  {name} {precision} g_{what} increment vs two-launch: {err:.2e}")
        assert err <= 1e-5, what
    if P.rho is None:
        assert np.array_equal(grad[2], g0[2].astype(np.float32))   # untouched
    # the oracle's transposed step (FP64) on the same inputs
    op = _oracle_problem(P, kw, bc == "neumann")
    gt, gs = np.zeros(nc), np.zeros(nc)
    gr = np.zeros(nc) if P.rho is not None else None
    want = o.adjoint_step(op, P.psi0, lam, P.dt, 1.2, 0.8, gt, gs, gr)
    err = rel_l2(out, want)
    print(f"  lam_n vs oracle: rel-L2 {err:.2e}")
    assert err <= TOL[precision]
    # g_sigma_t and g_rho hold no product term (FP32 sums of lam psi and psi times the
    # downwind sum); g_sigma_s sums psi G over the row, which cancels for an adjoint state of
    # random sign, so its relative error exceeds the product's by up to an order of magnitude
    for i, ref_i in enumerate((gt, gs, gr)[:nr]):
        e = rel_l2(grad[i] - g0[i], ref_i)
        bar = 10 * TOL[precision] if i == 1 else 1e-5
        print(f"  gradient {i} vs oracle: rel-L2 {e:.2e} (bar {bar:.0e})")
        assert e <= bar


def test_fused_rollout_equals_two_launch_rollout_in_a_fresh_process():
    """SNRT_STEP_FUSED=0 (read once per process): the same 6-step rollouts with the product
    and the step kernel as two launches, dense BF16x3 on 512 ordinates and the moment form
    on 256, bit for bit against the one-launch rollouts here."""
    script = (
        "import sys, numpy as np, torch\n"
        f"sys.path.insert(0, {ROOT!r}); sys.path.insert(0, {os.path.join(ROOT, 'tests')!r})\n"
        "import test_gpu_step_fused as T\n"
        "from paper_2205_08417_amd.solver import Solver\n"
        "name, out = sys.argv[1], sys.argv[2]\n"
        "P, kw, bc = T._case(name, 23)\n"
        "S = Solver(P, precision='bf16x3', **kw)\n"
        "psi, _ = S.rollout(S.initial_state(), 6)\n"
        "np.save(out, S.to_user(psi).cpu().numpy())\n")
    from paper_2205_08417_amd.solver import Solver
    env = dict(os.environ, SNRT_STEP_FUSED="0")
    for name in ("512-neumann", "moments-256"):
        with tempfile.TemporaryDirectory() as tmp:
            path = os.path.join(tmp, "psi.npy")
            print(f"child: two-launch rollout, {name}", flush=True)
            r = subprocess.run([sys.executable, "-c", script, name, path], env=env,
                               capture_output=True, text=True, timeout=300)
            assert r.returncode == 0, r.stderr[-2000:]
            sep = np.load(path)
        P, kw, bc = _case(name, 23)
        S = Solver(P, precision="bf16x3", **kw)
        psi, _ = S.rollout(S.initial_state(), 6)
        got = S.to_user(psi).cpu().numpy()
        S.close()
        print(f"{name}: max |fused - two-launch| = {np.abs(got - sep).max():.3e}")
        assert np.array_equal(got, sep)


def _dose_gradient(config):
    """Density gradient of a target-minus-organ dose functional through the reverse rollout,
    whose transposed steps carry the dose functional's term (fused unless SNRT_STEP_FUSED=0)."""
    from paper_2205_08417_amd.solver import Solver, differentiable_rollout
    npol, naz, precision = {"dense-64": (4, 16, "fp32"), "dense-256": (16, 16, "bf16x3")}[config]
    P = I.build("csd_phantom_s512", n_side=14, n_polar=npol, n_azimuth=naz, nsteps=24,
                rho_air=0.3)
    n = P.nsteps
    at = np.linspace(1.0, 1.3, n)
    T = I.region_mask(P.mesh, (3.0, 7.0, 7.0, 10.0))
    O = I.region_mask(P.mesh, (0.0, 3.5, 5.0, 10.0))
    dJdD = P.mesh.area * (T.astype(float) - O.astype(float))
    S = Solver(P, precision=precision)
    r = S.cells_to_internal(P.rho).requires_grad_(True)
    psiN, dose = differentiable_rollout(S, S.initial_state(), n, rho=r, ckpt_every=8,
                                        alpha_t=at, alpha_s=at,
                                        inflow_scale=np.asarray(P.meta["inflow_scale"]),
                                        dose_coeff=np.asarray(P.meta["dose_coeff"]))
    J = torch.sum(S.cells_to_internal(dJdD, torch.float64) * dose)
    J.backward()
    return r.grad.detach().cpu().numpy(), dose.detach().cpu().numpy()


def test_reverse_rollout_dose_term_equals_separate_pass_in_a_fresh_process():
    """The reverse rollout adds the dose functional's term to the transposed step's output
    rows; a child process with SNRT_STEP_FUSED=0 adds it in a pass of its own (and runs the
    forward dense steps in two launches).  The density gradients agree bit for bit; the doses
    to FP64 rounding (the one-launch step sums them over 128-ordinate pieces, the two-launch
    step over 256-ordinate chunks).  With BF16 products the transposed steps run in one
    launch as well, whose gradient sums over 128-ordinate pieces round differently from the
    whole-row sums: there the gradients agree to 1e-6 of their largest entry."""
    script = (
        "import sys, numpy as np\n"
        f"sys.path.insert(0, {ROOT!r}); sys.path.insert(0, {os.path.join(ROOT, 'tests')!r})\n"
        "import test_gpu_step_fused as T\n"
        "g, d = T._dose_gradient(sys.argv[1])\n"
        "np.save(sys.argv[2], g); np.save(sys.argv[3], d)\n")
    env = dict(os.environ, SNRT_STEP_FUSED="0")
    for config in ("dense-64", "dense-256"):
        with tempfile.TemporaryDirectory() as tmp:
            pg, pd = os.path.join(tmp, "g.npy"), os.path.join(tmp, "d.npy")
            print(f"child: separate dose-term pass, {config}", flush=True)
            r = subprocess.run([sys.executable, "-c", script, config, pg, pd], env=env,
                               capture_output=True, text=True, timeout=300)
            assert r.returncode == 0, r.stderr[-2000:]
            g_ref, d_ref = np.load(pg), np.load(pd)
        g, d = _dose_gradient(config)
        print(f"{config}: max |grad - separate| = {np.abs(g - g_ref).max():.3e}")
        assert np.abs(d - d_ref).max() <= 1e-14 * np.abs(d_ref).max()
        if config == "dense-64":
            assert np.array_equal(g, g_ref)
        else:
            assert np.abs(g - g_ref).max() <= 1e-6 * np.abs(g_ref).max()
