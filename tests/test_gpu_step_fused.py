"""GPU tests of the one-launch dense step: the low-precision scattering product whose tiles
run the transport update (Sec. 4.2 explicit step, eq. SNEqns / SNEqns2) on the cells and
ordinates they hold, instead of writing S for a second kernel.

snrt_step takes this path for triangles with nq % 256 == 0 and a BF16 / FP16 product;
snrt_step_dose keeps the two launches (product, then the step kernel with the dose), and
its state is the plain step's bit for bit.  So in one process the fused state can be held
against the two-launch state exactly, and against the FP64 oracle to the product's
precision.  The launch shapes cover full 256 x 256 tiles with a ragged last row tile, the
last-round 64 x 128 and 64 x 256 tiles of larger meshes, a single cell, 256 / 512 / 1024
ordinates, densities, sources, Dirichlet inflow, Neumann and vacuum boundaries, and the
moment form (moments, then the fused second product).  A child process with
SNRT_STEP_FUSED=0 runs the same rollout with the two launches throughout.
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


@pytest.mark.parametrize("precision", ["bf16x3", "bf16x2", "bf16x1", "fp16x3"])
@pytest.mark.parametrize("name", CASES)
def test_fused_step_equals_two_launch_step_and_oracle(name, precision):
    from oracle import oracle as o
    from paper_2205_08417_amd import snrt
    from paper_2205_08417_amd.solver import Solver
    if name in ("256-eighth", "256-quarter") and precision not in ("bf16x3", "fp16x3"):
        pytest.skip("the last-round tile shapes are covered by two precisions")
    P, kw, bc = _case(name, 17)
    boundary = {"dirichlet": snrt.SNRT_BC_DIRICHLET, "neumann": snrt.SNRT_BC_NEUMANN,
                "vacuum": snrt.SNRT_BC_DIRICHLET}[bc]
    if bc == "vacuum":
        assert P.inflow is None
    S = Solver(P, precision=precision, **kw)
    rows1, tail = _plan(S.nc, S.nq)
    print(f"{name} {precision}: {S.nc} cells x {S.nq} ordinates, 256-row tiles up to row "
          f"{rows1}, last-round tiles {'64x%d' % tail if tail else 'none'}", flush=True)
    if name == "256-eighth":
        assert tail == 128
    if name == "256-quarter":
        assert tail == 256
    args = S.args(alpha_t=1.1, alpha_s=0.9, inflow_scale=0.6, boundary=boundary)
    psi = S.initial_state()
    out = torch.empty_like(psi)
    ref = torch.empty_like(psi)
    dose = torch.zeros(S.nc, dtype=torch.float64, device="cuda")
    snrt.snrt_step(S.mesh, S.quad, S.scatter, args, psi, out, S.ws, S.ws_bytes)
    snrt.snrt_step_dose(S.mesh, S.quad, S.scatter, args, psi, ref, 1.0, dose, S.ws, S.ws_bytes)
    torch.cuda.synchronize()
    if not torch.equal(out, ref):
        diff = (out - ref).abs()
        bad = (diff > 0).nonzero()
        print(f"  differing elements {bad.shape[0]} of {out.numel()}, max |diff| "
              f"{float(diff.max()):.3e} (max |ref| {float(ref.abs().max()):.3e}); first "
              f"(row, col): {bad[:8].tolist()}", flush=True)
    assert torch.equal(out, ref), "the one-launch step must equal the two-launch step"
    # the oracle on sampled cells: every row of a small mesh, else cells of the full tiles
    # and of the last-round tiles (internal order: the last rows)
    got = S.to_user(out).cpu().numpy()
    if S.nc <= 4000:
        cells = np.arange(S.nc)
    else:
        rng = np.random.default_rng(3)
        inner = S.perm[rng.choice(min(rows1, S.nc), 80, replace=False)]
        last = S.perm[rows1 + rng.choice(S.nc - rows1, 80, replace=False)] if rows1 < S.nc \
            else S.perm[-80:]
        cells = np.unique(np.concatenate([inner, last, S.perm[-1:]]))
    op = _oracle_problem(P, kw, bc == "neumann")
    want = o.step(op, P.psi0, P.dt, 1.1, 0.9, 0.6, cells=cells)
    err = rel_l2(got[cells], want)
    worst = float(np.max(np.abs(got[cells] - want)) / np.max(np.abs(want)))
    print(f"  vs oracle on {cells.size} cells: rel-L2 {err:.2e}, max {worst:.2e}")
    assert err <= TOL[precision]
    assert worst <= 10 * TOL[precision]
    S.close()


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
