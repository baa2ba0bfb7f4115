"""GPU parity of dense (anisotropic) scattering: FP32 product, BF16 hi+lo (three MFMA
products) and BF16 single product, against the FP64 oracle.

Tolerances: the FP32 product follows the FP32 step (1e-5 rel-L2 over the run); BF16x3 keeps
about 16 significant bits per operand, so 1e-3 is the bound and ~1e-5 the expectation; the
single BF16 product keeps 8 bits and is held to 1e-2.
"""
import dataclasses

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


def _run(P, nsteps, precision):
    from paper_2205_08417_amd.solver import Solver
    S = Solver(P, precision=precision)
    psi, _ = S.rollout(S.initial_state(), nsteps)
    out = S.to_user(psi).cpu().numpy()
    S.close()
    return out


def _oracle(P, nsteps):
    from oracle import oracle as o
    return o.rollout(o.OracleProblem.from_problem(P), P.psi0, P.dt, nsteps)[0]


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("bf16x3", 1e-3), ("bf16x2", 1e-3),
                                           ("bf16x1", 1e-2), ("fp16x3", 1e-4)])
def test_hg_linesource_256_ordinates(precision, tol):
    """HG g=0.9 line source, 30x30 points (1 682 cells, two ragged 128-cell tiles), 16x16
    ordinates, 40 steps."""
    P = I.build("linesource_hg_s32", n_side=30, n_polar=16, n_azimuth=16, nsteps=40)
    ref = _oracle(P, 40)
    err = rel_l2(_run(P, 40, precision), ref)
    print(f"dense {precision}: rel-L2 after 40 steps = {err:.3e}")
    assert err <= tol


@pytest.mark.parametrize("precision,tol", [("bf16x3", 1e-5), ("bf16x2", 1e-4), ("fp16x3", 1e-6)])
def test_bf16_512_ordinates_rough_state(precision, tol):
    """16x32 = 512 ordinates (two N tiles), a state spanning 6 decades, one step."""
    P = I.build("csd_phantom_s512", n_side=14, nsteps=1)
    P = dataclasses.replace(P, psi0=I.random_state(P.ncells, P.nq, seed=5))
    ref = _oracle(P, 1)
    err = rel_l2(_run(P, 1, precision), ref)
    print(f"{precision} 512 ordinates one step: {err:.3e}")
    assert err <= tol


@pytest.mark.parametrize("precision", ["bf16x3", "bf16x2", "fp16x3"])
def test_bf16_full_size_linesource_sampled(precision):
    """Full HG line source (100 352 cells x 1024 ordinates) in the benchmark's launch shape:
    one step from the seeded pulse, sampled cells checked one by one."""
    from oracle import oracle as o
    P = I.build("linesource_hg_s32")
    out = _run(P, 1, precision)
    rng = np.random.default_rng(1)
    r2 = np.sum(P.mesh.centroid ** 2, axis=1)
    hot = np.nonzero(r2 < 0.01)[0]
    cells = np.unique(np.concatenate([hot[:100], rng.choice(P.ncells, 100, False)]))
    ref = o.step(o.OracleProblem.from_problem(P), P.psi0, P.dt, cells=cells)
    err = rel_l2(out[cells], ref)
    print(f"{precision} full-size sampled: {err:.3e}")
    assert err <= 1e-4


def test_bf16x3_full_size_csd_sampled():
    """Full CSD phantom (299 538 cells x 512 ordinates, HG g=0.95, densities 1.85 / 1 /
    0.001, beam inflow scaled by S(E) G_E) in the benchmark's launch shape: the dose
    accumulated from a rough state, then one step; sampled cells checked one by one (beam
    faces, the air cavity and random cells), the dose everywhere."""
    from oracle import oracle as o
    from paper_2205_08417_amd.solver import Solver
    P = I.build("csd_phantom_s512")
    P = dataclasses.replace(P, psi0=I.random_state(P.ncells, P.nq, seed=11, decades=4))
    isc, c0 = float(P.meta["inflow_scale"][0]), float(P.meta["dose_coeff"][0])
    S = Solver(P, precision="bf16x3")
    psi, dose = S.rollout(S.initial_state(), 1, inflow_scale=[isc], dose_coeff=[c0])
    out = S.to_user(psi).cpu().numpy()
    dose = S.to_user(dose.reshape(S.nc, 1)).cpu().numpy().ravel()
    S.close()
    rng = np.random.default_rng(2)
    beam = np.unique(P.mesh.bface_cell[np.abs(P.mesh.bface_mid[:, 1] - 10.0) < 1e-12])
    c = P.mesh.centroid
    air = np.nonzero((c[:, 0] - 4.0) ** 2 + (c[:, 1] - 7.0) ** 2 <= 0.75 ** 2)[0]
    cells = np.unique(np.concatenate([beam[:80], air[:40], rng.choice(P.ncells, 120, False)]))
    op = o.OracleProblem.from_problem(P)
    ref = o.step(op, P.psi0, P.dt, inflow_scale=isc, cells=cells)
    err = rel_l2(out[cells], ref)
    print(f"bf16x3 full-size CSD sampled: {err:.3e}")
    assert err <= 1e-4
    # the GPU sums the FP32 state it holds in FP64 and scales by the FP32 copy of 1/rho
    # (relative rounding <= 6e-8)
    psi32 = P.psi0.astype(np.float32).astype(np.float64)
    dref = o.dose_accumulate(op, psi32, c0, np.zeros(P.ncells))
    derr = rel_l2(dose, dref)
    print(f"dose rel-L2: {derr:.3e}")
    assert derr <= 1e-6


@pytest.mark.parametrize("precision", ["bf16x3", "fp16x3"])
def test_low_precision_requires_32_multiple(precision):
    """The product runs K in chunks of 32: 6 x 8 = 48 ordinates are refused."""
    from paper_2205_08417_amd import snrt
    from paper_2205_08417_amd.solver import _PREC
    omega, w = I.product_quadrature(6, 8)
    K = I.henyey_greenstein_kernel(omega, w, 0.5)
    q = snrt.snrt_quad_create(omega, w)
    with pytest.raises(snrt.SnrtError) as ei:
        snrt.snrt_scatter_dense(q, K, _PREC[precision])
    assert ei.value.status == snrt.SNRT_E_UNSUPPORTED
    snrt.snrt_quad_destroy(q)


@pytest.mark.parametrize("precision,tol", [("bf16x3", 2e-5), ("bf16x2", 2e-3), ("bf16x1", 1e-2),
                                           ("fp16x3", 1e-6)])
def test_bf16_product_with_partial_last_round(precision, tol):
    """71 442 cells x 256 ordinates: 280 row tiles of 256 over the compute units leave a
    partial last round, whose rows the library runs as 64-row blocks (ragged at the end).
    Every row of the product S = Psi B is checked against FP64, the tail rows on their own."""
    from paper_2205_08417_amd import snrt
    from paper_2205_08417_amd.solver import Solver
    mesh = I.jittered_delaunay_mesh(190, -1.5, 1.5, seed=61)
    omega, w = I.product_quadrature(16, 16)
    K = I.henyey_greenstein_kernel(omega, w, 0.8)
    rng = np.random.default_rng(62)
    psi = rng.uniform(0.1, 1.0, (mesh.ncells, 256))
    P = I.Problem(name="product", mesh=mesh, omega=omega, w=w, K=K,
                  sigma_t=np.ones(mesh.ncells), sigma_s=np.ones(mesh.ncells), rho=None,
                  source=None, inflow=None, psi0=psi, dt=1e-3, nsteps=1)
    S = Solver(P, precision=precision)
    x = S.to_internal(psi)
    out = torch.empty_like(x)
    snrt.snrt_scatter_apply(S.mesh, S.quad, S.scatter, x, out, 0, S.ws, S.ws_bytes)
    got = out.cpu().numpy().astype(np.float64)
    ref = x.cpu().numpy().astype(np.float64) @ (w[:, None] * K.T)
    S.close()
    tail = 65536 if mesh.ncells > 65536 else 0
    err, err_tail = rel_l2(got, ref), rel_l2(got[tail:], ref[tail:])
    print(f"{precision}: all {err:.2e}, tail rows {err_tail:.2e}")
    assert err <= tol and err_tail <= tol


@pytest.mark.parametrize("npol,naz", [(8, 8), (4, 24), (5, 32)])
@pytest.mark.parametrize("precision,tol", [("bf16x3", 1e-5), ("bf16x2", 2e-4), ("fp16x3", 1e-6)])
def test_low_precision_products_on_padded_widths(npol, naz, precision, tol):
    """Ordinate counts that are multiples of 32 but not of 128 (64, 96, 160): the product's
    operand is zero-padded to the next 128 columns and only nq are written.  One step from a
    state spanning 6 decades (the FP16 mode's per-row scaling), every element against the
    oracle, on 17 x 17 points (512 cells: two full 256-row tiles)."""
    from _util import small_problem
    omega, w = I.product_quadrature(npol, naz)
    K = I.henyey_greenstein_kernel(omega, w, 0.9)
    P = small_problem(I.jittered_delaunay_mesh(17, 0.0, 1.0, seed=81), omega_w=(omega, w), K=K,
                      rho=True, seed=81, scatter=(0.5, 1.0), nsteps=1)
    P = dataclasses.replace(P, psi0=I.random_state(P.ncells, P.nq, seed=82))
    ref = _oracle(P, 1)
    got = _run(P, 1, precision)
    err = rel_l2(got, ref)
    worst = float(np.max(np.abs(got - ref) / (np.abs(ref) + 1e-30)))
    print(f"{precision} nq={P.nq}: rel-L2 {err:.2e}, worst element relative {worst:.2e}")
    assert err <= tol
