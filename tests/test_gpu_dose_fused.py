"""GPU tests of snrt_step_dose: the step with the dose of its input fused (Sec. 2 pseudo-time
dose, left endpoint), against snrt_dose_accumulate followed by snrt_step and against the
oracle's dose.

The state it writes must be bitwise the plain step's; the dose is formed per 256-ordinate
row chunk of the dense step in FP64 and differs from the one-pass sum only by FP64
rounding.  Cases: isotropic (whole rows), FP32 dense rows of 48 ordinates (a ragged lane
slice), BF16 dense rows of 256, 512 and 1024 ordinates (1, 2 and 4 chunks per row), the
moment form, densities, triangle and quadrilateral meshes.
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


def _problem(kind, seed):
    mesh = (I.quad_grid_mesh(13, 11) if kind.endswith("quad")
            else I.jittered_delaunay_mesh(12, 0.0, 1.0, seed=seed))
    if kind.startswith("iso"):
        return small_problem(mesh, 4, 16, seed=seed, rho=True, source=True, inflow=True), {}
    if kind == "fp32-48":
        omega, w = I.product_quadrature(4, 12)
        K = I.henyey_greenstein_kernel(omega, w, 0.6)
        return small_problem(mesh, omega_w=(omega, w), K=K, seed=seed, rho=True,
                             inflow=True), {"precision": "fp32"}
    if kind == "moments":
        omega, w = I.product_quadrature(16, 32)
        P = small_problem(mesh, omega_w=(omega, w), seed=seed, rho=True, inflow=True)
        return P, {"precision": "bf16x3", "moments": I.hg_legendre_moments(0.8, 6)}
    npol, naz = {"bf16-256": (16, 16), "bf16-512": (16, 32), "bf16-1024": (32, 32)}[kind]
    omega, w = I.product_quadrature(npol, naz)
    K = I.henyey_greenstein_kernel(omega, w, 0.8)
    return small_problem(mesh, omega_w=(omega, w), K=K, seed=seed, rho=True,
                         inflow=True), {"precision": "bf16x3"}


@pytest.mark.parametrize("kind", ["iso", "iso-quad", "fp32-48", "bf16-256", "bf16-512",
                                  "bf16-1024", "moments"])
def test_fused_dose_equals_separate_passes(kind):
    from oracle import oracle as o
    from paper_2205_08417_amd import snrt
    from paper_2205_08417_amd.solver import Solver
    P, kw = _problem(kind, 40)
    S = Solver(P, **kw)
    psi = S.initial_state()
    args = S.args(inflow_scale=0.7)
    out_ref = torch.empty_like(psi)
    out = torch.empty_like(psi)
    dose_ref = torch.full((S.nc,), 0.25, dtype=torch.float64, device="cuda")
    dose = dose_ref.clone()
    snrt.snrt_dose_accumulate(S.mesh, S.quad, psi, S.mats32["inv_rho"], 0.37, dose_ref)
    snrt.snrt_step(S.mesh, S.quad, S.scatter, args, psi, out_ref, S.ws, S.ws_bytes)
    snrt.snrt_step_dose(S.mesh, S.quad, S.scatter, args, psi, out, 0.37, dose, S.ws,
                        S.ws_bytes)
    torch.cuda.synchronize()
    assert torch.equal(out, out_ref), "the fused step must write the plain step's state"
    d, dr = dose.cpu().numpy(), dose_ref.cpu().numpy()
    assert np.abs(d - dr).max() <= 1e-14 * np.abs(dr).max()
    # and the oracle's dose of the FP32 state (FP32 copy of 1/rho, as on the device)
    op32 = o.OracleProblem.from_problem(P).replace(
        rho=1.0 / (1.0 / P.rho).astype(np.float32).astype(np.float64))
    psi32 = P.psi0.astype(np.float32).astype(np.float64)
    ref = o.dose_accumulate(op32, psi32, 0.37, np.full(P.ncells, 0.25))
    got = S.to_user(dose.reshape(-1, 1)).cpu().numpy().ravel()
    err = rel_l2(got, ref)
    print(f"fused dose {kind}: {err:.2e}")
    assert err <= 1e-12
    S.close()


def test_fused_dose_rollout_vs_oracle():
    """20 steps of a small CSD-like problem (densities, scaled inflow, per-step alpha and
    dose coefficients) through Solver.rollout, which takes the fused path."""
    from oracle import oracle as o
    from paper_2205_08417_amd.solver import Solver
    P, kw = _problem("bf16-512", 41)
    n = 20
    rng = np.random.default_rng(42)
    at = rng.uniform(0.8, 1.2, n)
    isc = rng.uniform(0.5, 1.0, n)
    coeff = rng.uniform(0.01, 0.1, n)
    S = Solver(P, precision="fp32")
    psi, dose = S.rollout(S.initial_state(), n, alpha_t=at, alpha_s=at, inflow_scale=isc,
                          dose_coeff=coeff)
    got_psi = S.to_user(psi).cpu().numpy()
    got = S.to_user(dose.reshape(-1, 1)).cpu().numpy().ravel()
    S.close()
    op = o.OracleProblem.from_problem(P)
    ref_psi, ref = P.psi0, np.zeros(P.ncells)
    for k in range(n):
        ref = o.dose_accumulate(op, ref_psi, coeff[k], ref)
        ref_psi = o.step(op, ref_psi, P.dt, alpha_t=at[k], alpha_s=at[k], inflow_scale=isc[k])
    e_psi, e_dose = rel_l2(got_psi, ref_psi), rel_l2(got, ref)
    print(f"fused dose rollout: psi {e_psi:.2e} dose {e_dose:.2e}")
    assert e_psi <= 1e-5
    assert e_dose <= 1e-5


def test_fused_dose_errors():
    from paper_2205_08417_amd import snrt
    from paper_2205_08417_amd.solver import Solver
    for kind in ("bf16-512", "iso"):
        P, kw = _problem(kind, 43)
        S = Solver(P, **kw)
        psi = S.initial_state()
        out = torch.empty_like(psi)
        dose = torch.zeros(S.nc, dtype=torch.float64, device="cuda")
        args = S.args()
        cases = [
            (dict(dose=None), snrt.SNRT_E_ARG),
            (dict(coeff=float("nan")), snrt.SNRT_E_NONFINITE),
            (dict(dose=S.ws), snrt.SNRT_E_ALIAS),
            (dict(dose=out), snrt.SNRT_E_ALIAS),
        ]
        if kind == "iso":
            # isotropic: the workspace holds exactly the per-cell sums
            assert S.ws_bytes == S.nc * 8
            cases.append((dict(ws_bytes=S.ws_bytes - 8), snrt.SNRT_E_ARG))
        for over, status in cases:
            kw2 = dict(dose=dose, coeff=1.0, ws_bytes=S.ws_bytes)
            kw2.update(over)
            with pytest.raises(snrt.SnrtError) as ei:
                snrt.snrt_step_dose(S.mesh, S.quad, S.scatter, args, psi, out, kw2["coeff"],
                                    kw2["dose"], S.ws, kw2["ws_bytes"])
            assert ei.value.status == status, (kind, over)
        if kind == "iso":
            # the plain isotropic step still needs no workspace
            snrt.snrt_step(S.mesh, S.quad, S.scatter, args, psi, out, None, 0)
            torch.cuda.synchronize()
        S.close()
