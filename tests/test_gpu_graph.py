"""GPU tests of the step and the transposed step under HIP graph capture.

The explicit step and its transpose are captured once into a graph (isotropic scattering:
k_step and k_adjoint_p; dense BF16 hi+lo scattering on 256 ordinates: the one-launch
k_gemm_step and k_gemm_adjoint with the fold of the gradient pieces), together with fill
kernels that zero the gradient accumulators.  The graph is then replayed several times, with
eager library work on the same buffers and workspace between the replays; every replay must
equal the eager result bit for bit.  Nothing on these paths may record a memset or
allocate while captured.
"""
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


@pytest.mark.parametrize("dense", [False, True])
def test_step_and_transposed_step_replays_equal_eager(dense):
    from paper_2205_08417_amd.solver import Solver
    omega, w = I.product_quadrature(16, 16)
    K = I.henyey_greenstein_kernel(omega, w, 0.85) if dense else None
    P = small_problem(I.jittered_delaunay_mesh(40, 0.0, 1.0, seed=5), omega_w=(omega, w), K=K,
                      seed=5, rho=True, source=True, inflow=True, scatter=(0.5, 2.0))
    S = Solver(P, precision="bf16x3" if dense else "fp32")
    print(f"graph replay, {'dense bf16x3' if dense else 'isotropic'}: {S.nc} cells x "
          f"{S.nq} ordinates", flush=True)
    args = S.args(alpha_t=1.1, alpha_s=0.9, inflow_scale=0.6)
    psi = S.initial_state()
    lam = S.to_internal(np.random.default_rng(3).standard_normal((P.ncells, S.nq)))
    out = torch.empty_like(psi)
    lam_out = torch.empty_like(lam)
    g = [torch.zeros(S.nc, dtype=torch.float32, device="cuda") for _ in range(3)]

    def work():
        for x in g:
            x.fill_(0.0)                      # a fill kernel, not a memset node
        S.step(psi, out, args)
        S.adjoint_step(psi, lam, lam_out, g[0], g[1], g[2], args=args)

    work()
    torch.cuda.synchronize()
    ref = [out.clone(), lam_out.clone()] + [x.clone() for x in g]
    assert all(torch.isfinite(x).all() for x in ref)
    assert float(ref[2].abs().max()) > 0.0     # the gradients are not trivially zero

    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        work()
    torch.cuda.synchronize()
    scratch = torch.empty_like(psi)
    for rep in range(3):
        # eager work between replays: other values in every output, and the library using
        # the same workspace for a step of another state
        out.fill_(float(rep) - 5.0)
        lam_out.fill_(float(rep) + 5.0)
        for x in g:
            x.fill_(7.0)
        S.step(lam.abs(), scratch, args)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = [out, lam_out] + g
        for name, a, b in zip(("psi_out", "lam_n", "g_sigma_t", "g_sigma_s", "g_rho"), got, ref):
            assert torch.equal(a, b), f"replay {rep}: {name} differs from the eager result"
    del graph
    S.close()
