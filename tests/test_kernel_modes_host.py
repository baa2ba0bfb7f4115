"""Host-side eigendecomposition behind the implicit collision solve of a dense kernel
(IMEX step of Sec. 4.2 with the scattering operator of the S_N equations), run without a
device through snrt_kernel_modes: A = K W = V diag(lam) V^-1, checked against numpy's
dense linear algebra and against closed forms.  The device path uploads exactly these
operands, so a mistake here (a transposed operand, a lost sqrt(r) scaling, a wrong
eigenvector row) fails one of the products below."""
import numpy as np
import pytest

from paper_2205_08417_amd import inputs as I


def _lib():
    from paper_2205_08417_amd import snrt
    try:
        snrt.lib()
    except OSError as e:
        pytest.skip(str(e))
    return snrt


def _solve_modes(lam, x0, x1, a, b, r):
    """(a I - b A)^-1 r through the modes, as the step computes it per cell."""
    u = r @ x0
    u = u * (b / (a - b * lam))
    return (r + u @ x1) / a


@pytest.mark.parametrize("order,g,normalise", [(4, 0.0, True), (4, 0.6, True),
                                               (8, 0.9, True), (8, 0.8, False)])
def test_hg_kernel_modes(order, g, normalise):
    snrt = _lib()
    omega, w = I.product_quadrature(order, 2 * order)
    K = I.henyey_greenstein_kernel(omega, w, g, normalise=normalise)
    A = K * w[None, :]
    lam, x0, x1, resid = snrt.snrt_kernel_modes(A)
    n = A.shape[0]
    assert resid < 1e-12
    # A = V diag(lam) V^-1 with x0 = (V^-1)^T and x1 = diag(lam) V^T
    scale = np.abs(A).max()
    assert np.abs((x0 @ x1).T - A).max() < 1e-12 * scale * n
    # real spectrum equal to numpy's (non-symmetric routine: nothing assumed about A)
    ref = np.sort(np.linalg.eigvals(A).real)
    assert np.abs(np.sort(lam) - ref).max() < 1e-12 * scale * n
    # the per-cell solve against a dense solve, over a spread of a, b
    rng = np.random.default_rng(7)
    for a, b in ((1.0, 0.0), (1.3, 0.9), (2.0, 1.99), (1.0 + 1e-3, 50.0)):
        r = rng.standard_normal(n)
        got = _solve_modes(lam, x0, x1, a, b, r)
        want = np.linalg.solve(a * np.eye(n) - b * A, r)
        assert np.abs(got - want).max() <= 1e-11 * np.abs(want).max()


def test_normalised_kernel_conserves():
    """Normalised columns: w^T A = w^T, so 1 is an eigenvalue (the particle count) and no
    eigenvalue exceeds it in size (A is column-stochastic up to the weights)."""
    snrt = _lib()
    omega, w = I.product_quadrature(6, 12)
    K = I.henyey_greenstein_kernel(omega, w, 0.7)
    lam, *_ = snrt.snrt_kernel_modes(K * w[None, :])
    assert abs(lam.max() - 1.0) < 1e-13
    assert np.abs(lam).max() <= 1.0 + 1e-13


def test_isotropic_kernel_closed_form():
    """K = 1/(4 pi): A = 1 w^T / (4 pi) has rank one, eigenvalue sum(w)/(4 pi) = 1 once and
    0 otherwise, and the solve is the closed form (r + b <r>_w / (a - b)) / a."""
    snrt = _lib()
    omega, w = I.product_quadrature(4, 8)
    n = len(w)
    A = np.full((n, n), 1.0 / (4 * np.pi)) * w[None, :]
    lam, x0, x1, _ = snrt.snrt_kernel_modes(A)
    lam = np.sort(lam)
    assert abs(lam[-1] - w.sum() / (4 * np.pi)) < 1e-13
    assert np.abs(lam[:-1]).max() < 1e-13
    lam, x0, x1, _ = snrt.snrt_kernel_modes(A)
    r = np.random.default_rng(3).standard_normal(n)
    a, b = 1.4, 0.8
    mean = (w @ r) / (4 * np.pi)
    assert np.abs(_solve_modes(lam, x0, x1, a, b, r) - (r + b * mean / (a - b)) / a).max() < 1e-13


def test_symmetric_matrix_gives_orthogonal_modes():
    """With A symmetric the diagonal similarity is the identity: V^-1 = V^T, so x0 is
    orthogonal."""
    snrt = _lib()
    rng = np.random.default_rng(11)
    B = rng.standard_normal((40, 40))
    A = B + B.T
    lam, x0, x1, _ = snrt.snrt_kernel_modes(A)
    assert np.abs(x0.T @ x0 - np.eye(40)).max() < 1e-13
    assert np.abs(np.sort(lam) - np.linalg.eigvalsh(A)).max() < 1e-12 * np.abs(A).max() * 40


def test_block_diagonal_and_tiny():
    """Disconnected blocks (one diagonal root each) and the 1 x 1 and 2 x 2 cases."""
    snrt = _lib()
    rng = np.random.default_rng(5)
    d1 = rng.uniform(0.5, 2.0, 3)
    s1 = rng.uniform(0.1, 1.0, (3, 3))
    s1 = s1 + s1.T
    d2 = rng.uniform(0.5, 2.0, 2)
    s2 = rng.uniform(0.1, 1.0, (2, 2))
    s2 = s2 + s2.T
    A = np.zeros((5, 5))
    A[:3, :3] = s1 * d1[None, :]                   # symmetric times a positive diagonal
    A[3:, 3:] = s2 * d2[None, :]
    lam, x0, x1, _ = snrt.snrt_kernel_modes(A)
    assert np.abs((x0 @ x1).T - A).max() < 1e-13
    lam, x0, x1, _ = snrt.snrt_kernel_modes(np.array([[0.37]]))
    assert lam[0] == pytest.approx(0.37, abs=1e-16)
    assert (x0 @ x1)[0, 0] == pytest.approx(0.37, abs=1e-16)
    A2 = np.array([[2.0, 1.0], [4.0, 3.0]])        # r = (4, 1) symmetrises it
    lam, x0, x1, _ = snrt.snrt_kernel_modes(A2)
    ref = np.sort(np.linalg.eigvals(A2).real)
    assert np.abs(np.sort(lam) - ref).max() < 1e-14 * 5
    assert np.abs((x0 @ x1).T - A2).max() < 1e-14 * 5


def test_refusals():
    snrt = _lib()
    rng = np.random.default_rng(9)
    # a generic positive matrix: no positive diagonal makes it symmetric (cycle condition)
    with pytest.raises(snrt.SnrtError) as ei:
        snrt.snrt_kernel_modes(rng.uniform(0.1, 1.0, (6, 6)))
    assert ei.value.status == snrt.SNRT_E_UNSUPPORTED
    assert "snrt_kernel_modes" in str(ei.value)
    # opposite signs across the diagonal: the ratio would have to be negative
    with pytest.raises(snrt.SnrtError) as ei:
        snrt.snrt_kernel_modes(np.array([[1.0, 0.5], [-0.5, 1.0]]))
    assert ei.value.status == snrt.SNRT_E_UNSUPPORTED
    # one-sided zero pattern
    with pytest.raises(snrt.SnrtError) as ei:
        snrt.snrt_kernel_modes(np.array([[1.0, 0.5], [0.0, 1.0]]))
    assert ei.value.status == snrt.SNRT_E_UNSUPPORTED
    with pytest.raises(snrt.SnrtError) as ei:
        snrt.snrt_kernel_modes(np.array([[1.0, np.nan], [0.5, 1.0]]))
    assert ei.value.status == snrt.SNRT_E_ARG
    with pytest.raises(snrt.SnrtError) as ei:
        snrt.snrt_kernel_modes(np.zeros((0, 0)))
    assert ei.value.status == snrt.SNRT_E_ARG
