"""Host-side set-up of the P_N step in libsnrt (no device): the library's flux Jacobians and
|A| = A^+ - A^- against the oracle's (Sec. 3.1 P_N closure, Sec. 4.3).  The library builds
them with its own product rule, harmonics and Jacobi eigen-solver (blockwise over the
reflection classes); the oracle with numpy's eigh on the full matrices."""
import numpy as np
import pytest

from oracle import pn


def _lib():
    from paper_2205_08417_amd import snrt
    try:
        snrt.lib()
    except OSError as e:
        pytest.skip(str(e))
    return snrt


@pytest.mark.parametrize("N", [0, 1, 2, 5, 9, 13])
def test_library_operators_match_oracle(N):
    snrt = _lib()
    ax, ay, axa, aya = snrt.snrt_pn_operators(N)
    Ax, Ay, _ = pn.flux_jacobians(N)
    axp, axm = pn.split(Ax)
    ayp, aym = pn.split(Ay)
    for got, ref in ((ax, Ax), (ay, Ay), (axa, axp - axm), (aya, ayp - aym)):
        assert np.abs(got - ref).max() < 1e-13


def test_operator_degree_range():
    snrt = _lib()
    with pytest.raises(snrt.SnrtError) as ei:
        snrt.snrt_pn_operators(31)
    assert ei.value.status == snrt.SNRT_E_ARG
    with pytest.raises(snrt.SnrtError):
        snrt.snrt_pn_operators(-1)
