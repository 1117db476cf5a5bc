"""CPU checks of the warm-start data preparation: the dual targets are made
canonical only on row pairs that encode equalities, which keeps A'y and b'y."""
import numpy as np
import pytest

from paper_2405_16160_amd import instances as I
from paper_2405_16160_amd import warmstart as W


def test_canonical_duals_keep_At_y_and_b_y():
    fam = I.mpc_family()
    plus, minus = W.pair_index(fam)
    A = fam.A.to_scipy()
    assert abs(A[plus] + A[minus]).max() == 0          # rows really are +/- pairs
    b = fam.b_for(I.mpc_initial_state(0, fam))
    assert np.array_equal(b[plus], -b[minus])           # ... of equalities
    rng = np.random.default_rng(0)
    Y = np.abs(rng.standard_normal((3, fam.A.nrows)))
    Yc = W.canonical_duals(Y, plus, minus)
    for y, yc in zip(Y, Yc):
        assert np.allclose(A.T @ y, A.T @ yc, atol=1e-12)
        assert b @ y == pytest.approx(b @ yc, abs=1e-10)
        assert np.all(np.minimum(yc[plus], yc[minus]) == 0)



def test_dual_code_round_trip():
    fam = I.mpc_family()
    plus, minus = W.pair_index(fam)
    code = W.DualCode(fam.A.nrows, plus, minus)
    rng = np.random.default_rng(1)
    Y = W.canonical_duals(np.abs(rng.standard_normal((4, fam.A.nrows))), plus, minus)
    assert code.width == fam.A.nrows - len(plus)
    assert np.allclose(code.decode(code.encode(Y)), Y, atol=0, rtol=0)
