"""Seeded input generators: the structure each family promises (no GPU)."""
import numpy as np

from paper_2405_16160_amd import instances as I


def test_kappa_qp_has_the_requested_condition_number():
    for kappa in (1.0, 1e2, 1e4):
        q = I.kappa_qp(kappa, n=160, m=120, a_density=0.05)
        Qd = q.Q.to_scipy().toarray()
        assert np.array_equal(Qd, Qd.T)
        ev = np.linalg.eigvalsh(Qd)
        assert ev.min() > 0
        assert abs(ev.max() / ev.min() - kappa) <= 1e-8 * kappa
        assert np.count_nonzero(Qd) <= 160 * 8


def test_portfolio_factor_reproduces_q():
    for i in range(3):
        q = I.portfolio_qp(i, nmax=300)
        F, d = I.portfolio_factor(i, nmax=300)
        assert F.shape == (q.n, -(-q.n // 10))
        Qd = q.Q.to_scipy().toarray()
        assert np.allclose(Qd, F @ F.T + np.diag(d), rtol=0, atol=1e-14)
