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


def test_row_scaled_keeps_the_optimum():
    # the manufactured instance fixes (x*, y*); scaling row i by s_i keeps x*
    # and divides y*_i by s_i, so the KKT residual of the mapped pair stays ~0
    from oracle import oracle as O
    qp = I.manufactured()
    k0 = O.kkt(qp, qp.x_star, qp.y_star)["rel_kkt"]
    rs = I.row_scaled(qp)
    assert rs.A.nnz == qp.A.nnz and not np.allclose(rs.b, qp.b)
    assert O.kkt(rs, rs.x_star, rs.y_star)["rel_kkt"] <= max(1e-12, 10 * k0)


def test_portfolio_lowrank_is_the_same_qp():
    """The factored generator draws the same F, d, A, b, c as the dense one,
    and F F' + diag(d) equals the dense Q up to rounding."""
    for i in (0, 3, 11):
        q = I.portfolio_qp(i, nmax=300)
        ql, (F, d) = I.portfolio_lowrank(i, nmax=300)
        assert np.array_equal(q.A.to_scipy().toarray(), ql.A.to_scipy().toarray())
        assert np.array_equal(q.b, ql.b) and np.array_equal(q.c, ql.c)
        Qd = q.Q.to_scipy().toarray()
        np.testing.assert_allclose(F @ F.T + np.diag(d), Qd, rtol=0, atol=1e-14)
