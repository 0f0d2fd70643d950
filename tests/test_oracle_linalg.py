"""Pins of the oracle's dense LU (used by the Newton step of the implicit
integrator) against LAPACK through numpy and against its own definition
P A = L U."""
import numpy as np
import pytest


@pytest.mark.parametrize("n", [1, 2, 7, 64, 131])
def test_lu_reconstructs_and_solves(oracle_mod, n):
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n))
    LU, piv, info = oracle_mod.lu_factor(A)
    assert info == 0
    L = np.tril(LU, -1) + np.eye(n)
    U = np.triu(LU)
    PA = A.copy()
    for k in range(n):
        PA[[k, piv[k]]] = PA[[piv[k], k]]
    np.testing.assert_allclose(L @ U, PA, atol=1e-12 * np.abs(A).max() * n)
    # partial pivoting: every multiplier is at most 1 in magnitude
    assert np.all(np.abs(np.tril(LU, -1)) <= 1.0)
    b = rng.standard_normal(n)
    x = oracle_mod.lu_solve(LU, piv, b)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-12)
    xt = oracle_mod.lu_solve(LU, piv, b, trans=True)
    np.testing.assert_allclose(xt, np.linalg.solve(A.T, b), rtol=1e-9, atol=1e-12)


def test_lu_newton_matrix(oracle_mod, medium):
    """M = I - c J of the paper-sized network over the range of c the
    integrator meets; solves agree with LAPACK."""
    net, cells = medium
    J = oracle_mod.jac_dense(net, cells.y0[:1], cells.T[:1])[0]
    rng = np.random.default_rng(0)
    for c in (1e-3, 1e4, 1e10):
        M = np.eye(J.shape[0]) - c * J
        LU, piv, info = oracle_mod.lu_factor(M)
        assert info == 0
        b = rng.standard_normal(J.shape[0])
        x = oracle_mod.lu_solve(LU, piv, b)
        r = M @ x - b
        assert np.linalg.norm(r) <= 1e-10 * (np.linalg.norm(M, 1) * np.linalg.norm(x) + np.linalg.norm(b))
        xt = oracle_mod.lu_solve(LU, piv, b, trans=True)
        rt = M.T @ xt - b
        assert np.linalg.norm(rt) <= 1e-10 * (np.linalg.norm(M, 1) * np.linalg.norm(xt) + np.linalg.norm(b))


def test_lu_reports_zero_pivot(oracle_mod):
    A = np.array([[1.0, 2.0, 3.0], [2.0, 4.0, 6.0], [1.0, 0.0, 1.0]])
    A[:, 2] = A[:, 0] + A[:, 1]        # rank 2
    A[2] = [0.0, 0.0, 0.0]
    _, _, info = oracle_mod.lu_factor(A)
    assert info > 0


def test_lu_row_swap_example(oracle_mod):
    """A matrix whose first pivot must come from the last row."""
    A = np.array([[0.0, 1.0], [3.0, 4.0]])
    LU, piv, info = oracle_mod.lu_factor(A)
    assert info == 0 and piv.tolist() == [1, 1]
    np.testing.assert_array_equal(LU, [[3.0, 4.0], [0.0, 1.0]])
