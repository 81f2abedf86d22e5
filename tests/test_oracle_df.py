"""Pins of the DF-factor oracle against facts that do not come from it."""
import numpy as np
import pytest

from oracle.dffactors import df_factors, metric_inverse_sqrt, mo_three_index
from paper_2103_08473_amd.synth import make_df_inputs


def test_inverse_sqrt_of_a_diagonal_metric_is_elementwise():
    d = np.array([4.0, 0.25, 9.0, 1e-3])
    np.testing.assert_allclose(metric_inverse_sqrt(np.diag(d)), np.diag(d ** -0.5), rtol=1e-14, atol=0)


def test_inverse_sqrt_squares_to_the_inverse():
    _, _, V, _ = make_df_inputs(6, 4, 30, seed=1)
    W = metric_inverse_sqrt(V)
    assert np.abs(W - W.T).max() < 1e-13
    np.testing.assert_allclose(W @ V @ W, np.eye(30), atol=1e-12, rtol=0)


@pytest.mark.parametrize("nao,n,X,seed", [(6, 4, 10, 0), (12, 12, 40, 3), (9, 5, 25, 7)])
def test_fitted_integrals_equal_the_closed_form(nao, n, X, seed):
    """J = L K and V = L L^T give J V^-1 J = K K: sum_P B B equals sum_P K~ K~, K~ = C^H K C,
    computed without the metric."""
    C, J, V, K = make_df_inputs(nao, n, X, seed=seed)
    B = df_factors(C, J, V)
    Kt = np.einsum("mp,Pmn,nq->Ppq", np.conj(C), K, C)
    lhs = np.einsum("Ppq,Prs->pqrs", B, B)
    rhs = np.einsum("Ppq,Prs->pqrs", Kt, Kt)
    assert np.abs(rhs).max() > 0.1
    np.testing.assert_allclose(lhs, rhs, atol=1e-12, rtol=0)


def test_fitted_integrals_equal_the_solve_route():
    """sum_P B B == (pq|Q) V^-1 (R|rs) with V^-1 applied by a linear solve (no square root)."""
    C, J, V, _ = make_df_inputs(8, 6, 20, seed=4)
    V = V + 0.3 * np.eye(20)                 # a metric that is not of the L L^T form
    B = df_factors(C, J, V)
    M = mo_three_index(C, J)
    X = np.linalg.solve(V, M.reshape(20, -1)).reshape(M.shape)
    np.testing.assert_allclose(np.einsum("Ppq,Prs->pqrs", B, B), np.einsum("Qpq,Qrs->pqrs", M, X),
                               atol=1e-12, rtol=0)


def test_factors_are_hermitian():
    C, J, V, _ = make_df_inputs(7, 5, 12, seed=2)
    B = df_factors(C, J, V)
    np.testing.assert_allclose(B, np.conj(B.transpose(0, 2, 1)), atol=1e-14, rtol=0)


def test_transform_equals_explicit_loops():
    C, J, V, _ = make_df_inputs(3, 2, 2, seed=5)
    M = mo_three_index(C, J)
    for Q in range(2):
        for p in range(2):
            for q in range(2):
                s = sum(np.conj(C[m, p]) * J[Q, m, nn] * C[nn, q] for m in range(3) for nn in range(3))
                assert abs(M[Q, p, q] - s) < 1e-14


def test_closed_form_detects_a_planted_missing_conjugate():
    C, J, V, K = make_df_inputs(6, 4, 10, seed=0)
    bad = np.einsum("PQ,Qpq->Ppq", metric_inverse_sqrt(V), np.einsum("mp,Qmn,nq->Qpq", C, J, C))
    Kt = np.einsum("mp,Pmn,nq->Ppq", np.conj(C), K, C)
    assert np.abs(np.einsum("Ppq,Prs->pqrs", bad, bad) - np.einsum("Ppq,Prs->pqrs", Kt, Kt)).max() > 1e-3
