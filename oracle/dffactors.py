"""Density-fitting factors from AO three-index integrals (oracle; test infrastructure).

The paper names density fitting and Cholesky decomposition (Introduction) as the way
to shrink the two-electron integral tensor, and finds the AO->MO integral
transformation a large share of the time at small node counts (Performance section;
its MOINT_SCHEME keyword selects a Cholesky-based scheme).  This is the step before
the CC iteration that produces its input factors.  The standard robust-fitting
definition, with (mu nu|Q) the AO three-index integrals, V_QR = (Q|R) the metric and
C the spinor coefficients:

    B^P_pq = sum_Q [V^-1/2]_PQ sum_{mu nu} conj(C_mu p) (mu nu|Q) C_nu q,

so that sum_P B^P_pq B^P_rs = sum_QR (pq|Q) [V^-1]_QR (R|rs), the fitted (pq|rs).
V^-1/2 is the symmetric inverse square root, written out from the eigendecomposition.
Pinned in tests/test_oracle_df.py (closed-form fitted integrals, the solve route,
Hermiticity, brute-force transform).
"""
import numpy as np


def metric_inverse_sqrt(V):
    """V^-1/2 = U diag(w^-1/2) U^T for the symmetric positive definite metric V."""
    w, U = np.linalg.eigh(V)
    if w[0] <= 0.0:
        raise ValueError("metric not positive definite")
    return (U * w ** -0.5) @ U.T


def mo_three_index(C, J):
    """(pq|Q) = sum_{mu nu} conj(C_mu p) (mu nu|Q) C_nu q, as M[Q][p][q]."""
    return np.einsum("mp,Qmn,nq->Qpq", np.conj(C), J, C, optimize=True)


def df_factors(C, J, V):
    """B[P][p][q] of the definition above."""
    return np.einsum("PQ,Qpq->Ppq", metric_inverse_sqrt(V), mo_three_index(C, J), optimize=True)
