"""DF-factor generation: HIP path vs the CPU oracle through the C ABI (run on an MI355X)."""
import sys

import numpy as np
import pytest

from oracle.dffactors import df_factors as df_oracle
from paper_2103_08473_amd.synth import make_df_inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# one element, below one 64-tile, ragged multi-tile, nspinor = nao
@pytest.mark.parametrize("nao,n,X", [(1, 1, 1), (6, 4, 10), (40, 30, 100), (130, 70, 300), (64, 64, 64)])
def test_df_factors_match_oracle(lib, nao, n, X):
    from paper_2103_08473_amd import exacc
    say("df case", nao, n, X)
    C, J, V, _ = make_df_inputs(nao, n, X, seed=nao + n + X)
    ref = df_oracle(C, J, V)
    B, iters = exacc.df_factors(C, J, V)
    say("  newton-schulz steps", iters)
    assert np.abs(B - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_df_factors_device_pointers_and_closed_form(lib):
    """Device-tensor path; the fitted integrals equal sum_P K~ K~ (J = L K, V = L L^T)."""
    import torch
    from paper_2103_08473_amd import exacc
    C, J, V, K = make_df_inputs(24, 16, 80, seed=9)
    B, _ = exacc.df_factors(torch.from_numpy(C).cuda(), torch.from_numpy(J).cuda(),
                            torch.from_numpy(V).cuda())
    B = B.cpu().numpy()
    Kt = np.einsum("mp,Pmn,nq->Ppq", np.conj(C), K, C)
    np.testing.assert_allclose(np.einsum("Ppq,Prs->pqrs", B, B), np.einsum("Ppq,Prs->pqrs", Kt, Kt),
                               atol=1e-11, rtol=0)
    np.testing.assert_allclose(B, np.conj(B.transpose(0, 2, 1)), atol=1e-13, rtol=0)


def test_df_factors_feed_a_ccsd_solve(lib):
    """Generated factors drive the amplitude iteration: the GPU solve on them equals the
    oracle's solve on the oracle's factors."""
    import oracle
    from paper_2103_08473_amd import exacc
    from paper_2103_08473_amd.exacc import CCSD
    nao, n, X, o = 20, 14, 40, 4
    C, J, V, _ = make_df_inputs(nao, n, X, seed=12, sigma=0.05)
    eps = np.concatenate([np.linspace(-1.5, -0.6, o), np.linspace(0.4, 2.0, n - o)])
    B, _ = exacc.df_factors(C, J, V)
    ref = oracle.solve(eps, df_oracle(C, J, V), o, max_iter=60, tol=1e-10)
    with CCSD(eps, B, o, tol=1e-10, max_iter=60) as cc:
        e, conv, _ = cc.solve()
    assert ref.converged and conv
    assert abs(e - ref.energy) <= 1e-10


def test_df_factors_reject_bad_input(lib):
    from paper_2103_08473_amd import exacc
    C, J, V, _ = make_df_inputs(6, 4, 10, seed=1)
    with pytest.raises(exacc.ExaccError) as e:
        exacc.df_factors(C, J, -V)           # negative definite metric: the iteration diverges
    assert e.value.status == exacc.ERR_INVALID_ARG
    with pytest.raises(exacc.ExaccError):
        exacc.df_factors(np.zeros((3, 5), np.complex128), J[:, :3, :3], V)   # nspinor > nao


def test_df_factors_ill_conditioned_metric(lib):
    """Metric eigenvalues spread over 1e-6..1 (condition number 1e6): about 20 Newton-Schulz
    steps; the factors still match the eigendecomposition route to 1e-9 relative."""
    from paper_2103_08473_amd import exacc
    nao, n, X = 30, 20, 200
    C, J, _, _ = make_df_inputs(nao, n, X, seed=21)
    rng = np.random.default_rng(22)
    U, _ = np.linalg.qr(rng.normal(size=(X, X)))
    V = (U * np.logspace(-6, 0, X)) @ U.T
    V = 0.5 * (V + V.T)
    ref = df_oracle(C, J, V)
    B, iters = exacc.df_factors(C, J, V)
    say("  newton-schulz steps", iters)
    assert iters < 60
    assert np.abs(B - ref).max() <= 1e-9 * np.abs(ref).max()
