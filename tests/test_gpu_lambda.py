"""Lambda equations (App. D) and the one-body density (App. E): HIP path vs the CPU
oracle, through the C ABI (run on an MI355X)."""
import sys

import numpy as np
import pytest

import oracle
from oracle.cclambda import density, lambda_residual, solve_lambda
from oracle.integrals import antisym
from paper_2103_08473_amd.synth import make_amplitudes, make_system

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _full_V(B, n):
    return antisym(B, slice(0, n), slice(0, n), slice(0, n), slice(0, n))


# below one 64-tile, several tiles with ragged tails, one occupied (no pairs), one virtual
LAMBDA_CASES = [(3, 4, 9), (5, 7, 13), (10, 40, 120), (12, 70, 150), (1, 9, 20), (2, 12, 30),
                (4, 1, 6)]


@pytest.mark.parametrize("group", [64, 0])
@pytest.mark.parametrize("o,v,X", LAMBDA_CASES)
def test_lambda_residual_matches_oracle(lib, o, v, X, group):
    """R1, R2 of App. D at random t and lambda, element by element, 1e-12 of max |R|; the
    ladder with all rows' tiles in one product (group 64) and per row (0)."""
    from paper_2103_08473_amd.exacc import CCSD
    say("lambda residual case", o, v, X, "ladder_group_nvir", group)
    eps, B = make_system(o, v, X, seed=o * 1000 + v + 5, sigma=0.2)
    t1, t2 = make_amplitudes(o, v, seed=17 + o, scale=0.1)
    l1, l2 = make_amplitudes(o, v, seed=29 + o, scale=0.1)
    R1, R2 = lambda_residual(eps, _full_V(B, o + v), o, t1, t2, l1, l2)
    with CCSD(eps, B, o, ladder_group_nvir=group) as cc:
        cc.set_amplitudes(t1, t2)
        cc.set_lambda(l1, l2)
        g1, g2 = cc.lambda_residual()
        m1, m2 = cc.get_lambda()
        r1, r2 = cc.amplitudes()
    assert np.array_equal(m1, l1) and np.array_equal(m2, l2)
    assert np.array_equal(r1, t1) and np.array_equal(r2, t2)
    scale = max(np.abs(R2).max() if R2.size else 0.0, np.abs(R1).max(), 1e-300)
    assert np.abs(g1 - R1).max() <= 1e-12 * scale
    if R2.size:
        assert np.abs(g2 - R2).max() <= 1e-12 * scale


@pytest.mark.parametrize("o,v,X", [(3, 5, 11), (7, 20, 48), (1, 9, 20)])
def test_density_matches_oracle(lib, o, v, X):
    """App. E density at random t and lambda, element by element."""
    from paper_2103_08473_amd.exacc import CCSD
    say("density case", o, v, X)
    eps, B = make_system(o, v, X, seed=o + 3 * v, sigma=0.2)
    t1, t2 = make_amplitudes(o, v, seed=41 + o, scale=0.1)
    l1, l2 = make_amplitudes(o, v, seed=43 + o, scale=0.1)
    ref = density(t1, t2, l1, l2)
    with CCSD(eps, B, o) as cc:
        cc.set_amplitudes(t1, t2)
        cc.set_lambda(l1, l2)
        g = cc.density()
    assert np.abs(g - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("o,v,X,seed", [(6, 24, 60, 17), (2, 14, 30, 3), (10, 40, 120, 0)])
def test_lambda_solve_matches_oracle(lib, o, v, X, seed):
    """Converged CCSD, then converged Lambda and the density, vs the oracle's solves:
    max |d lambda| and max |d gamma| within 1e-9; for two electrons the density plus the
    reference has trace 2 (the oracle's is pinned to the exact 1-RDM)."""
    from paper_2103_08473_amd.exacc import CCSD
    say("lambda solve case", o, v, X, seed)
    eps, B = make_system(o, v, X, seed=seed)
    ref = oracle.solve(eps, B, o, max_iter=80, tol=1e-11)
    lam = solve_lambda(eps, _full_V(B, o + v), o, ref.t1, ref.t2, tol=1e-11, max_iter=80)
    assert ref.converged and lam.converged
    gref = density(ref.t1, ref.t2, lam.l1, lam.l2)
    with CCSD(eps, B, o, tol=1e-11, max_iter=80) as cc:
        _, conv, _ = cc.solve()
        lconv, hist = cc.lambda_solve()
        l1, l2 = cc.get_lambda()
        g = cc.density()
    assert conv and lconv
    say("  lambda iterations gpu %d oracle %d" % (len(hist), lam.iterations))
    assert np.abs(l1 - lam.l1).max() <= 1e-9
    assert np.abs(l2 - lam.l2).max() <= 1e-9
    assert np.abs(g - gref).max() <= 1e-9
    assert abs(np.trace(g)) <= 1e-12


def test_lambda_rejects_other_methods_and_low_precision(lib):
    from paper_2103_08473_amd import exacc
    from paper_2103_08473_amd.exacc import CCSD
    eps, B = make_system(4, 12, 30, seed=2)
    with CCSD(eps, B, 4, doubles_only=1) as cc:
        with pytest.raises(exacc.ExaccError) as e:
            cc.lambda_iterate(1)
        assert e.value.status == exacc.ERR_INVALID_ARG
    with CCSD(eps, B, 4, cc2=1) as cc:
        with pytest.raises(exacc.ExaccError):
            cc.density()
    with CCSD(eps, B, 4, precision=exacc.MIXED_FP32) as cc:
        assert cc.phase()[0]
        with pytest.raises(exacc.ExaccError) as e:
            cc.lambda_iterate(1)
        assert e.value.status == exacc.ERR_INVALID_ARG


def test_later_allocations_respect_the_budget(lib):
    """The Lambda buffers are allocated after create: with the budget set to the create plan
    (nocc=12, nvir=14: the buffers, about 2.4 MB, exceed the plan's 0.8 MB of create-time
    temporaries) they are refused with NOMEM, nothing stays allocated and the handle keeps
    iterating; with twice the plan the Lambda step and the triples run."""
    from paper_2103_08473_amd import exacc
    from paper_2103_08473_amd.exacc import CCSD
    o, v, X = 12, 14, 42
    eps, B = make_system(o, v, X, seed=5)
    plan = exacc.memory_estimate(o, v, X)
    with CCSD(eps, B, o, hbm_budget_bytes=plan, tol=1e-10) as cc:
        cc.solve(max_iter=40)
        for _ in range(2):   # a second attempt is refused the same way (nothing leaked)
            with pytest.raises(exacc.ExaccError) as e:
                cc.lambda_iterate(1)
            assert e.value.status == exacc.ERR_NOMEM
        st, _, r, _ = cc.iterate(1)
        assert np.isfinite(r)
    with CCSD(eps, B, o, hbm_budget_bytes=2 * plan, tol=1e-10) as cc:
        cc.solve(max_iter=40)
        cc.lambda_iterate(1)
        assert all(np.isfinite(x) for x in cc.triples())
