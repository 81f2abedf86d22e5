"""HIP path vs the CPU oracle, through the C ABI (run on an MI355X)."""
import sys

import numpy as np
import pytest

import oracle
from oracle.ccsd import build_integrals, energy, residual
from paper_2103_08473_amd.synth import make_amplitudes, make_system

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# (nocc, nvir, naux): below one 64-tile, several tiles with ragged tails, degenerate pair spaces
RESIDUAL_CASES = [(3, 4, 9), (5, 7, 13), (10, 40, 120), (12, 70, 150), (16, 67, 131),
                  (1, 9, 20), (2, 12, 30), (4, 1, 6), (1, 1, 3)]


@pytest.mark.parametrize("o,v,X", RESIDUAL_CASES)
def test_residual_matches_oracle(lib, o, v, X):
    from paper_2103_08473_amd.exacc import CCSD
    say("residual case", o, v, X)
    eps, B = make_system(o, v, X, seed=o * 1000 + v, sigma=0.2)
    t1, t2 = make_amplitudes(o, v, seed=7 + o, scale=0.1)
    ints = build_integrals(B, o)
    S1, S2 = residual(eps, ints, t1, t2)
    E = energy(eps, ints, t1, t2)
    with CCSD(eps, B, o) as cc:
        cc.set_amplitudes(t1, t2)
        g1, g2 = cc.residual()
        ge = cc.energy()
        r1, r2 = cc.amplitudes()
    assert np.array_equal(r1, t1) and np.array_equal(r2, t2)
    scale = max(np.abs(S2).max() if S2.size else 0.0, np.abs(S1).max(), 1e-300)
    assert np.abs(g1 - S1).max() <= 1e-12 * scale
    if S2.size:
        assert np.abs(g2 - S2).max() <= 1e-12 * scale
    assert abs(ge - E) <= 1e-12 * max(1.0, abs(E))


@pytest.mark.parametrize("o,v,X,seed,sigma,iters", [
    (10, 40, 120, 0, 0.05, 30),     # the (10, 40, 120) configuration, literal generator
    (6, 50, 150, 1, None, 25),      # ragged tiles, size-scaled generator
])
def test_iterations_match_oracle(lib, o, v, X, seed, sigma, iters):
    """Energy after every iteration (MP2 start, Jacobi step, DIIS(8)) within 1e-10 Eh."""
    from paper_2103_08473_amd.exacc import CCSD
    say("iteration case", o, v, X, seed, sigma)
    eps, B = make_system(o, v, X, seed=seed, sigma=sigma)
    ref = oracle.solve(eps, B, o, max_iter=iters, tol=1e-10)
    with CCSD(eps, B, o, tol=1e-10) as cc:
        _, conv, hist = cc.solve(max_iter=iters)
    assert len(hist) == len(ref.history)
    for (it, eg, rg), (_, eo, ro) in zip(hist, ref.history):
        assert abs(eg - eo) <= 1e-10, (it, eg, eo)
        assert abs(rg - ro) <= 1e-8 * max(1.0, ro), (it, rg, ro)
    assert conv == ref.converged


@pytest.mark.parametrize("v,X,seed", [(8, 20, 0), (14, 30, 1)])
def test_two_electron_equals_fci(lib, v, X, seed):
    from paper_2103_08473_amd.exacc import CCSD
    say("fci case", v, X, seed)
    eps, B = make_system(2, v, X, seed=seed, sigma=0.05)
    e_fci, _, _ = oracle.fci_two_electron(eps, B)
    with CCSD(eps, B, 2, tol=1e-12, max_iter=80) as cc:
        e, conv, _ = cc.solve()
    assert conv
    assert abs(e - e_fci) < 1e-10


def test_one_electron_is_exact_at_first_step(lib):
    from paper_2103_08473_amd.exacc import CCSD
    eps, B = make_system(1, 9, 20, seed=4, sigma=0.1)
    with CCSD(eps, B, 1, tol=1e-14) as cc:
        st, steps, r, conv = cc.iterate(5)
        assert conv and steps == 1 and r == 0.0
        assert cc.energy() == 0


def test_deterministic(lib):
    from paper_2103_08473_amd.exacc import CCSD
    eps, B = make_system(8, 36, 100, seed=3)
    out = []
    for _ in range(2):
        with CCSD(eps, B, 8) as cc:
            cc.iterate(6)
            out.append((cc.energy(), cc.amplitudes()[1]))
    assert out[0][0] == out[1][0]
    assert np.array_equal(out[0][1], out[1][1])


def test_invalid_inputs_are_rejected(lib):
    from paper_2103_08473_amd import exacc
    eps, B = make_system(4, 10, 20, seed=1)
    bad = B.copy()
    bad[3, 1, 2] += 1e-3                         # not Hermitian
    with pytest.raises(exacc.ExaccError) as e:
        exacc.CCSD(eps, bad, 4)
    assert e.value.status == exacc.ERR_INVALID_ARG
    nanB = B.copy()
    nanB[0, 0, 0] = np.nan
    with pytest.raises(exacc.ExaccError) as e:
        exacc.CCSD(eps, nanB, 4)
    assert e.value.status == exacc.ERR_INVALID_ARG
    e2 = eps.copy()
    e2[4] = e2[:4].max()                         # no gap
    with pytest.raises(exacc.ExaccError) as e:
        exacc.CCSD(e2, B, 4)
    assert e.value.status == exacc.ERR_INVALID_ARG
    with pytest.raises(exacc.ExaccError) as e:
        exacc.CCSD(eps, B, 4, hbm_budget_bytes=1 << 20)
    assert e.value.status == exacc.ERR_NOMEM


def test_not_converged_status(lib):
    from paper_2103_08473_amd import exacc
    eps, B = make_system(4, 10, 20, seed=1)
    with exacc.CCSD(eps, B, 4) as cc:
        st, steps, r, conv = cc.iterate(1)
        assert st == exacc.NOT_CONVERGED and steps == 1 and not conv and r > 0
