"""Graph-replayed residual (opts.graph_residual) against direct launches (run on an MI355X).

With graph_residual set, the first iteration of each kind (low precision, FP64, FP64 with
the defect-corrected products) records its residual kernels into a HIP graph and later
iterations replay it.  Between replays the iteration runs its own direct work (assembly,
DIIS with a host readback, energy), so every replay is checked against that eager
interleaving: each step's energy and step norm, and the final amplitudes, must be bitwise
those of a handle that launches every kernel directly; the converged energy is checked
against the oracle."""
import sys

import numpy as np
import pytest

from paper_2103_08473_amd.synth import make_system

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = [
    # (nocc, nvir, naux, precision name, steps)
    (6, 40, 120, "FP64", 14),
    (8, 48, 144, "MIXED_FP32", 60),
    (7, 42, 126, "MIXED_BF16X3", 60),
]


@pytest.mark.parametrize("o,v,X,prec,steps", CASES)
def test_graph_replay_is_bitwise_direct(o, v, X, prec, steps, lib):
    from paper_2103_08473_amd import exacc
    say("graph replay", o, v, X, prec)
    eps, B = make_system(o, v, X, seed=11)
    p = getattr(exacc, prec)
    hist = {}
    amps = {}
    kinds = {}
    for graph in (0, 1):
        rows, seen = [], set()
        with exacc.CCSD(eps, B, o, precision=p, tol=1e-10, max_iter=200, graph_residual=graph) as cc:
            for _ in range(steps):
                seen.add(cc.phase()[0])
                st, n, r, conv = cc.iterate(1)
                rows.append((cc.energy(), r))
                if conv:
                    break
            amps[graph] = cc.amplitudes()
        hist[graph] = rows
        kinds[graph] = seen
    assert len(hist[0]) == len(hist[1])
    for k, (a, b) in enumerate(zip(hist[0], hist[1])):
        assert a[0] == b[0] and a[1] == b[1], (k, a, b)
    assert np.array_equal(amps[0][0], amps[1][0]) and np.array_equal(amps[0][1], amps[1][1])
    if prec != "FP64":  # low precision, corrected and FP64 kinds all replayed
        assert kinds[1] == {0, 1, 2}
    say("  %d steps bitwise equal, kinds %s, last |Delta| %.2e" % (len(hist[1]), sorted(kinds[1]), hist[1][-1][1]))


def test_graph_solve_matches_oracle(lib):
    from oracle.ccsd import solve as oracle_solve
    from paper_2103_08473_amd import exacc
    o, v, X = 5, 40, 120
    eps, B = make_system(o, v, X, seed=12)
    res = oracle_solve(eps, B, o, max_iter=80, tol=1e-10)
    assert res.converged
    e_or = res.energy
    with exacc.CCSD(eps, B, o, precision=exacc.MIXED_BF16X3, tol=1e-10, max_iter=80, graph_residual=1) as cc:
        e, conv, _ = cc.solve()
    say("  graph BF16x3 solve E %.12f, oracle %.12f" % (e.real, e_or.real))
    assert conv and abs(e - e_or) <= 1e-8
