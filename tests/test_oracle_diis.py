"""Pins of the oracle's Pulay DIIS step (section "Coupled cluster implementation").

DIIS picks the combination of stored error vectors with the smallest norm among
those whose coefficients sum to one.  That is a constrained linear least-squares
problem with a textbook solution independent of the bordered Gram system the
oracle solves: eliminate c_0 = 1 - sum_{k>=1} c_k, so that
sum_k c_k e_k = e_0 + sum_{k>=1} c_k (e_k - e_0), and minimise over the free c_k
with numpy's least-squares routine.  Both must give the same coefficients and the
same extrapolated vector.
"""
import numpy as np
import pytest

from oracle.ccsd import DIIS


def _constrained_lstsq(es):
    """argmin ||sum c_k e_k||_2 subject to sum c_k = 1 (complex c), by elimination."""
    e0 = es[0]
    D = np.stack([e - e0 for e in es[1:]], axis=1)
    cf, *_ = np.linalg.lstsq(D, -e0, rcond=None)
    return np.concatenate([[1.0 - cf.sum()], cf])


def _vectors(m, L, seed):
    rng = np.random.default_rng(seed)
    es = [rng.normal(size=L) + 1j * rng.normal(size=L) for _ in range(m)]
    xs = [rng.normal(size=L) + 1j * rng.normal(size=L) for _ in range(m)]
    return xs, es


@pytest.mark.parametrize("m", [2, 3, 5, 8])
def test_diis_coefficients_are_the_constrained_least_squares_minimiser(m):
    xs, es = _vectors(m, 40, seed=m)
    d = DIIS(8)
    for x, e in zip(xs, es):
        d.push(x, e)
    c = d.coefficients()
    ref = _constrained_lstsq(es)
    assert abs(c.sum() - 1.0) < 1e-13
    assert np.abs(c - ref).max() < 1e-11 * max(1.0, np.abs(ref).max())
    # the extrapolated vector is sum c_k x_k with those coefficients
    assert np.abs(d.extrapolate() - sum(ck * xk for ck, xk in zip(ref, xs))).max() < 1e-10
    # and its error combination is no longer than any single stored error vector
    comb = np.linalg.norm(sum(ck * ek for ck, ek in zip(c, es)))
    assert comb <= min(np.linalg.norm(e) for e in es) + 1e-12


def test_diis_pin_fails_for_a_transposed_gram_matrix():
    """The plausible slip G_kl = <e_l, e_k> (the conjugate on the wrong side, i.e. G^T) is
    what the oracle computes when it is handed the conjugated error vectors; the
    least-squares pin must reject it."""
    xs, es = _vectors(5, 40, seed=11)
    d = DIIS(8)
    for x, e in zip(xs, es):
        d.push(x, np.conj(e))            # <conj e_k, conj e_l> = conj(G_kl) = G_lk
    c_wrong = d.coefficients()
    ref = _constrained_lstsq(es)
    assert np.abs(c_wrong - ref).max() > 1e-3


def test_diis_keeps_only_the_last_size_pairs():
    xs, es = _vectors(11, 30, seed=3)
    d = DIIS(4)
    for x, e in zip(xs, es):
        d.push(x, e)
    assert len(d.es) == 4
    ref = _constrained_lstsq(es[-4:])
    assert np.abs(d.coefficients() - ref).max() < 1e-11 * max(1.0, np.abs(ref).max())


def test_diis_drops_the_oldest_pair_of_a_degenerate_subspace():
    """Two equal error vectors make G singular: the oldest pair goes and the least-squares
    solution over what remains is used."""
    xs, es = _vectors(3, 30, seed=5)
    es = [es[0], es[0].copy(), es[1], es[2]]
    xs = xs + [xs[0]]
    d = DIIS(8)
    for x, e in zip(xs, es):
        d.push(x, e)
    c = d.coefficients()
    assert len(d.es) == 3
    ref = _constrained_lstsq(es[1:])
    assert np.abs(c - ref).max() < 1e-9 * max(1.0, np.abs(ref).max())


def test_diis_with_one_pair_is_the_jacobi_step():
    xs, es = _vectors(1, 10, seed=2)
    d = DIIS(8)
    d.push(xs[0], es[0])
    assert np.array_equal(d.extrapolate(), xs[0])
