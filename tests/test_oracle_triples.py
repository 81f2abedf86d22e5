"""Pins of the oracle's perturbative triples (App. C) against brute-force second quantisation.

The brute force builds W_N T2 |0> and W_N T1 |0> in the full Fock space (the
Hamiltonian of tests/sq_brute.py; its diagonal Fock part cannot reach triples)
and projects on every |Phi_ijk^abc>, i<j<k, a<b<c.  Fourth-order triples energy
sum_T |<T|W_N T2|0>|^2 / (E_0 - E_T); fifth-order singles-triples energy
2 Re sum_T conj(<T|W_N T1|0>) <T|W_N T2|0> / (E_0 - E_T).
"""
import itertools

import numpy as np
import pytest

from oracle.integrals import antisym
from oracle.triples import triples_W, triples_Y, triples_Z, triples_energies
from paper_2103_08473_amd.synth import make_amplitudes, make_system
import sq_brute


def brute_triples(eps, V, o, t1, t2):
    n = eps.size
    v = n - o
    F = sq_brute.Fock(n)
    h = sq_brute.core_h(eps, V, o)
    phi0 = np.zeros(1 << n, dtype=np.complex128)
    phi0[(1 << o) - 1] = 1.0
    chi2 = sq_brute.apply_H(F, h, V, sq_brute.apply_T(F, o, np.zeros_like(t1), t2, phi0))
    chi1 = sq_brute.apply_H(F, h, V, sq_brute.apply_T(F, o, t1, np.zeros_like(t2), phi0))
    chiY = sq_brute.exp_T(F, o, t1, t2, phi0)        # e^(T1 + T2) |0>
    W, Z, Y, e4, e5 = {}, {}, {}, 0.0, 0.0
    for i, j, k in itertools.combinations(range(o), 3):
        for a, b, c in itertools.combinations(range(v), 3):
            basis = F.ad(o + a, F.ad(o + b, F.ad(o + c, F.a(k, F.a(j, F.a(i, phi0))))))
            w, z = np.vdot(basis, chi2), np.vdot(basis, chi1)
            D = eps[o + a] + eps[o + b] + eps[o + c] - eps[i] - eps[j] - eps[k]
            W[(i, j, k, a, b, c)], Z[(i, j, k, a, b, c)] = w, z
            Y[(i, j, k, a, b, c)] = np.vdot(basis, chiY)
            e4 += -abs(w) ** 2 / D
            e5 += -2.0 * (np.conj(z) * w).real / D
    return W, Z, Y, e4, e5


@pytest.mark.parametrize("o,v,X,seed", [(3, 4, 9, 5), (4, 3, 8, 6), (4, 4, 10, 7)])
def test_triples_match_brute_force(o, v, X, seed):
    eps, B = make_system(o, v, X, seed=seed, sigma=0.3)
    t1, t2 = make_amplitudes(o, v, seed=seed + 50, scale=0.2)
    n = o + v
    V = antisym(B, slice(0, n), slice(0, n), slice(0, n), slice(0, n))
    Wb, Zb, Yb, e4b, e5b = brute_triples(eps, V, o, t1, t2)
    Wt, Zt, Yt = triples_W(V, o, t2), triples_Z(V, o, t1), triples_Y(t1, t2)
    assert max(abs(w) for w in Wb.values()) > 0.05
    assert max(abs(Wt[key] - Wb[key]) for key in Wb) < 1e-13
    assert max(abs(Zt[key] - Zb[key]) for key in Zb) < 1e-13
    assert max(abs(Yt[key] - Yb[key]) for key in Yb) < 1e-13
    e4, e_t, e_mt = triples_energies(eps, V, o, t1, t2)
    assert abs(e4 - e4b) < 1e-13
    assert abs((e_t - e4) - 0.5 * e5b) < 1e-13
    ey = sum((np.conj(Yb[key]) * Wb[key]).real for key in Wb)    # unique triples: 36 / 36
    assert abs((e_mt - e4) - ey) < 1e-13


def test_two_fifth_order_forms_agree_at_a_converged_solve():
    """At converged CCSD amplitudes the E((T)) and E(-T) singles-triples terms are two
    estimates of the same fifth-order quantity: same sign, same order of magnitude."""
    from oracle.ccsd import build_integrals, solve
    o, v, X = 4, 12, 30
    eps, B = make_system(o, v, X, seed=3, sigma=0.05)
    res = solve(eps, B, o, max_iter=100, tol=1e-11, ints=build_integrals(B, o))
    assert res.converged
    n = o + v
    V = antisym(B, slice(0, n), slice(0, n), slice(0, n), slice(0, n))
    e4, e_t, e_mt = triples_energies(eps, V, o, res.t1, res.t2)
    d5, dy = e_t - e4, e_mt - e4
    assert e4 < 0 and abs(d5) > 0 and d5 * dy > 0 and 0.2 < dy / d5 < 5.0


def test_printed_elements_differ_only_for_complex_spinors():
    """With real factors the printed <ie||ab>, <ij||am> equal the excitation elements."""
    o, v, X = 3, 4, 9
    eps, B = make_system(o, v, X, seed=8, sigma=0.3)
    t1, t2 = make_amplitudes(o, v, seed=9, scale=0.2)
    n = o + v
    for real in (True, False):
        Bx = 0.5 * (B.real + B.real.transpose(0, 2, 1)).astype(np.complex128) if real else B
        t2x = t2.real.astype(np.complex128) if real else t2
        V = antisym(Bx, slice(0, n), slice(0, n), slice(0, n), slice(0, n))
        O, Vs = slice(0, o), slice(o, n)
        Ve, Vm = V[O, Vs, Vs, Vs], V[O, O, Vs, O]      # printed <ie||ab>, <ij||am>
        W = (np.einsum('ieab,jkec->ijkabc', Ve, t2x) + np.einsum('jeab,kiec->ijkabc', Ve, t2x)
             + np.einsum('keab,ijec->ijkabc', Ve, t2x) + np.einsum('ijam,kmbc->ijkabc', Vm, t2x)
             + np.einsum('jkam,imbc->ijkabc', Vm, t2x) + np.einsum('kiam,jmbc->ijkabc', Vm, t2x))
        Wp = W + W.transpose(0, 1, 2, 4, 5, 3) + W.transpose(0, 1, 2, 5, 3, 4)
        d = np.abs(Wp - triples_W(V, o, t2x)).max()
        assert (d < 1e-14) if real else (d > 1e-3)


def test_no_triples_for_two_electrons():
    eps, B = make_system(2, 6, 12, seed=1, sigma=0.2)
    t1, t2 = make_amplitudes(2, 6, seed=2, scale=0.2)
    V = antisym(B, slice(0, 8), slice(0, 8), slice(0, 8), slice(0, 8))
    assert triples_energies(eps, V, 2, t1, t2) == (0.0, 0.0, 0.0)
