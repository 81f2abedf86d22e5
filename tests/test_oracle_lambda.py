"""Pins of the Lambda / density oracle (App. D, App. E) against facts that do not come
from it: the gradient of the CC Lagrangian and the density built by brute-force second
quantisation, the exact two-electron density, and the derivative of the CC energy."""
import numpy as np
import pytest

import oracle
from oracle.cclambda import density, hbar, lambda_residual, solve_lambda
from oracle.integrals import antisym
from paper_2103_08473_amd.synth import make_amplitudes, make_system
import sq_brute


def _full_V(B, n):
    return antisym(B, slice(0, n), slice(0, n), slice(0, n), slice(0, n))


def _converged(o, v, X, seed, sigma=0.3):
    eps, B = make_system(o, v, X, seed=seed, sigma=sigma)
    res = oracle.solve(eps, B, o, max_iter=200, tol=1e-13)
    assert res.converged
    return eps, B, res


@pytest.mark.parametrize("o,v,X,seed", [(3, 4, 9, 3), (2, 5, 8, 1), (4, 3, 9, 5)])
def test_lambda_residual_is_the_lagrangian_gradient(o, v, X, seed):
    """App. D residuals == dL/dt_mu = <0|(1+Lambda) e^-T [H, tau_mu] e^T|0> at converged t,
    for random lambda (every term of both equations enters)."""
    eps, B, res = _converged(o, v, X, seed)
    V = _full_V(B, o + v)
    l1, l2 = make_amplitudes(o, v, seed=seed + 11, scale=0.2)
    R1, R2 = lambda_residual(eps, V, o, res.t1, res.t2, l1, l2)
    G1, G2 = sq_brute.lagrangian_gradient(eps, V, o, res.t1, res.t2, l1, l2)
    assert np.abs(G1).max() > 0.1 and np.abs(G2).max() > 0.1
    np.testing.assert_allclose(R1, G1, atol=1e-12, rtol=0)
    np.testing.assert_allclose(R2, G2, atol=1e-12, rtol=0)


def test_brute_force_detects_planted_lambda_error():
    """A residual with one intermediate's sign flipped must fail the comparison."""
    o, v, X = 3, 4, 9
    eps, B, res = _converged(o, v, X, 3)
    V = _full_V(B, o + v)
    l1, l2 = make_amplitudes(o, v, seed=14, scale=0.2)
    h = hbar(eps, V, o, res.t1, res.t2)
    h['ovoo'] = -h['ovoo']           # planted: wrong sign of W_mbij
    R1, _ = lambda_residual(eps, V, o, res.t1, res.t2, l1, l2, h)
    G1, _ = sq_brute.lagrangian_gradient(eps, V, o, res.t1, res.t2, l1, l2)
    assert np.abs(R1 - G1).max() > 1e-3


@pytest.mark.parametrize("o,v,seed", [(3, 4, 2), (2, 5, 7)])
def test_density_is_the_lagrangian_expectation(o, v, seed):
    """App. E density == <0|(1+Lambda) e^-T {q+ p} e^T|0> for random t and lambda."""
    t1, t2 = make_amplitudes(o, v, seed=seed, scale=0.2)
    l1, l2 = make_amplitudes(o, v, seed=seed + 5, scale=0.2)
    g = density(t1, t2, l1, l2)
    gb = sq_brute.lagrangian_density(o, t1, t2, l1, l2)
    assert np.abs(gb[:o, :o]).max() > 0.01 and np.abs(gb[o:, :o]).max() > 0.01
    np.testing.assert_allclose(g, gb, atol=1e-14, rtol=0)
    # the printed oo block is the transpose of <{j+ i}>
    assert np.abs(g[:o, :o] - g[:o, :o].T).max() > 1e-3


@pytest.mark.parametrize("v,X,seed", [(6, 14, 0), (5, 12, 4)])
def test_two_electron_density_equals_fci(v, X, seed):
    """Two electrons: CCSD is exact, so the Lambda density plus the reference equals the
    1-RDM <Psi|q+ p|Psi>/<Psi|Psi> of the exact ground state (every block)."""
    o = 2
    eps, B = make_system(o, v, X, seed=seed, sigma=0.08)
    res = oracle.solve(eps, B, o, max_iter=200, tol=1e-13)
    assert res.converged
    n = o + v
    V = _full_V(B, n)
    lam = solve_lambda(eps, V, o, res.t1, res.t2, tol=1e-13, max_iter=200)
    assert lam.converged
    g = density(res.t1, res.t2, lam.l1, lam.l2)
    g[:o, :o] += np.eye(o)
    # exact ground state in the two-electron sector of the Fock space
    F = sq_brute.Fock(n)
    h = sq_brute.core_h(eps, V, o)
    states = [s for s in range(1 << n) if bin(s).count('1') == 2]
    basis = np.zeros((len(states), 1 << n))
    for k, s in enumerate(states):
        basis[k, s] = 1.0
    H = np.array([[np.vdot(bk, sq_brute.apply_H(F, h, V, bl.astype(np.complex128)))
                   for bl in basis] for bk in basis])
    H0 = np.vdot(basis[states.index(3)], sq_brute.apply_H(F, h, V, basis[states.index(3)]
                                                             .astype(np.complex128)))
    w, U = np.linalg.eigh(H)
    psi = U[:, 0] @ basis
    assert abs((w[0] - H0) - res.energy) < 1e-10
    rho = np.array([[np.vdot(psi, F.ad(q, F.a(p, psi))) for q in range(n)] for p in range(n)])
    rho /= np.vdot(psi, psi)
    np.testing.assert_allclose(g, rho, atol=1e-10, rtol=0)


def test_density_diagonal_is_the_energy_derivative():
    """gamma_pp = dE_CC/d e_p (the Lagrangian is stationary in t and lambda), by central
    differences of two converged amplitude solves per spinor."""
    o, v, X, seed = 4, 8, 20, 6
    eps, B = make_system(o, v, X, seed=seed, sigma=0.1)
    res = oracle.solve(eps, B, o, max_iter=200, tol=1e-13)
    V = _full_V(B, o + v)
    lam = solve_lambda(eps, V, o, res.t1, res.t2, tol=1e-13, max_iter=200)
    assert res.converged and lam.converged
    g = density(res.t1, res.t2, lam.l1, lam.l2)
    d = 1e-4
    for p in (0, o - 1, o, o + v - 1):
        ep, em = eps.copy(), eps.copy()
        ep[p] += d
        em[p] -= d
        Ep = oracle.solve(ep, B, o, max_iter=200, tol=1e-13).energy
        Em = oracle.solve(em, B, o, max_iter=200, tol=1e-13).energy
        assert abs((Ep - Em) / (2 * d) - g[p, p]) < 1e-7


def test_density_trace_is_zero():
    """The correlation density conserves the electron count for any t and lambda."""
    o, v = 5, 9
    t1, t2 = make_amplitudes(o, v, seed=21, scale=0.2)
    l1, l2 = make_amplitudes(o, v, seed=22, scale=0.2)
    assert abs(np.trace(density(t1, t2, l1, l2))) < 1e-13
