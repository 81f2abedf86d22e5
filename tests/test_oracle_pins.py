"""Pins of the CPU oracle against facts that do not come from the oracle itself."""
import numpy as np
import pytest

import oracle
from oracle.ccsd import build_integrals, energy, pack_t2, residual, unpack_t2
from oracle.integrals import antisym
from paper_2103_08473_amd.synth import make_amplitudes, make_system
import sq_brute


# ---------------------------------------------------------------- App. A residual
@pytest.mark.parametrize("o,v,X,seed", [(2, 4, 7, 0), (3, 4, 9, 3), (4, 5, 11, 4), (3, 3, 5, 9)])
def test_residual_equals_second_quantisation(o, v, X, seed):
    """eq. CC_general == <Phi_l| e^-T H e^T |Phi_0> built in the full Fock space (eq. CCSD)."""
    eps, B = make_system(o, v, X, seed=seed, sigma=0.3)
    t1, t2 = make_amplitudes(o, v, seed=seed + 100, scale=0.15)
    ints = build_integrals(B, o)
    S1, S2 = residual(eps, ints, t1, t2)
    E = energy(eps, ints, t1, t2)
    n = o + v
    V = antisym(B, slice(0, n), slice(0, n), slice(0, n), slice(0, n))
    Eb, S1b, S2b = sq_brute.cc_residual(eps, V, o, t1, t2)
    assert np.abs(S2b).max() > 0.1 and np.abs(S1b).max() > 0.01
    assert abs(E - Eb) < 1e-13
    np.testing.assert_allclose(S1, S1b, atol=1e-13, rtol=0)
    np.testing.assert_allclose(S2, S2b, atol=1e-13, rtol=0)


def test_brute_force_detects_planted_sign_error():
    """A residual with one term's sign flipped must fail the brute-force comparison."""
    o, v, X = 3, 4, 9
    eps, B = make_system(o, v, X, seed=3, sigma=0.3)
    t1, t2 = make_amplitudes(o, v, seed=7, scale=0.15)
    ints = build_integrals(B, o)
    S1, S2 = residual(eps, ints, t1, t2)
    bad = dict(ints)
    bad['vovo'] = -ints['vovo']   # planted: wrong sign of <ak||ci>
    S1x, S2x = residual(eps, bad, t1, t2)
    n = o + v
    V = antisym(B, slice(0, n), slice(0, n), slice(0, n), slice(0, n))
    _, S1b, S2b = sq_brute.cc_residual(eps, V, o, t1, t2)
    assert np.abs(S2 - S2b).max() < 1e-13
    assert np.abs(S2x - S2b).max() > 1e-3


# ---------------------------------------------------------------- whole solver = FCI
@pytest.mark.parametrize("v,X,seed,sigma", [(8, 20, 0, 0.05), (14, 30, 1, 0.05), (12, 25, 2, 0.08)])
def test_two_electron_ccsd_equals_fci(v, X, seed, sigma):
    eps, B = make_system(2, v, X, seed=seed, sigma=sigma)
    res = oracle.solve(eps, B, 2, max_iter=80, tol=1e-12)
    assert res.converged
    e_fci, vec, dets = oracle.fci_two_electron(eps, B)
    assert abs(res.energy - e_fci) < 1e-10
    # doubles of the FCI vector in intermediate normalisation equal tau_01^ab
    c0 = vec[dets.index((0, 1))]
    tau = oracle.tau(res.t1, res.t2)
    for a in range(v):
        for b in range(a + 1, v):
            cab = vec[dets.index((2 + a, 2 + b))] / c0
            assert abs(cab - tau[0, 1, a, b]) < 1e-8


@pytest.mark.parametrize("v,X,seed,sigma", [(8, 20, 0, 0.05), (14, 30, 1, 0.05), (12, 25, 2, 0.08)])
def test_two_electron_ccd_equals_cid(v, X, seed, sigma):
    """CCD (T1 = 0) for two electrons is CI over the reference and its doubles."""
    eps, B = make_system(2, v, X, seed=seed, sigma=sigma)
    res = oracle.solve(eps, B, 2, max_iter=80, tol=1e-12, doubles_only=True)
    assert res.converged
    assert np.abs(res.t1).max() == 0
    e_cid, vec, dets = oracle.fci_two_electron(eps, B, doubles_only=True)
    assert abs(res.energy - e_cid) < 1e-10
    c0 = vec[dets.index((0, 1))]
    for a in range(v):
        for b in range(a + 1, v):
            assert abs(vec[dets.index((2 + a, 2 + b))] / c0 - res.t2[0, 1, a, b]) < 1e-8
    # the singles matter: CCSD (= FCI) differs from CCD (= CID) here
    e_fci, _, _ = oracle.fci_two_electron(eps, B)
    assert abs(e_fci - e_cid) > 1e-8


def test_ccd_residual_is_brute_force_projection():
    """The CCD equations are the CCSD doubles equations at t1 = 0: brute-force check."""
    o, v, X = 3, 5, 12
    eps, B = make_system(o, v, X, seed=13, sigma=0.3)
    _, t2 = make_amplitudes(o, v, seed=14, scale=0.1)
    t1 = np.zeros((o, v), dtype=np.complex128)
    _, S2 = residual(eps, build_integrals(B, o), t1, t2)
    n = o + v
    V = antisym(B, slice(0, n), slice(0, n), slice(0, n), slice(0, n))
    _, _, S2b = sq_brute.cc_residual(eps, V, o, t1, t2)
    assert np.abs(S2b).max() > 0.1
    np.testing.assert_allclose(S2, S2b, atol=1e-13, rtol=0)


@pytest.mark.parametrize("o,v,X,seed", [(2, 4, 7, 0), (3, 4, 9, 3), (3, 5, 11, 5)])
def test_cc2_residual_equals_second_quantisation(o, v, X, seed):
    """CC2: singles = <mu1| e^-T H e^T |0> (T = T1 + T2), doubles =
    <mu2| e^-T1 H e^T1 |0> + (e_a + e_b - e_i - e_j) t2, both by brute force."""
    eps, B = make_system(o, v, X, seed=seed, sigma=0.3)
    t1, t2 = make_amplitudes(o, v, seed=seed + 200, scale=0.15)
    S1, S2 = oracle.cc2_residual(eps, build_integrals(B, o), t1, t2)
    n = o + v
    V = antisym(B, slice(0, n), slice(0, n), slice(0, n), slice(0, n))
    _, S1b, _ = sq_brute.cc_residual(eps, V, o, t1, t2)
    _, _, S2t1 = sq_brute.cc_residual(eps, V, o, t1, np.zeros_like(t2))
    eo, ev = eps[:o], eps[o:]
    D2 = ev[None, None, :, None] + ev[None, None, None, :] - eo[:, None, None, None] - eo[None, :, None, None]
    assert np.abs(S2t1).max() > 0.05
    np.testing.assert_allclose(S1, S1b, atol=1e-13, rtol=0)
    np.testing.assert_allclose(S2, S2t1 + D2 * t2, atol=1e-13, rtol=0)
    # and CC2 is not CCSD: the T2-quadratic and T1-T2 doubles terms are missing
    _, S2ccsd = residual(eps, build_integrals(B, o), t1, t2)
    assert np.abs(S2ccsd - S2).max() > 1e-3


def test_cc2_solve_converges_between_mp2_and_ccsd_scale():
    """A converged CC2 solve: residual below tol, and its energy differs from CCSD's."""
    o, v, X = 4, 16, 40
    eps, B = make_system(o, v, X, seed=21)
    r2 = oracle.solve(eps, B, o, max_iter=80, tol=1e-11, cc2=True)
    rs = oracle.solve(eps, B, o, max_iter=80, tol=1e-11)
    assert r2.converged and rs.converged
    S1, S2 = oracle.cc2_residual(eps, build_integrals(B, o), r2.t1, r2.t2)
    assert max(np.abs(S1).max(), np.abs(S2).max()) < 1e-9
    assert abs(r2.energy - rs.energy) > 1e-6


def test_one_electron_degenerate_case():
    """nocc = 1: no doubles; canonical spinors make the reference exact (E = FCI = 0)."""
    eps, B = make_system(1, 9, 20, seed=4, sigma=0.1)
    res = oracle.solve(eps, B, 1, max_iter=5, tol=1e-14)
    assert res.converged and res.iterations == 1
    assert res.energy == 0
    assert abs(oracle.fci_one_electron(eps, B)) < 1e-14


# ---------------------------------------------------------------- MP2 start
@pytest.mark.parametrize("o,v,X", [(4, 12, 30), (10, 40, 120)])
def test_first_iteration_is_mp2(o, v, X):
    eps, B = make_system(o, v, X, seed=11)
    e1 = oracle.mp2_energy_iterative(eps, B, o)
    # closed form E_MP2 = 1/4 sum |<ij||ab>|^2 / (e_i + e_j - e_a - e_b), integrals from B directly
    Bov = B[:, :o, o:]
    coul = np.einsum('Pia,Pjb->ijab', Bov, Bov)
    g = coul - coul.transpose(0, 1, 3, 2)
    D = (eps[:o, None, None, None] + eps[None, :o, None, None]
         - eps[None, None, o:, None] - eps[None, None, None, o:])
    emp2 = 0.25 * np.sum(np.abs(g) ** 2 / D)
    assert abs(e1.imag) < 1e-14
    assert abs(e1 - emp2) < 1e-12 * abs(emp2)


# ---------------------------------------------------------------- symmetries
def test_integral_symmetries():
    o, v, X = 3, 5, 8
    eps, B = make_system(o, v, X, seed=2, sigma=0.2)
    n = o + v
    s = slice(0, n)
    V = antisym(B, s, s, s, s)
    assert np.abs(V + V.transpose(1, 0, 2, 3)).max() < 1e-15
    assert np.abs(V + V.transpose(0, 1, 3, 2)).max() < 1e-15
    assert np.abs(V.conj() - V.transpose(2, 3, 0, 1)).max() < 1e-15


def test_amplitudes_antisymmetric_and_pack_roundtrip():
    o, v, X = 5, 12, 30
    eps, B = make_system(o, v, X, seed=6)
    res = oracle.solve(eps, B, o, max_iter=4, tol=0.0)
    t2 = res.t2
    assert np.abs(t2 + t2.transpose(1, 0, 2, 3)).max() == 0
    assert np.abs(t2 + t2.transpose(0, 1, 3, 2)).max() == 0
    assert np.array_equal(unpack_t2(pack_t2(t2), o, v), t2)


def test_orbital_phase_invariance():
    """p -> e^{i theta_p} p leaves E unchanged and rotates t by the phase factors."""
    o, v, X = 4, 10, 24
    eps, B = make_system(o, v, X, seed=8)
    th = np.random.default_rng(1).uniform(0, 2 * np.pi, o + v)
    ph = np.exp(1j * th)
    B2 = ph.conj()[None, :, None] * B * ph[None, None, :]
    r1 = oracle.solve(eps, B, o, max_iter=100, tol=1e-11)
    r2 = oracle.solve(eps, B2, o, max_iter=100, tol=1e-11)
    assert r1.converged and r2.converged
    assert abs(r1.energy - r2.energy) < 1e-10
    po, pv = ph[:o], ph[o:]
    fac = (pv.conj()[None, None, :, None] * pv.conj()[None, None, None, :]
           * po[:, None, None, None] * po[None, :, None, None])
    np.testing.assert_allclose(r2.t2, r1.t2 * fac, atol=1e-8)


def test_real_factors_give_real_results():
    o, v, X = 4, 10, 24
    eps, B = make_system(o, v, X, seed=5)
    Br = B.real.astype(np.complex128)
    Br = 0.5 * (Br + Br.transpose(0, 2, 1))
    r = oracle.solve(eps, Br, o, max_iter=30, tol=1e-11)
    assert r.converged
    assert abs(r.energy.imag) < 1e-14
    assert np.abs(r.t2.imag).max() < 1e-14 and np.abs(r.t1.imag).max() < 1e-14


def test_diis_and_jacobi_reach_same_fixed_point():
    o, v, X = 4, 10, 24
    eps, B = make_system(o, v, X, seed=9, sigma=0.02)
    rj = oracle.solve(eps, B, o, max_iter=200, tol=1e-12, diis_size=0)
    rd = oracle.solve(eps, B, o, max_iter=60, tol=1e-12, diis_size=8)
    assert rj.converged and rd.converged
    assert rd.iterations < rj.iterations
    assert abs(rj.energy - rd.energy) < 1e-11


def test_level_shift_same_fixed_point():
    o, v, X = 4, 10, 24
    eps, B = make_system(o, v, X, seed=9, sigma=0.02)
    r0 = oracle.solve(eps, B, o, max_iter=80, tol=1e-12)
    r1 = oracle.solve(eps, B, o, max_iter=120, tol=1e-12, level_shift=0.3)
    assert r0.converged and r1.converged
    assert abs(r0.energy - r1.energy) < 1e-11
