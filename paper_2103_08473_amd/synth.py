"""Seeded synthetic CCSD inputs: spinor energies and complex density-fitting factors.

This module only draws random numbers; it holds none of the coupled-cluster
arithmetic.  Both the CPU oracle (through the tests and the benchmark) and the
HIP path receive the arrays it returns.

The recipe stands in for the molecular spinors the paper obtains from DIRAC or
ReSpect (section "Molecular spinors: interface to DIRAC and ReSpect"): an active
space of ``nocc`` occupied and ``nvir`` virtual spinors with diagonal Fock
matrix f = diag(eps), and two-electron integrals given in factorised form
(pq|rs) = sum_P B[P,p,q] B[P,r,s] with every B[P] Hermitian, so that the
antisymmetrised integrals <pq||rs> = (pr|qs) - (ps|qr) have the permutational
and Hermitian symmetry of the paper's complex V tensor (eq. two_electron).

Draw order (one ``numpy.random.default_rng(seed)`` stream):
  1. eps_occ ~ U[-2, -0.5]  (nocc values)
  2. eps_vir ~ U[0.2, 3]    (nvir values)
  3. for P = 0 .. naux-1:  Re ~ N(0, sigma^2) (n x n), Im ~ N(0, sigma^2) (n x n),
     A = Re + i Im,  B[P] = (A + A^H) / 2
so E|B[P,p,q]|^2 = sigma^2 for every p, q (real diagonal, circular off-diagonal).

``sigma=None`` selects the size-scaled width
sigma_B = min(0.05, sigma_s), sigma_s^2 = 0.05^2 * (40 * sqrt(10 * 120)) / (nvir * sqrt(nocc * naux)),
and sigma_s equals 0.05 exactly at (nocc, nvir, naux) = (10, 40, 120).  It holds
nocc * nvir^2 * naux * sigma^4, the size of the coherent one-body dressing
terms (sums of <kl||cd> tau over nocc^2 nvir or nocc nvir^2 entries) at or
below its (10, 40, 120) value; the spread of the particle-particle ladder operator,
~ 2 * nvir * sqrt(2 naux) * sigma^2, then shrinks as 1/sqrt(nocc / 10).
Passing ``sigma=0.05`` gives the literal distribution at every size.
"""
from __future__ import annotations

import math

import numpy as np

SIGMA_LITERAL = 0.05
_REF_NOCC, _REF_NVIR, _REF_NAUX = 10, 40, 120


def scaled_sigma(nocc: int, nvir: int, naux: int) -> float:
    """The literal 0.05, reduced where it would exceed the width that keeps
    nocc * nvir^2 * naux * sigma^4 at its (10, 40, 120, 0.05) value."""
    s2 = SIGMA_LITERAL ** 2 * (_REF_NVIR * math.sqrt(_REF_NOCC * _REF_NAUX)) / (
        nvir * math.sqrt(nocc * naux))
    return min(SIGMA_LITERAL, math.sqrt(s2))


def make_system(nocc: int, nvir: int, naux: int, seed: int = 0, sigma: float | None = None):
    """Return (eps[n] float64, B[naux, n, n] complex128), occupied spinors first."""
    if nocc < 1 or nvir < 1 or naux < 1:
        raise ValueError("nocc, nvir and naux must be >= 1")
    if sigma is None:
        sigma = scaled_sigma(nocc, nvir, naux)
    n = nocc + nvir
    rng = np.random.default_rng(seed)
    eps_occ = rng.uniform(-2.0, -0.5, nocc)
    eps_vir = rng.uniform(0.2, 3.0, nvir)
    eps = np.concatenate([eps_occ, eps_vir])
    B = np.empty((naux, n, n), dtype=np.complex128)
    for P in range(naux):
        re = rng.normal(0.0, sigma, (n, n))
        im = rng.normal(0.0, sigma, (n, n))
        A = re + 1j * im
        B[P] = 0.5 * (A + A.conj().T)
    return eps, B


def make_amplitudes(nocc: int, nvir: int, seed: int, scale: float = 0.05):
    """Random complex amplitudes with the antisymmetry of the cluster operator.

    t1[i, a] ~ scale * (N + iN);  t2[i, j, a, b] = -t2[j, i, a, b] = -t2[i, j, b, a]
    drawn on the unique i<j, a<b entries (diagonals zero).  Used to feed the
    same amplitudes to the oracle and to the GPU residual.
    """
    rng = np.random.default_rng(seed)
    t1 = scale * (rng.normal(size=(nocc, nvir)) + 1j * rng.normal(size=(nocc, nvir)))
    raw = scale * (rng.normal(size=(nocc, nocc, nvir, nvir))
                   + 1j * rng.normal(size=(nocc, nocc, nvir, nvir)))
    iu = np.triu(np.ones((nocc, nocc), dtype=bool), 1)
    au = np.triu(np.ones((nvir, nvir), dtype=bool), 1)
    mask = iu[:, :, None, None] & au[None, None, :, :]
    t2 = np.where(mask, raw, 0.0)
    t2 = t2 - t2.transpose(1, 0, 2, 3)
    t2 = t2 - t2.transpose(0, 1, 3, 2)
    return t1, t2


def serving_request(k: int):
    """Shape of serving request k: nocc ~ U{6..40}, nvir = round(r*nocc) with
    r ~ U[5, 9], naux = 3*nvir, seed 1000+k."""
    rng = np.random.default_rng(7_000_000 + k)
    nocc = int(rng.integers(6, 41))
    r = float(rng.uniform(5.0, 9.0))
    nvir = int(round(r * nocc))
    return nocc, nvir, 3 * nvir, 1000 + k


def make_df_inputs(nao: int, nspinor: int, naux: int, seed: int = 0, sigma: float = 0.1):
    """Inputs of DF-factor generation: AO three-index integrals J[Q][mu][nu] (complex,
    Hermitian in mu nu), the fitting metric V[Q][R] (real, symmetric positive definite)
    and orthonormal spinor coefficients C[mu][p] (complex, nspinor <= nao).

    J and V come from an underlying factorisation: K[P][mu][nu] ~ N(0, sigma^2)
    (Hermitian), L = I + (strictly lower, N(0, (0.3 / sqrt(naux))^2)), J = L K
    (J[Q] = sum_P L[Q][P] K[P]) and V = L L^T, so that J V^-1 J = K K exactly (the
    fitted integrals have a known closed form).  C: the first nspinor columns of the
    unitary factor of a complex Gaussian matrix.  Returns (C, J, V, K)."""
    if nspinor > nao:
        raise ValueError("nspinor > nao")
    rng = np.random.default_rng(seed)
    K = rng.normal(0.0, sigma, (naux, nao, nao)) + 1j * rng.normal(0.0, sigma, (naux, nao, nao))
    K = 0.5 * (K + np.conj(K.transpose(0, 2, 1)))
    L = np.eye(naux) + np.tril(rng.normal(0.0, 0.3 / math.sqrt(naux), (naux, naux)), -1)
    J = np.einsum("QP,Pmn->Qmn", L, K)
    V = L @ L.T
    G = rng.normal(size=(nao, nao)) + 1j * rng.normal(size=(nao, nao))
    Q, _ = np.linalg.qr(G)
    C = np.ascontiguousarray(Q[:, :nspinor])
    return C, np.ascontiguousarray(J), np.ascontiguousarray(V), K
