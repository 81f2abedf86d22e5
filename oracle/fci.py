"""Brute-force full CI for one and two electrons (oracle pin; test infrastructure).

CCSD is exact for at most two electrons, so the converged CCSD correlation
energy must equal E_FCI - E_ref.  The Hamiltonian is the paper's
second-quantised no-virtual-pair operator (eq. Hamiltonian),
H = sum h_pq p+ q + 1/4 sum <pq||rs> p+ q+ s r, with the core Hamiltonian
h chosen so that the Fock matrix of the reference |0 .. o-1> is diag(eps):
h_pq = eps_p delta_pq - sum_k <pk||qk>.

The reported root is the eigenvector with the largest overlap with the
reference determinant.
"""
import numpy as np
import scipy.linalg

from .integrals import antisym


def _core_h(eps, B, nocc):
    n = eps.size
    allp = slice(0, n)
    occ = slice(0, nocc)
    pkqk = antisym(B, allp, occ, allp, occ)          # <pk||qk>[p,k,q,k']
    h = np.diag(eps).astype(np.complex128)
    for k in range(nocc):
        h -= pkqk[:, k, :, k]
    return h


def fci_two_electron(eps, B, doubles_only=False):
    """Correlation energy of the 2-electron FCI ground state (reference |01>).

    doubles_only: CI in the space of the reference and its double excitations
    |ab> (a, b >= 2) only (CID).  For two electrons CCD is exactly this: T2^2
    cannot act on the reference, so the CCD doubles equations are the CID
    eigenproblem in intermediate normalisation.
    """
    n = eps.size
    h = _core_h(eps, B, 2)
    allp = slice(0, n)
    V = antisym(B, allp, allp, allp, allp)
    dets = [(p, q) for p in range(n) for q in range(p + 1, n)]
    if doubles_only:
        dets = [(p, q) for (p, q) in dets if (p, q) == (0, 1) or p >= 2]
    m = len(dets)
    H = np.zeros((m, m), dtype=np.complex128)
    for I, (p, q) in enumerate(dets):
        for J, (r, s) in enumerate(dets):
            val = V[p, q, r, s]
            if q == s:
                val += h[p, r]
            if p == r:
                val += h[q, s]
            if q == r:
                val -= h[p, s]
            if p == s:
                val -= h[q, r]
            H[I, J] = val
    w, U = scipy.linalg.eigh(H)
    ref = dets.index((0, 1))
    root = int(np.argmax(np.abs(U[ref, :])))
    e_ref = H[ref, ref].real
    return float(w[root] - e_ref), U[:, root], dets


def fci_one_electron(eps, B):
    """Correlation energy of 1 electron in n spinors (reference spinor 0)."""
    h = _core_h(eps, B, 1)
    w, U = scipy.linalg.eigh(h)
    root = int(np.argmax(np.abs(U[0, :])))
    return float(w[root] - h[0, 0].real)
