"""Brute-force second quantisation in the full Fock space (test helper).

Independent of the oracle's working equations: it builds the states
e^T |Phi_0>, H e^T |Phi_0> and e^-T H e^T |Phi_0> as vectors over all 2^n
occupation bitstrings, applying creation/annihilation operators with the
Jordan-Wigner sign, and projects on |Phi_i^a> = a+_a a_i |Phi_0> and
|Phi_ij^ab> = a+_a a+_b a_j a_i |Phi_0>.  This is the definition of the CC
residual in the paper's eq. CCSD, with H the second-quantised operator of
eq. Hamiltonian and T1, T2 of eq. t_amp read with the standard 1/4 and
a_j a_i order.
"""
import numpy as np


class Fock:
    def __init__(self, n):
        self.n = n
        dim = 1 << n
        idx = np.arange(dim)
        self.ann = []
        self.cre = []
        for p in range(n):
            below = idx & ((1 << p) - 1)
            sign = np.where(np.array([bin(x).count('1') for x in below]) % 2 == 0, 1.0, -1.0)
            occ = (idx >> p) & 1
            src_a = idx[occ == 1]
            self.ann.append((src_a, src_a ^ (1 << p), sign[occ == 1]))
            src_c = idx[occ == 0]
            self.cre.append((src_c, src_c | (1 << p), sign[occ == 0]))

    @staticmethod
    def _apply(op, psi):
        src, dst, sg = op
        out = np.zeros_like(psi)
        out[dst] = sg * psi[src]
        return out

    def a(self, p, psi):
        return self._apply(self.ann[p], psi)

    def ad(self, p, psi):
        return self._apply(self.cre[p], psi)


def core_h(eps, V, nocc):
    h = np.diag(eps).astype(np.complex128)
    for k in range(nocc):
        h -= V[:, k, :, k]
    return h


def apply_H(F, h, V, psi):
    n = F.n
    out = np.zeros_like(psi)
    for q in range(n):
        aq = F.a(q, psi)
        if not aq.any():
            continue
        for p in range(n):
            if h[p, q] != 0:
                out += h[p, q] * F.ad(p, aq)
    for r in range(n):
        ar = F.a(r, psi)
        for s in range(r + 1, n):
            asr = F.a(s, ar)            # a_s a_r psi
            if not asr.any():
                continue
            for p in range(n):
                for q in range(p + 1, n):
                    c = V[p, q, r, s]
                    if c != 0:
                        out += c * F.ad(p, F.ad(q, asr))
    return out


def apply_T(F, o, t1, t2, psi):
    v = t1.shape[1]
    out = np.zeros_like(psi)
    for i in range(o):
        ai = F.a(i, psi)
        if not ai.any():
            continue
        for a in range(v):
            out += t1[i, a] * F.ad(o + a, ai)
        for j in range(i + 1, o):
            aji = F.a(j, ai)            # a_j a_i psi
            if not aji.any():
                continue
            for a in range(v):
                for b in range(a + 1, v):
                    out += t2[i, j, a, b] * F.ad(o + a, F.ad(o + b, aji))
    return out


def exp_T(F, o, t1, t2, psi, sign=1.0):
    out = psi.copy()
    term = psi.copy()
    for k in range(1, o + 2):
        term = apply_T(F, o, sign * t1, sign * t2, term) / k
        out += term
    return out


def cc_residual(eps, V, nocc, t1, t2):
    """Return (E_corr, S1[i,a], S2[i,j,a,b]) = projections of e^-T H e^T |Phi_0>."""
    n = eps.size
    o = nocc
    v = n - o
    F = Fock(n)
    h = core_h(eps, V, o)
    phi0 = np.zeros(1 << n, dtype=np.complex128)
    phi0[(1 << o) - 1] = 1.0
    e_ref = np.vdot(phi0, apply_H(F, h, V, phi0))
    chi = exp_T(F, o, t1, t2, phi0)
    chi = apply_H(F, h, V, chi)
    chi = exp_T(F, o, t1, t2, chi, sign=-1.0)
    S1 = np.zeros((o, v), dtype=np.complex128)
    S2 = np.zeros((o, o, v, v), dtype=np.complex128)
    for i in range(o):
        ai = F.a(i, phi0)
        for a in range(v):
            basis = F.ad(o + a, ai)
            S1[i, a] = np.vdot(basis, chi)
        for j in range(o):
            if j == i:
                continue
            aji = F.a(j, ai)
            for a in range(v):
                for b in range(v):
                    if a == b:
                        continue
                    basis = F.ad(o + a, F.ad(o + b, aji))
                    S2[i, j, a, b] = np.vdot(basis, chi)
    return complex(np.vdot(phi0, chi) - e_ref), S1, S2


# ---------------------------------------------------------------- CC Lagrangian
def _tau_mu(F, o, mu, psi):
    """tau_mu psi for mu = (i, a) (a+_a a_i) or (i, j, a, b) (a+_a a+_b a_j a_i)."""
    if len(mu) == 2:
        i, a = mu
        return F.ad(o + a, F.a(i, psi))
    i, j, a, b = mu
    return F.ad(o + a, F.ad(o + b, F.a(j, F.a(i, psi))))


def _excitations(o, v):
    singles = [(i, a) for i in range(o) for a in range(v)]
    doubles = [(i, j, a, b) for i in range(o) for j in range(i + 1, o)
               for a in range(v) for b in range(a + 1, v)]
    return singles, doubles


def lagrangian_bra(F, o, l1, l2):
    """The bra <0|(1 + Lambda) as a vector L with <L|psi> = L . psi (no conjugation):
    <0| i+ a = <Phi_i^a| and <0| i+ j+ b a = <Phi_ij^ab|, with lambda as coefficients."""
    v = l1.shape[1]
    phi0 = np.zeros(1 << F.n, dtype=np.complex128)
    phi0[(1 << o) - 1] = 1.0
    L = phi0.copy()
    singles, doubles = _excitations(o, v)
    for mu in singles:
        L += l1[mu] * _tau_mu(F, o, mu, phi0)
    for mu in doubles:
        L += l2[mu] * _tau_mu(F, o, mu, phi0)
    return phi0, L


def lagrangian_gradient(eps, V, nocc, t1, t2, l1, l2):
    """dL/dt_mu = <0|(1+Lambda) e^-T [H, tau_mu] e^T|0> for every single and double
    (L = <0|(1+Lambda) e^-T H e^T|0>, holomorphic in t), as (G1[i,a], G2[i,j,a,b])."""
    n = eps.size
    o = nocc
    v = n - o
    F = Fock(n)
    h = core_h(eps, V, o)
    phi0, L = lagrangian_bra(F, o, l1, l2)

    def hbar(psi):
        chi = exp_T(F, o, t1, t2, psi)
        chi = apply_H(F, h, V, chi)
        return exp_T(F, o, t1, t2, chi, sign=-1.0)

    hb0 = hbar(phi0)
    G1 = np.zeros((o, v), dtype=np.complex128)
    G2 = np.zeros((o, o, v, v), dtype=np.complex128)
    singles, doubles = _excitations(o, v)
    for mu in singles + doubles:
        val = np.dot(L, hbar(_tau_mu(F, o, mu, phi0))) - np.dot(L, _tau_mu(F, o, mu, hb0))
        if len(mu) == 2:
            G1[mu] = val
        else:
            i, j, a, b = mu
            G2[i, j, a, b] = val
            G2[j, i, a, b] = -val
            G2[i, j, b, a] = -val
            G2[j, i, b, a] = val
    return G1, G2


def lagrangian_density(nocc, t1, t2, l1, l2):
    """gamma[p, q] = <0|(1+Lambda) e^-T {q+ p} e^T|0>: the element <q+ p>, minus the
    reference's delta_pq for occupied p (normal order)."""
    o, v = t1.shape
    n = o + v
    F = Fock(n)
    phi0, L = lagrangian_bra(F, o, l1, l2)
    chi = exp_T(F, o, t1, t2, phi0)
    g = np.zeros((n, n), dtype=np.complex128)
    for p in range(n):
        ap = F.a(p, chi)
        for q in range(n):
            g[p, q] = np.dot(L, exp_T(F, o, t1, t2, F.ad(q, ap), sign=-1.0))
    g[:o, :o] -= np.eye(o)
    return g
