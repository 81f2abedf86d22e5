"""Selected entries of the CCSD residual at large sizes (oracle; test infrastructure).

Evaluates S2[i,j,a,b] and S1[i,a] of eq. CC_general (Appendix A) one entry at
a time, without any array larger than o^2 v^2: the needed intermediates are
formed only for the index values an entry touches.  Integrals with three or
four virtual indices are contracted through the density-fitting factors,
(pq|rs) = sum_P B[P,p,q] B[P,r,s], evaluated in the order the sums are
written (first over P, then over the remaining index) only where forming the
integral block itself would need O(v^3) memory per entry.

Pinned against oracle.ccsd.residual on every entry at small sizes
(tests/test_oracle_elements.py); used for full-size GPU parity on samples.
"""
from __future__ import annotations

import numpy as np

from .ccsd import tau as make_tau
from .integrals import antisym


def _ein(s, *a):
    return np.einsum(s, *a, optimize=True)


class ResidualElements:
    """Shared pieces for one (eps, B, t1, t2); entries computed on demand."""

    def __init__(self, eps, B, nocc, t1, t2):
        self.eps, self.B, self.o = eps, B, nocc
        o = nocc
        n = B.shape[1]
        self.v = v = n - o
        O, Vs = slice(0, o), slice(o, n)
        self.Bov = B[:, O, Vs]          # B^P_kd   [P, k, d]
        self.Boo = B[:, O, O]           # B^P_ki
        self.Bvv = B[:, Vs, Vs]         # B^P_ac
        self.Bvo = B[:, Vs, O]          # B^P_ak
        self.t1, self.t2 = t1, t2
        self.tau = make_tau(t1, t2)
        self.Voovv = antisym(B, O, O, Vs, Vs)   # <kl||cd>
        self.Vooov = antisym(B, O, O, O, Vs)    # <kl||ic>
        self.Voooo = antisym(B, O, O, O, O)     # <kl||ij>
        e_o, e_v = eps[:o], eps[o:]
        fo = np.diag(e_o).astype(np.complex128)
        fv = np.diag(e_v).astype(np.complex128)
        tau_ = self.tau
        # one-body intermediates (App. A), f_kc = 0
        self.Hac = fv + 0.5 * _ein('klcd,klda->ac', self.Voovv, tau_)
        # sum_kd <ak||cd> t_k^d = sum_kd (ac|kd) t_k^d - sum_kd (ad|kc) t_k^d
        y = _ein('Pkd,kd->P', self.Bov, t1)
        Z = _ein('kd,Pkc->Pdc', t1, self.Bov)
        self.Gac = self.Hac + _ein('Pac,P->ac', self.Bvv, y) - _ein('Pad,Pdc->ac', self.Bvv, Z)
        self.Hki = -fo + 0.5 * _ein('klcd,licd->ki', self.Voovv, tau_)
        self.Gki = self.Hki - _ein('klic,lc->ki', self.Vooov, t1)
        self.Hkc = _ein('klcd,ld->kc', self.Voovv, t1)
        # U^P_{k i} = sum_d B^P_kd t_i^d (used by the t1 part of H^{ak}_{ci})
        self.U = _ein('Pkd,id->Pki', self.Bov, t1)
        self._H = {}
        self._C = {}
        self._A = {}
        self._Y = {}

    # <ak||ci> for fixed a, i as [k, c]:  (ac|ki) - (ai|kc)
    def _vovo_ai(self, a, i):
        return (_ein('Pc,Pk->kc', self.Bvv[:, a, :], self.Boo[:, :, i])
                - _ein('P,Pkc->kc', self.Bvo[:, a, i], self.Bov))

    def H_ai(self, a, i):
        """H^{ak}_{ci} for fixed a, i as [k, c]."""
        key = (a, i)
        if key not in self._H:
            t1, t2 = self.t1, self.t2
            h = self._vovo_ai(a, i)
            # sum_d <ak||cd> t_i^d = sum_d (ac|kd) t_i^d - sum_d (ad|kc) t_i^d
            h += _ein('Pc,Pk->kc', self.Bvv[:, a, :], self.U[:, :, i])
            h -= _ein('P,Pkc->kc', _ein('Pd,d->P', self.Bvv[:, a, :], t1[i]), self.Bov)
            h -= _ein('klc,l->kc', self.Vooov[:, :, i, :], t1[:, a])
            X = 0.5 * t2[:, i, a, :] + np.outer(t1[:, a], t1[i, :])   # [l, d]
            h += _ein('klcd,ld->kc', self.Voovv, X)
            self._H[key] = h
        return self._H[key]

    def C_aij(self, a, i, j):
        """C^{ka}_{ij} for fixed a, i, j as [k]."""
        key = (a, i, j)
        if key not in self._C:
            t1 = self.t1
            c = np.conj(self.Vooov[i, j, :, a])                     # V^{ij dagger}_{ka}
            c = c + self._vovo_ai(a, i) @ t1[j] - self._vovo_ai(a, j) @ t1[i]
            # -1/2 sum_cd <ak||cd> tau_ij^cd = -sum_cd (ac|kd) tau_ij^cd
            if (i, j) not in self._Y:
                self._Y[(i, j)] = _ein('Pkd,cd->Pkc', self.Bov, self.tau[i, j])
            c = c - _ein('Pc,Pkc->k', self.Bvv[:, a, :], self._Y[(i, j)])
            self._C[key] = c
        return self._C[key]

    def A_ij(self, i, j):
        """A^{kl}_{ij} for fixed i, j as [k, l]."""
        key = (i, j)
        if key not in self._A:
            t1 = self.t1
            A = (self.Voooo[:, :, i, j]
                 + self.Vooov[:, :, i, :] @ t1[j] - self.Vooov[:, :, j, :] @ t1[i]
                 + 0.5 * _ein('klcd,cd->kl', self.Voovv, self.tau[i, j]))
            self._A[key] = A
        return self._A[key]

    def S2(self, i, j, a, b):
        t1, t2, tau_ = self.t1, self.t2, self.tau

        def ring(a_, i_, j_, b_):
            return np.sum(self.H_ai(a_, i_) * t2[j_, :, :, b_])    # sum_kc H_akci t_jk^cb

        s = ring(a, i, j, b) - ring(a, j, i, b) - ring(b, i, j, a) + ring(b, j, i, a)
        s += self.Gki[:, j] @ t2[i, :, a, b] - self.Gki[:, i] @ t2[j, :, a, b]

        def vt(i_, j_):   # sum_c <ab||cj> t_i^c,  <ab||cj> = (ac|bj) - (aj|bc)
            acbj = _ein('Pc,P->c', self.Bvv[:, a, :], self.Bvo[:, b, j_])
            ajbc = _ein('P,Pc->c', self.Bvo[:, a, j_], self.Bvv[:, b, :])
            return (acbj - ajbc) @ t1[i_]

        s += vt(i, j) - vt(j, i)
        s += self.Gac[a] @ t2[i, j, :, b] - self.Gac[b] @ t2[i, j, :, a]
        s += self.C_aij(a, i, j) @ t1[:, b] - self.C_aij(b, i, j) @ t1[:, a]
        s += 0.5 * np.sum(self.A_ij(i, j) * tau_[:, :, a, b])
        # 1/2 sum_cd <ab||cd> tau_ij^cd, <ab||cd> = (ac|bd) - (ad|bc)
        acbd = _ein('Pc,Pd->cd', self.Bvv[:, a, :], self.Bvv[:, b, :])
        adbc = _ein('Pd,Pc->cd', self.Bvv[:, a, :], self.Bvv[:, b, :])
        s += 0.5 * np.sum((acbd - adbc) * tau_[i, j])
        s += np.conj(self.Voovv[i, j, a, b])
        return complex(s)

    def S1(self, i, a):
        t1, t2, tau_ = self.t1, self.t2, self.tau
        s = self.Hac[a] @ t1[i] + self.Hki[:, i] @ t1[:, a] + np.sum(self.Hkc * t2[i, :, a, :])
        s += (self.Hkc @ t1[i]) @ t1[:, a]
        # 1/2 sum_kcd <ak||cd> tau_ik^cd = sum_kcd (ac|kd) tau_ik^cd
        Y = _ein('Pkd,kcd->Pc', self.Bov, tau_[i])
        s += np.sum(self.Bvv[:, a, :] * Y)
        s += 0.5 * np.sum(self.Vooov[:, :, i, :] * tau_[:, :, :, a])
        # - sum_kc <ak||ci> t_k^c
        s -= np.sum(self._vovo_ai(a, i) * t1)
        return complex(s)

    def energy(self):
        return complex(0.25 * np.sum(self.Voovv * self.tau))
