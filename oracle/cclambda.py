"""CCSD Lambda equations (App. D) and the Lagrangian one-body density (App. E).

Oracle; test infrastructure.  Plain numpy over full spinor-integral blocks:
small systems only.

Index convention as in ccsd.py: l1[i, a] = lambda_a^i, l2[i, j, a, b] =
lambda_ab^ij (antisymmetric in ij and ab), with
Lambda = sum l1 {i+ a} + 1/4 sum l2 {i+ j+ b a}; V[p, q, r, s] = <pq||rs>.

The CC Lagrangian is L(t, lambda) = <0| (1 + Lambda) e^-T H e^T |0>; at converged
amplitudes the Lambda equations are dL/dt = 0, linear in lambda.  App. D prints
the two residual equations and four of their intermediates and defers the rest to
the standard spin-orbital similarity-transformed Hamiltonian elements.  Readings
(each pinned in tests/test_oracle_lambda.py against dL/dt built by brute-force
second quantisation, not against this module):

* The intermediates are the one- and two-body elements of e^-T H e^T: F (ov, oo,
  vv), W (oooo, vvvv, ovvo, ooov, vovv, ovoo, vvvo), each a function of the
  converged t only.  App. D's W^{ij}_{mn}, W^{mb}_{ej}, W^{ef}_{am} and F^e_a are
  the oooo, ovvo, vvvo and vv elements written out.
* G^e_a (vv) and G^i_m (oo) are the two lambda-t2 contractions App. D prints.
* Complex spinors change nothing: L is holomorphic in t and lambda (no complex
  conjugation anywhere), the integrals enter with the index order printed.
* Update: lambda <- lambda - R / D with the same denominators as t (the diagonal
  Fock part of R is D lambda); DIIS as for the amplitudes.
* Density (App. E): gamma[p, q] = <0|(1 + Lambda) e^-T {q+ p} e^T|0> for the ov, vo
  and vv blocks as printed.  The printed oo block is the transpose of that
  element ({i+ j} rather than {j+ i}); this module returns the consistent matrix
  gamma[p, q] = <{q+ p}>, whose oo block is gamma_ji of the printed formula.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .ccsd import DIIS, P, denominators, from_vector, tau, to_vector


def _ein(s, *a):
    return np.einsum(s, *a, optimize=True)


def hbar(eps, V, nocc, t1, t2):
    """One- and two-body elements of e^-T H e^T at amplitudes t (f = diag(eps))."""
    o = nocc
    n = eps.size
    O, Vs = slice(0, o), slice(o, n)
    fo = np.diag(eps[:o]).astype(np.complex128)
    fv = np.diag(eps[o:]).astype(np.complex128)
    fov = np.zeros((o, n - o), dtype=np.complex128)   # zero for canonical spinors
    v_oooo, v_ooov, v_oovv = V[O, O, O, O], V[O, O, O, Vs], V[O, O, Vs, Vs]
    v_ovvo, v_ovvv, v_vovv = V[O, Vs, Vs, O], V[O, Vs, Vs, Vs], V[Vs, O, Vs, Vs]
    v_vvvv, v_ovoo, v_vvvo = V[Vs, Vs, Vs, Vs], V[O, Vs, O, O], V[Vs, Vs, Vs, O]
    v_oovo = V[O, O, Vs, O]
    tt = tau(t1, t2)
    h = {}
    h['ov'] = fov + _ein('nf,mnef->me', t1, v_oovv)
    h['vv'] = (fv - _ein('ma,me->ae', t1, h['ov']) + _ein('mf,amef->ae', t1, v_vovv)
               - 0.5 * _ein('mnaf,mnef->ae', t2, v_oovv))
    h['oo'] = (fo + _ein('ie,me->mi', t1, fov) + _ein('ne,mnie->mi', t1, v_ooov)
               + 0.5 * _ein('inef,mnef->mi', tt, v_oovv))
    h['oooo'] = (v_oooo + P(_ein('je,mnie->mnij', t1, v_ooov), 2, 3)
                 + 0.5 * _ein('ijef,mnef->mnij', tt, v_oovv))
    h['vvvv'] = (v_vvvv - P(_ein('mb,amef->abef', t1, v_vovv), 0, 1)
                 + 0.5 * _ein('mnab,mnef->abef', tt, v_oovv))
    h['ovvo'] = (v_ovvo + _ein('jf,mbef->mbej', t1, v_ovvv) - _ein('nb,mnej->mbej', t1, v_oovo)
                 - _ein('jnfb,mnef->mbej', t2 + _ein('jf,nb->jnfb', t1, t1), v_oovv))
    h['ooov'] = v_ooov + _ein('if,mnfe->mnie', t1, v_oovv)
    h['vovv'] = v_vovv - _ein('na,nmef->amef', t1, v_oovv)
    h['ovoo'] = (v_ovoo - _ein('me,ijbe->mbij', h['ov'], t2) - _ein('nb,mnij->mbij', t1, h['oooo'])
                 + 0.5 * _ein('mbef,ijef->mbij', v_ovvv, tt)
                 + P(_ein('mnie,jnbe->mbij', v_ooov, t2), 2, 3)
                 + P(_ein('ie,mbej->mbij', t1,
                          v_ovvo - _ein('njbf,mnef->mbej', t2, v_oovv)), 2, 3))
    h['vvvo'] = (v_vvvo - _ein('me,miab->abei', h['ov'], t2) + _ein('if,abef->abei', t1, h['vvvv'])
                 + 0.5 * _ein('mnei,mnab->abei', v_oovo, tt)
                 - P(_ein('mbef,miaf->abei', v_ovvv, t2), 0, 1)
                 - P(_ein('ma,mbei->abei', t1,
                          v_ovvo - _ein('nibf,mnef->mbei', t2, v_oovv)), 0, 1))
    return h


def lambda_residual(eps, V, nocc, t1, t2, l1, l2, h=None):
    """(R1[i,a], R2[i,j,a,b]) of the App. D Lambda equations at amplitudes t1, t2.

    R is linear in lambda and contains the diagonal Fock part D * lambda, so the
    solution satisfies R = 0.
    """
    o = nocc
    n = eps.size
    O, Vs = slice(0, o), slice(o, n)
    if h is None:
        h = hbar(eps, V, o, t1, t2)
    # G^e_a and G^i_m of App. D (lambda-t2 contractions), as Gv[a, e] and Go[m, i]
    Gv = -0.5 * _ein('mnef,mnaf->ae', t2, l2)
    Go = 0.5 * _ein('mnef,inef->mi', t2, l2)

    R1 = (h['ov'].copy() + _ein('ie,ea->ia', l1, h['vv']) - _ein('ma,im->ia', l1, h['oo'])
          + _ein('me,ieam->ia', l1, h['ovvo'])
          + 0.5 * _ein('imef,efam->ia', l2, h['vvvo'])
          - 0.5 * _ein('mnae,iemn->ia', l2, h['ovoo'])
          - _ein('ef,eifa->ia', Gv, h['vovv'])
          - _ein('mn,mina->ia', Go, h['ooov']))

    R2 = V[O, O, Vs, Vs].copy()
    R2 += P(_ein('ijae,eb->ijab', l2, h['vv']), 2, 3)
    R2 -= P(_ein('imab,jm->ijab', l2, h['oo']), 0, 1)
    R2 += 0.5 * _ein('mnab,ijmn->ijab', l2, h['oooo'])
    R2 += 0.5 * _ein('ijef,efab->ijab', l2, h['vvvv'])
    R2 += P(_ein('ie,ejab->ijab', l1, h['vovv']), 0, 1)
    R2 -= P(_ein('ma,ijmb->ijab', l1, h['ooov']), 2, 3)
    R2 += P(P(_ein('imae,jebm->ijab', l2, h['ovvo']), 0, 1), 2, 3)
    R2 += P(P(_ein('ia,jb->ijab', l1, h['ov']), 0, 1), 2, 3)
    R2 += P(_ein('ijae,be->ijab', V[O, O, Vs, Vs], Gv), 2, 3)
    R2 -= P(_ein('imab,mj->ijab', V[O, O, Vs, Vs], Go), 0, 1)
    return R1, R2


@dataclasses.dataclass
class LambdaResult:
    l1: np.ndarray
    l2: np.ndarray
    converged: bool
    iterations: int
    history: list


def solve_lambda(eps, V, nocc, t1, t2, tol=1e-10, max_iter=60, diis_size=8):
    """Jacobi + DIIS iteration of the Lambda equations from lambda = 0, with the
    amplitude solver's denominators, vectors (t1, then t2 over i<j, a<b) and DIIS.

    The first step gives lambda_ab^ij = <ij||ab> / (e_i + e_j - e_a - e_b) and
    lambda_a^i = F_ia / (e_i - e_a).
    """
    o = nocc
    v = eps.size - o
    d1, d2 = denominators(eps, o)
    h = hbar(eps, V, o, t1, t2)
    l1 = np.zeros((o, v), dtype=np.complex128)
    l2 = np.zeros((o, o, v, v), dtype=np.complex128)
    diis = DIIS(diis_size) if diis_size > 0 else None
    hist = []
    conv = False
    it = 0
    for it in range(1, max_iter + 1):
        R1, R2 = lambda_residual(eps, V, o, t1, t2, l1, l2, h)
        x = to_vector(l1, l2)
        e = to_vector(-R1 / d1, -R2 / d2)
        rnorm = float(np.linalg.norm(e))
        hist.append(rnorm)
        if diis is not None:
            diis.push(x + e, e)
            x = diis.extrapolate()
        else:
            x = x + e
        l1, l2 = from_vector(x, o, v)
        if not np.isfinite(rnorm):
            break
        if rnorm <= tol:
            conv = True
            break
    return LambdaResult(l1, l2, conv, it, hist)


def density(t1, t2, l1, l2):
    """Correlation part of the one-body density, gamma[p, q] = <0|(1+Lambda) e^-T {q+ p} e^T|0>
    (App. E), as an (o+v) x (o+v) matrix: blocks [i, j], [i, a], [a, i], [a, b]."""
    o, v = t1.shape
    g = np.zeros((o + v, o + v), dtype=np.complex128)
    # oo: the printed gamma_ij is this element with i and j exchanged
    goo = 0.5 * _ein('imef,efmj->ij', t2, l2.transpose(2, 3, 0, 1)) - _ein('ie,je->ij', t1, l1)
    g[:o, :o] = goo.T
    g[:o, o:] = l1
    g[o:, :o] = (t1.T + _ein('me,imae->ai', l1, t2) - _ein('me,ie,ma->ai', l1, t1, t1)
                 - 0.5 * _ein('mnef,inef,ma->ai', l2, t2, t1)
                 - 0.5 * _ein('mnef,ie,mnaf->ai', l2, t1, t2))
    g[o:, o:] = 0.5 * _ein('mnae,mnbe->ab', t2, l2) + _ein('ma,mb->ab', t1, l1)
    return g
