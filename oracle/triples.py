"""Perturbative triples corrections E(+T) and E((T)) (App. C; oracle, test infrastructure).

Plain numpy over the full o^3 v^3 triples space: small systems only.

Readings of App. C (each pinned in tests/test_oracle_triples.py against brute-force
second quantisation, not against this module):

* W.  The printed intermediate W^abc_ijk uses the elements <ie||ab> and <ij||am>.
  For complex spinors the sums W^abc + W^bca + W^cab equal the connected triples
  projection <Phi_ijk^abc| W_N T2 |0> only with the excitation elements
  <ab||ie> and <am||ij> (bra and ket exchanged, i.e. the complex conjugates of the
  printed ones); for real spinors the two coincide.  This module uses the
  excitation elements.
* E(+T) = -(1/36) sum over all ijk, abc of |W~|^2 / D, D = e_a + e_b + e_c - e_i -
  e_j - e_k, with W~ = W^abc + W^bca + W^cab: one factor conjugated (the printed
  product of two W~ is read as |W~|^2).  This is the fourth-order triples energy
  sum_T |<T| W_N T2 |0>|^2 / (E_0 - E_T).
* Z~ = Z^abc + Z^cab + Z^bca with the printed Z (f_kc = 0 for canonical spinors)
  equals the disconnected projection <Phi_ijk^abc| W_N T1 |0>.
* E((T)) = E(+T) - (1/36) sum Re(conj(Z~) W~) / D: the singles-triples term of
  CCSD(T) with one factor conjugated.  The paper prints it with a plus sign and
  the same D; with D > 0 (which the sign of E(+T) fixes) that would raise the
  energy where the fifth-order singles-triples term lowers it, so the sign is
  read as garbled.  The term is half of the fifth-order perturbation-theory
  singles-triples energy 2 Re sum_T <0|T1^+ W_N|T><T|W_N T2|0> / (E_0 - E_T).
* Y~ = Y^abc + Y^cab + Y^bca with the printed Y equals the triples projection of
  e^(T1+T2) |0> (the disconnected triples T1 T2 + T1^3/6).
* E(-T) = E(+T) + (1/36) sum Re(conj(Y~) W~), as printed (one factor conjugated).
  At lowest order Y~ ~ -Z~/D, so this term and the singles-triples term of
  E((T)) carry the same sign, which is what makes the plus here and the minus
  above one consistent reading.
"""
import numpy as np


def _split(eps, nocc):
    return eps[:nocc], eps[nocc:]


def triples_W(V, nocc, t2):
    """W~[i,j,k,a,b,c] = W^abc + W^bca + W^cab with the excitation elements (App. C)."""
    n = V.shape[0]
    O, Vs = slice(0, nocc), slice(nocc, n)
    Ve = V[Vs, Vs, O, Vs].transpose(2, 3, 0, 1)   # <ab||ie> as [i, e, a, b]
    Vm = V[Vs, O, O, O].transpose(2, 3, 0, 1)     # <am||ij> as [i, j, a, m]
    W = (np.einsum('ieab,jkec->ijkabc', Ve, t2) + np.einsum('jeab,kiec->ijkabc', Ve, t2)
         + np.einsum('keab,ijec->ijkabc', Ve, t2))
    W += (np.einsum('ijam,kmbc->ijkabc', Vm, t2) + np.einsum('jkam,imbc->ijkabc', Vm, t2)
          + np.einsum('kiam,jmbc->ijkabc', Vm, t2))
    return W + W.transpose(0, 1, 2, 4, 5, 3) + W.transpose(0, 1, 2, 5, 3, 4)


def triples_Z(V, nocc, t1):
    """Z~[i,j,k,a,b,c] = Z^abc + Z^cab + Z^bca with the printed Z (f_kc = 0)."""
    n = V.shape[0]
    O, Vs = slice(0, nocc), slice(nocc, n)
    Vd = V[Vs, Vs, O, O].transpose(2, 3, 0, 1)    # <ab||ij> = <ij||ab>^* as [i, j, a, b]
    Z = (np.einsum('ijab,kc->ijkabc', Vd, t1) + np.einsum('jkab,ic->ijkabc', Vd, t1)
         + np.einsum('kiab,jc->ijkabc', Vd, t1))
    return Z + Z.transpose(0, 1, 2, 5, 3, 4) + Z.transpose(0, 1, 2, 4, 5, 3)


def triples_Y(t1, t2):
    """Y~[i,j,k,a,b,c] = Y^abc + Y^cab + Y^bca with the printed Y."""
    Y = (np.einsum('ia,jb,kc->ijkabc', t1, t1, t1) - np.einsum('ja,ib,kc->ijkabc', t1, t1, t1)
         + np.einsum('ja,kb,ic->ijkabc', t1, t1, t1) - np.einsum('ka,jb,ic->ijkabc', t1, t1, t1)
         + np.einsum('ka,ib,jc->ijkabc', t1, t1, t1) - np.einsum('ia,kb,jc->ijkabc', t1, t1, t1)) / 3.0
    Y += (np.einsum('ijab,kc->ijkabc', t2, t1) + np.einsum('jkab,ic->ijkabc', t2, t1)
          + np.einsum('kiab,jc->ijkabc', t2, t1))
    return Y + Y.transpose(0, 1, 2, 5, 3, 4) + Y.transpose(0, 1, 2, 4, 5, 3)


def triples_denominator(eps, nocc):
    eo, ev = _split(eps, nocc)
    return (ev[None, None, None, :, None, None] + ev[None, None, None, None, :, None]
            + ev[None, None, None, None, None, :] - eo[:, None, None, None, None, None]
            - eo[None, :, None, None, None, None] - eo[None, None, :, None, None, None])


def triples_energies(eps, V, nocc, t1, t2):
    """Return (E(+T), E((T)), E(-T)) for amplitudes t1, t2 (real parts; Hartree)."""
    o = nocc
    v = eps.size - o
    if o < 3 or v < 3:
        return 0.0, 0.0, 0.0     # no triple excitation exists
    D = triples_denominator(eps, o)
    Wt = triples_W(V, o, t2)
    Zt = triples_Z(V, o, t1)
    Yt = triples_Y(t1, t2)
    e4 = -float((np.abs(Wt) ** 2 / D).sum()) / 36.0
    e5 = -float((np.conj(Zt) * Wt / D).real.sum()) / 36.0
    ey = float((np.conj(Yt) * Wt).real.sum()) / 36.0
    return e4, e4 + e5, e4 + ey
