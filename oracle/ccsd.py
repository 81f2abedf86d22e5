"""Complex spin-orbital CCSD, following the paper's Appendix A (oracle; test infrastructure).

Index convention: i, j, k, l occupied (0..o-1); a, b, c, d virtual (0..v-1,
spinor o+a).  t1[i, a] = t_i^a, t2[i, j, a, b] = t_ij^ab with
T2 = 1/4 sum t_ij^ab a+_a a+_b a_j a_i (so t2 is antisymmetric in ij and ab).
Fock matrix f = diag(eps) (the generator's spinors are canonical).

Readings of the paper used here (it is silent or inconsistent on these):
  * V^{pq}_{rs} = <pq||rs> = (pr|qs) - (ps|qr); V^{pq dagger}_{rs} = conj(<pq||rs>).
  * P^-_{pq} f(p, q) = f(p, q) - f(q, p) (first equation of Appendix A); P^-_{ji} is
    the same operator as P^-_{ij}.
  * The correlation energy is E = sum_ia f_ia t_i^a + 1/4 sum_ijab <ij||ab> tau_ij^ab
    (the paper shows only the contraction pattern E() += V+ * T); it is complex.
  * Start from t = 0: the first Jacobi step gives the MP2 amplitudes and the first
    energy is E_MP2 (section "Coupled cluster implementation").
  * Update (the denominator scaling): t <- t - S / D with D_i^a = e_a - e_i + s and
    D_ij^ab = e_a + e_b - e_i - e_j + 2 s (s = level shift, default 0).
  * DIIS (Pulay): vectors x = [t1, t2 packed over i<j, a<b], error e = the Jacobi
    step, extrapolated from the updated vectors x + e; see class DIIS.
  * Residual norm = ||e||_2 over the unique amplitudes; converged when <= tol.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .integrals import antisym

_LADDER_BLOCK_BYTES = 256 << 20


# --------------------------------------------------------------------------- helpers
def P(x, ax1, ax2):
    """P^-_{pq} applied to an array: x - x with axes ax1, ax2 swapped (App. A, first line)."""
    return x - np.swapaxes(x, ax1, ax2)


def tau(t1, t2):
    """tau_ij^ab = t_ij^ab + P^-_ij (t_i^a t_j^b)   (App. A, second line)."""
    tt = np.einsum('ia,jb->ijab', t1, t1)
    return t2 + P(tt, 0, 1)


def build_integrals(B, nocc):
    """The stored integral classes used by the App. A equations, as dense arrays.

    vvvv is not stored: the ladder builds it in blocks of a (see ``_ladder``).
    """
    o = nocc
    n = B.shape[1]
    O, V = slice(0, o), slice(o, n)
    return {
        'B': B, 'o': o,
        'oooo': antisym(B, O, O, O, O),   # <kl||ij>
        'ooov': antisym(B, O, O, O, V),   # <kl||ic>
        'oovv': antisym(B, O, O, V, V),   # <kl||cd>
        'vovo': antisym(B, V, O, V, O),   # <ak||ci>
        'vovv': antisym(B, V, O, V, V),   # <ak||cd>
    }


def ladder_rows(B, o, tau_, a0, a1):
    """Rows a0 <= a < a1 of the particle ladder 1/2 sum_cd V^{ab}_{cd} tau_ij^cd,
    with <ab||cd> formed from B for those rows; returns [i, j, a-a0, b]."""
    n = B.shape[1]
    vabcd = antisym(B, slice(o + a0, o + a1), slice(o, n), slice(o, n), slice(o, n))
    return 0.5 * np.einsum('abcd,ijcd->ijab', vabcd, tau_, optimize=True)


def _ladder(ints, tau_):
    """1/2 sum_cd V^{ab}_{cd} tau_ij^cd with <ab||cd> formed for blocks of a."""
    B, o = ints['B'], ints['o']
    n = B.shape[1]
    v = n - o
    out = np.zeros(tau_.shape, dtype=np.complex128)
    blk = max(1, int(_LADDER_BLOCK_BYTES // (16 * v ** 3)))
    for a0 in range(0, v, blk):
        a1 = min(v, a0 + blk)
        out[:, :, a0:a1, :] = ladder_rows(B, o, tau_, a0, a1)
    return out


# --------------------------------------------------------------------------- residual
def residual(eps, ints, t1, t2):
    """Return (S1[i,a], S2[i,j,a,b]) of eq. CC_general (Appendix A) for amplitudes t1, t2.

    S is the full projected equation <Phi_l| e^-T H e^T |Phi_0> including the
    diagonal Fock contribution, so the converged amplitudes satisfy S = 0.
    """
    o = ints['o']
    e_o, e_v = eps[:o], eps[o:]
    v = e_v.size
    fo = np.diag(e_o).astype(np.complex128)      # f_ki
    fv = np.diag(e_v).astype(np.complex128)      # f_ac
    fov = np.zeros((o, v), dtype=np.complex128)  # f_kc (zero for canonical spinors)
    fvo = fov.conj().T                           # f_ai = conj(f_ia)
    Voooo, Vooov, Voovv = ints['oooo'], ints['ooov'], ints['oovv']
    Vvovo, Vvovv = ints['vovo'], ints['vovv']
    ein = lambda s, *a: np.einsum(s, *a, optimize=True)  # noqa: E731

    tau_ = tau(t1, t2)

    # one-body intermediates
    Hac = fv + 0.5 * ein('klcd,klda->ac', Voovv, tau_)
    Gac = Hac + ein('akcd,kd->ac', Vvovv, t1) - ein('kc,ka->ac', fov, t1)
    Hki = -fo + 0.5 * ein('klcd,licd->ki', Voovv, tau_)
    Gki = Hki - ein('klic,lc->ki', Vooov, t1) - ein('kc,ic->ki', fov, t1)
    Hkc = fov + ein('klcd,ld->kc', Voovv, t1)

    # H^{ak}_{ci}
    Hakci = (Vvovo
             + ein('akcd,id->akci', Vvovv, t1)
             - ein('klic,la->akci', Vooov, t1)
             + ein('klcd,liad->akci', Voovv, 0.5 * t2 + ein('la,id->liad', t1, t1)))

    # C^{kb}_{ij}: V^{ij dagger}_{kb} = conj(<ij||kb>) stored as [k,b,i,j]
    Ckbij = (np.conj(Vooov).transpose(2, 3, 0, 1)
             + P(ein('bkci,jc->kbij', Vvovo, t1), 2, 3)
             - 0.5 * ein('bkcd,ijcd->kbij', Vvovv, tau_))

    # A^{kl}_{ij}
    Aklij = (Voooo
             + P(ein('klic,jc->klij', Vooov, t1), 2, 3)
             + 0.5 * ein('klcd,ijcd->klij', Voovv, tau_))

    # S^{ab}_{ij}
    ring = ein('akci,jkcb->ijab', Hakci, t2)
    S2 = P(P(ring, 0, 1), 2, 3)
    S2 += ein('kj,ikab->ijab', Gki, t2) - ein('ki,jkab->ijab', Gki, t2)
    Vcj_dag = np.conj(Vvovv).transpose(2, 3, 0, 1)   # conj(<cj||ab>) as [a,b,c,j]
    S2 += P(ein('abcj,ic->ijab', Vcj_dag, t1), 0, 1)
    S2 += P(ein('ac,ijcb->ijab', Gac, t2), 2, 3)
    S2 += P(ein('kaij,kb->ijab', Ckbij, t1), 2, 3)
    S2 += 0.5 * ein('klij,klab->ijab', Aklij, tau_)
    S2 += _ladder(ints, tau_)
    S2 += np.conj(Voovv)                             # V^{ij dagger}_{ab} as [i,j,a,b]

    # S^a_i
    S1 = fvo.T.copy()                                # F^{i dagger}_a = f_ai, as [i,a]
    S1 += ein('ac,ic->ia', Hac, t1)
    S1 += ein('ki,ka->ia', Hki, t1)
    S1 += ein('kc,ikac->ia', Hkc, t2)
    S1 += ein('kc,ic,ka->ia', Hkc - 2.0 * fov, t1, t1)
    S1 += 0.5 * ein('akcd,ikcd->ia', Vvovv, tau_)
    S1 += 0.5 * ein('klic,klca->ia', Vooov, tau_)
    S1 -= ein('akci,kc->ia', Vvovo, t1)
    return S1, S2


def energy(eps, ints, t1, t2):
    """E = sum_ia f_ia t_i^a + 1/4 sum_ijab <ij||ab> tau_ij^ab (complex)."""
    o = ints['o']
    fov = np.zeros((o, eps.size - o), dtype=np.complex128)
    return complex(np.sum(fov * t1) + 0.25 * np.einsum('ijab,ijab->', ints['oovv'], tau(t1, t2)))


def denominators(eps, nocc, level_shift=0.0):
    """D_i^a = e_a - e_i + s,  D_ij^ab = e_a + e_b - e_i - e_j + 2 s."""
    e_o, e_v = eps[:nocc], eps[nocc:]
    d1 = e_v[None, :] - e_o[:, None] + level_shift
    d2 = (e_v[None, None, :, None] + e_v[None, None, None, :]
          - e_o[:, None, None, None] - e_o[None, :, None, None] + 2.0 * level_shift)
    return d1, d2


def jacobi_step(S1, S2, d1, d2):
    """Denominator update step: Delta = -S / D."""
    return -S1 / d1, -S2 / d2


# --------------------------------------------------------------------------- packing
def _pair_masks(o, v):
    iu, ju = np.triu_indices(o, 1)
    au, bu = np.triu_indices(v, 1)
    return iu, ju, au, bu


def pack_t2(t2):
    """Unique amplitudes t2[i<j, a<b] as a 2-D array [(i<j), (a<b)] (row-major pairs)."""
    o, v = t2.shape[0], t2.shape[2]
    iu, ju, au, bu = _pair_masks(o, v)
    return t2[iu, ju][:, au, bu]


def unpack_t2(p, o, v):
    """Inverse of pack_t2: the full antisymmetric t2[i,j,a,b]."""
    iu, ju, au, bu = _pair_masks(o, v)
    t2 = np.zeros((o, o, v, v), dtype=np.complex128)
    blk = np.zeros((len(iu), v, v), dtype=np.complex128)
    blk[:, au, bu] = p
    blk[:, bu, au] = -p
    t2[iu, ju] = blk
    t2[ju, iu] = -blk
    return t2


def to_vector(t1, t2):
    return np.concatenate([t1.ravel(), pack_t2(t2).ravel()])


def from_vector(x, o, v):
    t1 = x[:o * v].reshape(o, v).copy()
    t2 = unpack_t2(x[o * v:].reshape(o * (o - 1) // 2, v * (v - 1) // 2), o, v)
    return t1, t2


# --------------------------------------------------------------------------- DIIS
class DIIS:
    """Pulay DIIS on complex vectors.

    Keeps the last ``size`` pairs (x_k + e_k, e_k).  With at least two pairs it
    minimises ||sum_k c_k e_k|| subject to sum_k c_k = 1 by solving
    [[G, 1], [1^T, 0]] [c; lam] = [0; 1] with G_kl = <e_k, e_l> = sum conj(e_k) e_l,
    and returns sum_k c_k (x_k + e_k).  If cond(G) = max eig / min eig exceeds
    1e14 (or G is singular) the oldest pair is dropped and the solve retried.
    With one pair it returns x + e (a plain Jacobi step).
    """

    COND_MAX = 1e14

    def __init__(self, size=8):
        self.size = size
        self.xs, self.es = [], []

    def push(self, x_new, e):
        self.xs.append(x_new)
        self.es.append(e)
        if len(self.xs) > self.size:
            self.xs.pop(0)
            self.es.pop(0)

    def coefficients(self):
        while len(self.es) >= 2:
            m = len(self.es)
            G = np.empty((m, m), dtype=np.complex128)
            for k in range(m):
                for l in range(m):
                    G[k, l] = np.vdot(self.es[k], self.es[l])
            w = np.linalg.eigvalsh(G)
            if w[0] <= 0.0 or w[-1] / w[0] > self.COND_MAX:
                self.xs.pop(0)
                self.es.pop(0)
                continue
            A = np.zeros((m + 1, m + 1), dtype=np.complex128)
            A[:m, :m] = G
            A[:m, m] = 1.0
            A[m, :m] = 1.0
            rhs = np.zeros(m + 1, dtype=np.complex128)
            rhs[m] = 1.0
            return np.linalg.solve(A, rhs)[:m]
        return np.ones(len(self.es), dtype=np.complex128)

    def extrapolate(self):
        c = self.coefficients()
        out = np.zeros_like(self.xs[-1])
        for ck, xk in zip(c, self.xs):
            out += ck * xk
        return out


# --------------------------------------------------------------------------- solver
@dataclasses.dataclass
class CCSDResult:
    energy: complex
    t1: np.ndarray
    t2: np.ndarray
    converged: bool
    iterations: int
    history: list  # (iteration, energy, residual norm)


def cc2_residual(eps, ints, t1, t2):
    """CC2 residuals (Christiansen, Koch and Joergensen's definition; the paper's App. B
    working equations are its expansion).

    Singles: the CCSD singles equation, unchanged (<mu1| e^-T H e^T |0> with T = T1 + T2
    reaches singles only through H + [H, T2] after the T1 transformation).
    Doubles: <mu2| e^-T1 H e^T1 + [F, T2] |0>, i.e. the CCSD doubles residual evaluated at
    T2 = 0 (the T1-transformed Hamiltonian's doubles projection) plus the diagonal Fock
    commutator (e_a + e_b - e_i - e_j) t_ij^ab.
    """
    o = t1.shape[0]
    S1, _ = residual(eps, ints, t1, t2)
    _, S2 = residual(eps, ints, t1, np.zeros_like(t2))
    _, d2 = denominators(eps, o)
    return S1, S2 + d2 * t2


def solve(eps, B, nocc, max_iter=30, tol=1e-10, diis_size=8, level_shift=0.0, ints=None,
          callback=None, doubles_only=False, cc2=False):
    """Iterate the CCSD equations from t = 0 (first step = MP2), with Jacobi + DIIS.

    Iteration k: S = residual(x_k); e_k = -S/D; push (x_k + e_k, e_k); x_{k+1} =
    DIIS extrapolation (or x_k + e_k); E_k = energy(x_{k+1}); stop when ||e_k|| <= tol.

    doubles_only: CCD (the paper's CCDOUBLES keyword), the same equations with
    T1 held at zero and no T1 equation (its step is zero).
    cc2: CC2 (the paper's CC2 keyword), the residuals of cc2_residual; the
    energy expression is the CCSD one.
    """
    if doubles_only and cc2:
        raise ValueError("CCD and CC2 are exclusive")
    eps = np.asarray(eps, dtype=np.float64)
    o = nocc
    v = eps.size - o
    if ints is None:
        ints = build_integrals(B, o)
    d1, d2 = denominators(eps, o, level_shift)
    t1 = np.zeros((o, v), dtype=np.complex128)
    t2 = np.zeros((o, o, v, v), dtype=np.complex128)
    diis = DIIS(diis_size) if diis_size > 0 else None
    history = []
    converged = False
    E = 0j
    it = 0
    for it in range(1, max_iter + 1):
        S1, S2 = cc2_residual(eps, ints, t1, t2) if cc2 else residual(eps, ints, t1, t2)
        dt1, dt2 = jacobi_step(S1, S2, d1, d2)
        if doubles_only:
            dt1 = np.zeros_like(dt1)
        x = to_vector(t1, t2)
        e = to_vector(dt1, dt2)
        rnorm = float(np.linalg.norm(e))
        if diis is not None:
            diis.push(x + e, e)
            x_next = diis.extrapolate()
        else:
            x_next = x + e
        t1, t2 = from_vector(x_next, o, v)
        E = energy(eps, ints, t1, t2)
        history.append((it, E, rnorm))
        if callback is not None:
            callback(it, E, rnorm)
        if not (np.isfinite(E.real) and np.isfinite(rnorm)):
            break
        if rnorm <= tol:
            converged = True
            break
    return CCSDResult(E, t1, t2, converged, it, history)


def mp2_energy_iterative(eps, B, nocc):
    """Energy after the first iteration from t = 0 (the MP2 start)."""
    res = solve(eps, B, nocc, max_iter=1, tol=0.0, diis_size=0)
    return res.energy
