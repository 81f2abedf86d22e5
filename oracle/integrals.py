"""Two-electron integrals from density-fitting factors (oracle; test infrastructure).

Definitions (no blocking, no symmetry tricks):
  (pq|rs)   = sum_P B[P,p,q] B[P,r,s]                       factorised Coulomb integrals
  <pq||rs>  = (pr|qs) - (ps|qr)                             antisymmetrised, physicist order

The second line is the antisymmetrisation and reordering the paper applies
after its integral transformation (section "Index transformation algorithms":
<pr||qs> = (pq|rs) - (ps|rq), relabelled).  In Appendix A the symbol
V^{pq}_{rs} is read as <pq||rs> (upper indices = bra = created spinors) and
V^{pq dagger}_{rs} as conj(<pq||rs>).
"""
import numpy as np


def mulliken(B, s1, s2, s3, s4):
    """(pq|rs) for p in s1, q in s2, r in s3, s in s4 (slices or index arrays)."""
    return np.einsum('Ppq,Prs->pqrs', B[:, s1, s2], B[:, s3, s4], optimize=True)


def antisym(B, s1, s2, s3, s4):
    """<pq||rs> = (pr|qs) - (ps|qr) for p in s1, q in s2, r in s3, s in s4."""
    direct = np.einsum('Ppr,Pqs->pqrs', B[:, s1, s3], B[:, s2, s4], optimize=True)
    exch = np.einsum('Pps,Pqr->pqrs', B[:, s1, s4], B[:, s2, s3], optimize=True)
    return direct - exch
