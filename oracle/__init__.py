"""CPU oracle for the complex spin-orbital CCSD amplitude iteration.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything in this
package.  The HIP library never calls it and shares no code with it.

Plain numpy complex128, written from the paper (Appendix A, eq. CC_general,
plus the implementation section for the MP2 start, the denominator update and
DIIS).  Every function cites the passage it follows.  Where the paper is
silent the readings used are listed in the module docstrings.

Pins (tests/test_oracle_*.py, all CPU):
  * residual == <Phi_l| e^-T H e^T |Phi_0> evaluated by brute-force second
    quantisation in the full Fock space (o = 3, 4) at random amplitudes;
  * converged CCSD == FCI for 2-electron systems and for 1 electron;
  * first-iteration energy == closed-form MP2;
  * integral symmetries, amplitude antisymmetry, orbital-phase invariance,
    real-factor limit, Jacobi and DIIS reaching the same fixed point;
  * the element-by-element residual (large sizes) == the full residual;
  * CCD (T1 = 0) for two electrons == CI over the reference and its doubles;
  * CC2 residuals == their defining second-quantised projections;
  * perturbative triples (oracle/triples.py): W~, Z~ == the connected and
    disconnected triples projections, E(+T) == fourth-order triples energy;
  * Lambda equations (oracle/cclambda.py) == the gradient of the CC Lagrangian
    by brute force; the App. E density == the Lagrangian expectation value of
    {q+ p}, == the exact 1-RDM for two electrons, diagonal == dE/d eps_p;
  * DF factors (oracle/dffactors.py): fitted integrals == their closed form for
    J = L K, V = L L^T, and == the linear-solve route.
"""
from .integrals import antisym, mulliken  # noqa: F401
from .ccsd import (  # noqa: F401
    CCSDResult, DIIS, cc2_residual, energy, jacobi_step, mp2_energy_iterative, pack_t2,
    residual, solve, tau, unpack_t2,
)
from .fci import fci_two_electron, fci_one_electron  # noqa: F401
from .triples import triples_energies  # noqa: F401
from .cclambda import density, lambda_residual, solve_lambda  # noqa: F401
from .dffactors import df_factors, metric_inverse_sqrt  # noqa: F401
