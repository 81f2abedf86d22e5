"""The element-by-element residual equals the full oracle residual on every entry."""
import numpy as np
import pytest

from oracle.ccsd import build_integrals, energy, residual
from oracle.elements import ResidualElements
from paper_2103_08473_amd.synth import make_amplitudes, make_system


@pytest.mark.parametrize("o,v,X,seed", [(3, 5, 9, 0), (5, 9, 17, 1), (2, 4, 6, 2)])
def test_elements_equal_full_residual(o, v, X, seed):
    eps, B = make_system(o, v, X, seed=seed, sigma=0.2)
    t1, t2 = make_amplitudes(o, v, seed=seed + 50, scale=0.1)
    S1, S2 = residual(eps, build_integrals(B, o), t1, t2)
    el = ResidualElements(eps, B, o, t1, t2)
    for i in range(o):
        for a in range(v):
            assert abs(el.S1(i, a) - S1[i, a]) < 1e-13
        for j in range(o):
            for a in range(v):
                for b in range(v):
                    assert abs(el.S2(i, j, a, b) - S2[i, j, a, b]) < 1e-13, (i, j, a, b)
    assert abs(el.energy() - energy(eps, build_integrals(B, o), t1, t2)) < 1e-13
