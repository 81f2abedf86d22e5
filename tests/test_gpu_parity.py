"""HIP path vs the CPU oracle, through the C ABI (run on an MI355X)."""
import sys

import numpy as np
import pytest

import oracle
from oracle.ccsd import build_integrals, energy, residual
from paper_2103_08473_amd.synth import make_amplitudes, make_system

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# (nocc, nvir, naux): below one 64-tile, several tiles with ragged tails, degenerate pair spaces
RESIDUAL_CASES = [(3, 4, 9), (5, 7, 13), (10, 40, 120), (12, 70, 150), (16, 67, 131),
                  (1, 9, 20), (2, 12, 30), (4, 1, 6), (1, 1, 3)]


@pytest.mark.parametrize("group", [64, 0])
@pytest.mark.parametrize("o,v,X", RESIDUAL_CASES)
def test_residual_matches_oracle(lib, o, v, X, group):
    """group: nvir up to which the particle ladder builds all rows' tiles in one product
    (64, the default) or 0 (the per-row Hermitian build at every size)."""
    from paper_2103_08473_amd.exacc import CCSD
    say("residual case", o, v, X, "ladder_group_nvir", group)
    eps, B = make_system(o, v, X, seed=o * 1000 + v, sigma=0.2)
    t1, t2 = make_amplitudes(o, v, seed=7 + o, scale=0.1)
    ints = build_integrals(B, o)
    S1, S2 = residual(eps, ints, t1, t2)
    E = energy(eps, ints, t1, t2)
    with CCSD(eps, B, o, ladder_group_nvir=group) as cc:
        cc.set_amplitudes(t1, t2)
        g1, g2 = cc.residual()
        ge = cc.energy()
        r1, r2 = cc.amplitudes()
    assert np.array_equal(r1, t1) and np.array_equal(r2, t2)
    scale = max(np.abs(S2).max() if S2.size else 0.0, np.abs(S1).max(), 1e-300)
    assert np.abs(g1 - S1).max() <= 1e-12 * scale
    if S2.size:
        assert np.abs(g2 - S2).max() <= 1e-12 * scale
    assert abs(ge - E) <= 1e-12 * max(1.0, abs(E))


@pytest.mark.parametrize("o,v,X,seed,sigma,iters,shift,ndiis", [
    (10, 40, 120, 0, 0.05, 30, 0.0, 8),     # the (10, 40, 120) configuration, literal generator
    (6, 50, 150, 1, None, 25, 0.0, 8),      # ragged tiles, size-scaled generator
    (6, 50, 150, 1, None, 25, 0.3, 8),      # level shift 0.3 (LSHIFT) in every denominator
    (6, 50, 150, 1, 0.02, 25, 0.0, 0),      # plain Jacobi steps (no DIIS; sigma_B 0.02, where
                                            # they converge)
    (6, 50, 150, 1, 0.02, 25, 0.3, 0),      # plain Jacobi with the level shift
    (5, 33, 99, 4, None, 20, 0.3, 3),       # both, with a DIIS subspace that drops pairs
])
def test_iterations_match_oracle(lib, o, v, X, seed, sigma, iters, shift, ndiis):
    """Energy after every iteration (MP2 start, Jacobi step with level shift s, DIIS of the
    given size or none) within 1e-10 Eh."""
    from paper_2103_08473_amd.exacc import CCSD
    say("iteration case", o, v, X, seed, sigma, "shift", shift, "diis", ndiis)
    eps, B = make_system(o, v, X, seed=seed, sigma=sigma)
    ref = oracle.solve(eps, B, o, max_iter=iters, tol=1e-10, diis_size=ndiis, level_shift=shift)
    with CCSD(eps, B, o, tol=1e-10, level_shift=shift, diis_size=ndiis) as cc:
        _, conv, hist = cc.solve(max_iter=iters)
    assert len(hist) == len(ref.history)
    for (it, eg, rg), (_, eo, ro) in zip(hist, ref.history):
        assert abs(eg - eo) <= 1e-10, (it, eg, eo)
        assert abs(rg - ro) <= 1e-8 * max(1.0, ro), (it, rg, ro)
    assert conv == ref.converged


@pytest.mark.parametrize("v,X,seed", [(8, 20, 0), (14, 30, 1)])
def test_two_electron_equals_fci(lib, v, X, seed):
    from paper_2103_08473_amd.exacc import CCSD
    say("fci case", v, X, seed)
    eps, B = make_system(2, v, X, seed=seed, sigma=0.05)
    e_fci, _, _ = oracle.fci_two_electron(eps, B)
    with CCSD(eps, B, 2, tol=1e-12, max_iter=80) as cc:
        e, conv, _ = cc.solve()
    assert conv
    assert abs(e - e_fci) < 1e-10


@pytest.mark.parametrize("o,v,X,seed,sigma,iters", [
    (10, 40, 120, 0, 0.05, 25),
    (6, 50, 150, 1, None, 20),
])
def test_ccd_iterations_match_oracle(lib, o, v, X, seed, sigma, iters):
    """CCD (doubles_only): energy after every iteration within 1e-10 Eh of the oracle's CCD,
    and t1 stays exactly zero."""
    from paper_2103_08473_amd.exacc import CCSD
    say("ccd iteration case", o, v, X, seed, sigma)
    eps, B = make_system(o, v, X, seed=seed, sigma=sigma)
    ref = oracle.solve(eps, B, o, max_iter=iters, tol=1e-10, doubles_only=True)
    with CCSD(eps, B, o, tol=1e-10, doubles_only=1) as cc:
        _, conv, hist = cc.solve(max_iter=iters)
        t1, t2 = cc.amplitudes()
    assert len(hist) == len(ref.history)
    for (it, eg, rg), (_, eo, ro) in zip(hist, ref.history):
        assert abs(eg - eo) <= 1e-10, (it, eg, eo)
        assert abs(rg - ro) <= 1e-8 * max(1.0, ro), (it, rg, ro)
    assert np.abs(t1).max() == 0
    assert np.abs(t2 - ref.t2).max() <= 1e-10


def test_ccd_two_electron_equals_cid(lib):
    from paper_2103_08473_amd.exacc import CCSD
    eps, B = make_system(2, 14, 30, seed=1, sigma=0.05)
    e_cid, _, _ = oracle.fci_two_electron(eps, B, doubles_only=True)
    with CCSD(eps, B, 2, tol=1e-12, max_iter=80, doubles_only=1) as cc:
        e, conv, _ = cc.solve()
    assert conv
    assert abs(e - e_cid) < 1e-10


@pytest.mark.parametrize("o,v,X", [(3, 4, 9), (10, 40, 120), (16, 67, 131), (1, 9, 20), (4, 1, 6)])
def test_cc2_residual_matches_oracle(lib, o, v, X):
    """CC2 residuals (T1-dressed doubles + diagonal Fock term; CCSD singles) at random
    amplitudes, element by element, FP64: 1e-12 of the largest entry."""
    from paper_2103_08473_amd.exacc import CCSD
    say("cc2 residual case", o, v, X)
    eps, B = make_system(o, v, X, seed=o * 1000 + v + 5, sigma=0.2)
    t1, t2 = make_amplitudes(o, v, seed=9 + o, scale=0.1)
    S1, S2 = oracle.cc2_residual(eps, build_integrals(B, o), t1, t2)
    with CCSD(eps, B, o, cc2=1) as cc:
        cc.set_amplitudes(t1, t2)
        g1, g2 = cc.residual()
    scale = max(np.abs(S2).max() if S2.size else 0.0, np.abs(S1).max(), 1e-300)
    assert np.abs(g1 - S1).max() <= 1e-12 * scale
    if S2.size:
        assert np.abs(g2 - S2).max() <= 1e-12 * scale


def test_cc2_iterations_match_oracle(lib):
    """CC2 solve: energy after every iteration within 1e-10 Eh of the oracle's CC2."""
    from paper_2103_08473_amd.exacc import CCSD
    o, v, X, iters = 8, 40, 120, 30
    eps, B = make_system(o, v, X, seed=3)
    ref = oracle.solve(eps, B, o, max_iter=iters, tol=1e-10, cc2=True)
    with CCSD(eps, B, o, tol=1e-10, cc2=1) as cc:
        _, conv, hist = cc.solve(max_iter=iters)
        t1, t2 = cc.amplitudes()
    assert len(hist) == len(ref.history)
    for (it, eg, rg), (_, eo, ro) in zip(hist, ref.history):
        assert abs(eg - eo) <= 1e-10, (it, eg, eo)
        assert abs(rg - ro) <= 1e-8 * max(1.0, ro), (it, rg, ro)
    assert conv == ref.converged
    assert max(np.abs(t1 - ref.t1).max(), np.abs(t2 - ref.t2).max()) <= 1e-10


@pytest.mark.parametrize("o,v,X", [(3, 3, 7), (5, 12, 30), (6, 17, 40), (8, 20, 50)])
def test_triples_match_oracle(lib, o, v, X):
    """E(+T), E((T)), E(-T) (App. C) at random amplitudes vs the oracle (pinned by brute
    force): 1e-12 of |E(+T)|."""
    from oracle.integrals import antisym
    from oracle.triples import triples_energies
    from paper_2103_08473_amd.exacc import CCSD
    say("triples case", o, v, X)
    eps, B = make_system(o, v, X, seed=o * 100 + v, sigma=0.2)
    t1, t2 = make_amplitudes(o, v, seed=3 + o, scale=0.1)
    n = o + v
    V = antisym(B, slice(0, n), slice(0, n), slice(0, n), slice(0, n))
    e4, et, em = triples_energies(eps, V, o, t1, t2)
    with CCSD(eps, B, o) as cc:
        cc.set_amplitudes(t1, t2)
        g4, gt, gm = cc.triples()
        r1, r2 = cc.amplitudes()
    assert np.array_equal(r1, t1) and np.array_equal(r2, t2)
    assert abs(e4) > 1e-6 and abs(et - e4) > 1e-9 and abs(em - e4) > 1e-9
    assert abs(g4 - e4) <= 1e-12 * abs(e4)
    assert abs(gt - et) <= 1e-12 * abs(e4)
    assert abs(gm - em) <= 1e-12 * abs(e4)


@pytest.mark.parametrize("block", [1, 2, 3, 4])
def test_triples_occupied_blocks_match_oracle(lib, block):
    """Three nested loops over occupied blocks of n_red spinors (tiles of three blocks
    resident): every block size gives the oracle's E(+T), E((T)), E(-T), 1e-12 relative."""
    from oracle.integrals import antisym
    from oracle.triples import triples_energies
    from paper_2103_08473_amd.exacc import CCSD
    o, v, X = 7, 13, 30
    say("triples blocks", block)
    eps, B = make_system(o, v, X, seed=77, sigma=0.2)
    t1, t2 = make_amplitudes(o, v, seed=78, scale=0.1)
    n = o + v
    ref = triples_energies(eps, antisym(B, slice(0, n), slice(0, n), slice(0, n), slice(0, n)), o, t1, t2)
    with CCSD(eps, B, o, triples_occ_block=block) as cc:
        cc.set_amplitudes(t1, t2)
        got = cc.triples()
    for g, r in zip(got, ref):
        assert abs(g - r) <= 1e-12 * abs(ref[0])


def test_ccsd_t_after_converged_solve(lib):
    """CCSD(T): converged GPU CCSD plus GPU triples vs the oracle's solve plus triples."""
    from oracle.integrals import antisym
    from oracle.triples import triples_energies
    from paper_2103_08473_amd.exacc import CCSD
    o, v, X = 6, 24, 60
    eps, B = make_system(o, v, X, seed=17)
    ref = oracle.solve(eps, B, o, max_iter=80, tol=1e-11)
    n = o + v
    e4, et, em = triples_energies(eps, antisym(B, slice(0, n), slice(0, n), slice(0, n), slice(0, n)),
                                  o, ref.t1, ref.t2)
    with CCSD(eps, B, o, tol=1e-11, max_iter=80) as cc:
        e, conv, _ = cc.solve()
        g4, gt, gm = cc.triples()
    assert conv and ref.converged
    assert abs(e - ref.energy) <= 1e-10
    assert abs(g4 - e4) <= 1e-10 and abs(gt - et) <= 1e-10 and abs(gm - em) <= 1e-10
    say("  CCSD %.10f  E(+T) %.3e  E((T)) %.3e  E(-T) %.3e" % (e.real, g4, gt, gm))


def test_one_electron_is_exact_at_first_step(lib):
    from paper_2103_08473_amd.exacc import CCSD
    eps, B = make_system(1, 9, 20, seed=4, sigma=0.1)
    with CCSD(eps, B, 1, tol=1e-14) as cc:
        st, steps, r, conv = cc.iterate(5)
        assert conv and steps == 1 and r == 0.0
        assert cc.energy() == 0


def test_deterministic(lib):
    from paper_2103_08473_amd.exacc import CCSD
    eps, B = make_system(8, 36, 100, seed=3)
    out = []
    for _ in range(2):
        with CCSD(eps, B, 8) as cc:
            cc.iterate(6)
            out.append((cc.energy(), cc.amplitudes()[1]))
    assert out[0][0] == out[1][0]
    assert np.array_equal(out[0][1], out[1][1])


def test_invalid_inputs_are_rejected(lib):
    from paper_2103_08473_amd import exacc
    eps, B = make_system(4, 10, 20, seed=1)
    bad = B.copy()
    bad[3, 1, 2] += 1e-3                         # not Hermitian
    with pytest.raises(exacc.ExaccError) as e:
        exacc.CCSD(eps, bad, 4)
    assert e.value.status == exacc.ERR_INVALID_ARG
    nanB = B.copy()
    nanB[0, 0, 0] = np.nan
    with pytest.raises(exacc.ExaccError) as e:
        exacc.CCSD(eps, nanB, 4)
    assert e.value.status == exacc.ERR_INVALID_ARG
    e2 = eps.copy()
    e2[4] = e2[:4].max()                         # no gap
    with pytest.raises(exacc.ExaccError) as e:
        exacc.CCSD(e2, B, 4)
    assert e.value.status == exacc.ERR_INVALID_ARG
    with pytest.raises(exacc.ExaccError) as e:
        exacc.CCSD(eps, B, 4, hbm_budget_bytes=1 << 20)
    assert e.value.status == exacc.ERR_NOMEM
    with pytest.raises(exacc.ExaccError) as e:      # CCD and CC2 are exclusive
        exacc.CCSD(eps, B, 4, doubles_only=1, cc2=1)
    assert e.value.status == exacc.ERR_INVALID_ARG
    # triples need the FP64 integrals: refused while a mixed handle is still in FP32
    with exacc.CCSD(eps, B, 4, precision=exacc.MIXED_FP32) as cc:
        assert cc.phase()[0] == 1
        with pytest.raises(exacc.ExaccError) as e:
            cc.triples()
        assert e.value.status == exacc.ERR_INVALID_ARG
        st, _, r, _ = cc.iterate(1)                  # the handle stays usable
        assert np.isfinite(r)


def test_not_converged_status(lib):
    from paper_2103_08473_amd import exacc
    eps, B = make_system(4, 10, 20, seed=1)
    with exacc.CCSD(eps, B, 4) as cc:
        st, steps, r, conv = cc.iterate(1)
        assert st == exacc.NOT_CONVERGED and steps == 1 and not conv and r > 0


@pytest.mark.timeout(900)
def test_full_size_residual_samples(lib):
    """nocc=40, nvir=360, naux=1200 (the benchmark system, device inputs on a torch stream):
    the GPU residual at random amplitudes vs the element-by-element oracle on a grid of
    sampled entries, and the energy.  Tolerance: FP64 sums of up to P_v = 64,620 products,
    1e-11 relative to the largest sampled |S|."""
    import torch
    from oracle.elements import ResidualElements
    from paper_2103_08473_amd.exacc import CCSD
    o, v, X = 40, 360, 1200
    say("full-size case", o, v, X, ": generating inputs")
    eps, B = make_system(o, v, X, seed=0)
    t1, t2 = make_amplitudes(o, v, seed=1, scale=0.01)
    say("  GPU residual")
    eps_d = torch.from_numpy(eps).cuda()
    B_d = torch.from_numpy(B).cuda()
    stream = torch.cuda.Stream()
    with CCSD(eps_d, B_d, o, stream=stream.cuda_stream, timing=1) as cc:
        del B_d
        cc.set_amplitudes(t1, t2)
        g1, g2 = cc.residual()
        ge = cc.energy()
    say("  oracle entries")
    el = ResidualElements(eps, B, o, t1, t2)
    rng = np.random.default_rng(2024)
    ij = [tuple(rng.choice(o, 2, replace=False)) for _ in range(3)] + [(0, o - 1)]
    ab = [tuple(rng.choice(v, 2, replace=False)) for _ in range(4)] + [(0, v - 1), (v - 2, v - 1)]
    ref, got = [], []
    for (i, j) in ij:
        for (a, b) in ab:
            ref.append(el.S2(i, j, a, b))
            got.append(g2[i, j, a, b])
    say("  S2 samples done")
    for (i, a) in [(0, 0), (o - 1, v - 1)] + [(int(rng.integers(o)), int(rng.integers(v))) for _ in range(6)]:
        ref.append(el.S1(i, a))
        got.append(g1[i, a])
    ref, got = np.array(ref), np.array(got)
    scale = np.abs(ref).max()
    err = np.abs(ref - got).max()
    say("  max |dS| %.3e  scale %.3e" % (err, scale))
    assert scale > 0 and err <= 1e-11 * scale
    assert np.abs(g2 + g2.transpose(1, 0, 2, 3)).max() <= 1e-14 * scale
    assert abs(ge - el.energy()) <= 1e-10


# ---------------------------------------------------------------- mixed precision
@pytest.mark.parametrize("group", [64, 0])
@pytest.mark.parametrize("o,v,X", [(10, 40, 120), (12, 70, 150), (1, 9, 20)])
def test_fp32_phase_residual(lib, o, v, X, group):
    """FP32 contractions, FP64 assembly: the residual agrees with the FP64 oracle to FP32
    accuracy (sums of <= P_v products of unit roundoff 6e-8: 1e-5 of the largest |S|)."""
    from paper_2103_08473_amd import exacc
    say("fp32 residual case", o, v, X)
    eps, B = make_system(o, v, X, seed=o * 1000 + v, sigma=0.2)
    t1, t2 = make_amplitudes(o, v, seed=7 + o, scale=0.1)
    S1, S2 = residual(eps, build_integrals(B, o), t1, t2)
    with exacc.CCSD(eps, B, o, precision=exacc.MIXED_FP32, ladder_group_nvir=group) as cc:
        assert cc.phase() == (True, 0)
        cc.set_amplitudes(t1, t2)
        g1, g2 = cc.residual()
    scale = max(np.abs(S2).max() if S2.size else 0.0, np.abs(S1).max())
    e1 = np.abs(g1 - S1).max() / scale
    e2 = np.abs(g2 - S2).max() / scale if S2.size else 0.0
    say("  rel err S1 %.2e S2 %.2e" % (e1, e2))
    assert e1 <= 1e-5 and e2 <= 1e-5
    assert e1 + e2 > 1e-12          # the FP32 phase really ran in FP32


@pytest.mark.parametrize("group", [64, 0])
@pytest.mark.parametrize("o,v,X,seed", [(6, 40, 120, 2), (8, 48, 144, 3)])
def test_mixed_precision_solve_matches_fp64_oracle(lib, o, v, X, seed, group):
    """FP32 phase, switch below 1e-5, >= 3 FP64 iterations to 1e-10: |dE| <= 1e-7 Eh
    against the converged FP64 oracle (and the amplitudes to 1e-7)."""
    from paper_2103_08473_amd import exacc
    say("mixed solve case", o, v, X, seed)
    eps, B = make_system(o, v, X, seed=seed)
    ref = oracle.solve(eps, B, o, max_iter=80, tol=1e-10)
    assert ref.converged
    phases = []
    with exacc.CCSD(eps, B, o, precision=exacc.MIXED_FP32, tol=1e-10, max_iter=80,
                    ladder_group_nvir=group) as cc:
        e, conv, hist = cc.solve(callback=lambda it, E, r: phases.append(cc.phase()[0]))
        t1, t2 = cc.amplitudes()
        _, n64 = cc.phase()
    assert conv and n64 >= 3
    assert phases[0] == 1 and phases[-1] == 0
    dE = abs(e - ref.energy)
    dT = max(np.abs(t1 - ref.t1).max(), np.abs(t2 - ref.t2).max())
    say("  iterations %d (fp32 %d, corrected ladder %d), |dE| %.2e Eh, max|dT| %.2e"
        % (len(hist), phases.count(1) + 1, phases.count(2), dE, dT))
    assert dE <= 1e-7
    assert dT <= 1e-7


@pytest.mark.parametrize("group", [64, 0])
@pytest.mark.parametrize("o,v,X", [(10, 40, 120), (12, 70, 150), (16, 67, 131), (6, 110, 100)])
def test_bf16x3_phase_residual(lib, o, v, X, group):
    """BF16x3 ladder (and FP32 elsewhere), FP64 assembly: agreement with the FP64 oracle at
    the split-BF16 level (each product ~2^-16 relative, FP32 sums: 1e-4 of the largest |S|).
    (6, 110, 100): the ladder contraction has K = P_v = 5995 (odd) over 47 output tiles, so it
    runs split over 5 K slices with a ragged last tile."""
    from paper_2103_08473_amd import exacc
    say("bf16x3 residual case", o, v, X)
    eps, B = make_system(o, v, X, seed=o * 1000 + v, sigma=0.2)
    t1, t2 = make_amplitudes(o, v, seed=7 + o, scale=0.1)
    S1, S2 = residual(eps, build_integrals(B, o), t1, t2)
    with exacc.CCSD(eps, B, o, precision=exacc.MIXED_BF16X3, ladder_group_nvir=group) as cc:
        cc.set_amplitudes(t1, t2)
        g1, g2 = cc.residual()
    scale = max(np.abs(S2).max(), np.abs(S1).max())
    e2 = np.abs(g2 - S2).max() / scale
    e1 = np.abs(g1 - S1).max() / scale
    say("  rel err S1 %.2e S2 %.2e" % (e1, e2))
    assert e1 <= 1e-4 and e2 <= 1e-4


@pytest.mark.parametrize("group", [64, 0])
def test_bf16x3_solve_matches_fp64_oracle(lib, group):
    """Low-precision, defect-corrected and final FP64 phases; the ladder grouped over all
    rows (64) and per row (0)."""
    from paper_2103_08473_amd import exacc
    o, v, X, seed = 6, 40, 120, 2
    eps, B = make_system(o, v, X, seed=seed)
    ref = oracle.solve(eps, B, o, max_iter=80, tol=1e-10)
    with exacc.CCSD(eps, B, o, precision=exacc.MIXED_BF16X3, tol=1e-10, max_iter=80,
                    ladder_group_nvir=group) as cc:
        e, conv, hist = cc.solve()
        t1, t2 = cc.amplitudes()
    dE = abs(e - ref.energy)
    dT = max(np.abs(t1 - ref.t1).max(), np.abs(t2 - ref.t2).max())
    say("  bf16x3 solve: iterations %d, |dE| %.2e Eh, max|dT| %.2e" % (len(hist), dE, dT))
    assert conv and dE <= 1e-7 and dT <= 1e-7


@pytest.mark.parametrize("prec,variant", [("MIXED_BF16X3", "no_correction"), ("MIXED_BF16X3", "ladder_only"),
                                          ("MIXED_FP32", "ladder_only")])
def test_mixed_tail_variants_match_fp64_oracle(lib, prec, variant):
    """The other tails of a mixed solve: without the corrected iterations (full FP64 from the
    switch on), and with the corrected ladder and C term but the ring in FP64, which create
    chooses when the ring part's reference arrays do not fit the HBM budget (as at
    60/540/1800 in device memory).  Both reach the FP64 oracle's converged answer."""
    from paper_2103_08473_amd import exacc
    o, v, X, seed = 6, 40, 120, 2
    p = getattr(exacc, prec)
    eps, B = make_system(o, v, X, seed=seed)
    ref = oracle.solve(eps, B, o, max_iter=80, tol=1e-10)
    opts = dict(precision=p, tol=1e-10, max_iter=80)
    if variant == "no_correction":
        opts["ladder_defect_correction"] = 0
    else:
        full = exacc.memory_estimate(o, v, X, precision=p)
        ladder_only = exacc.memory_estimate(o, v, X, precision=p, hbm_budget_bytes=full - 1)
        assert ladder_only < full     # the ring part is what the smaller budget leaves out
        opts["hbm_budget_bytes"] = ladder_only
    phases = []
    with exacc.CCSD(eps, B, o, **opts) as cc:
        e, conv, hist = cc.solve(callback=lambda it, E, r: phases.append(cc.phase()[0]))
        t1, t2 = cc.amplitudes()
        _, n64 = cc.phase()
    dE = abs(e - ref.energy)
    dT = max(np.abs(t1 - ref.t1).max(), np.abs(t2 - ref.t2).max())
    say("  %s %s: iterations %d (low %d, corrected %d, final FP64 %d), |dE| %.2e Eh, max|dT| %.2e"
        % (prec, variant, len(hist), phases.count(1) + 1, phases.count(2), n64, dE, dT))
    assert conv and n64 >= 3 and phases[0] == 1 and phases[-1] == 0
    assert (2 in phases) == (variant == "ladder_only")
    assert dE <= 1e-7 and dT <= 1e-7

