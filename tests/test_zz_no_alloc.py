"""exacc_df_factors_noalloc (temporaries in the library's static per-GPU array, no
device allocation) against the allocating exacc_df_factors, through the C ABI."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

# floating-point bar of the DF-factor parity tests: the two entry points run the same
# kernels; only the split-K partitioning of a GEMM may differ with the slice width
TOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def plain_inputs(nao, n, X, seed):
    """Hermitian J[Q] (complex), symmetric positive definite V, orthonormal C."""
    rng = np.random.default_rng(seed)
    J = rng.normal(0, 0.1, (X, nao, nao)) + 1j * rng.normal(0, 0.1, (X, nao, nao))
    J = 0.5 * (J + np.conj(J.transpose(0, 2, 1)))
    A = rng.normal(0, 0.3 / np.sqrt(X), (X, X))
    V = np.eye(X) + 0.5 * (A + A.T)
    V = V @ V.T
    Q, _ = np.linalg.qr(rng.normal(size=(nao, nao)) + 1j * rng.normal(size=(nao, nao)))
    return np.ascontiguousarray(Q[:, :n]), np.ascontiguousarray(J), np.ascontiguousarray(V)


def both(nao, n, X, seed):
    import torch
    from paper_2103_08473_amd import exacc
    C, J, V = plain_inputs(nao, n, X, seed)
    Cd, Jd, Vd = (torch.from_numpy(a).cuda() for a in (C, J, V))
    ref, it_ref = exacc.df_factors(Cd, Jd, Vd)
    B = torch.full((X, n, n), complex("nan"), dtype=torch.complex128, device="cuda")
    it = exacc.df_factors_noalloc(Cd, Jd, Vd, B)
    torch.cuda.synchronize()
    ref, B = ref.cpu().numpy(), B.cpu().numpy()
    return ref, B, it_ref, it


def check(nao, n, X, seed):
    say("no-alloc DF factors: nao=%d nspinor=%d naux=%d seed=%d" % (nao, n, X, seed))
    ref, B, it_ref, it = both(nao, n, X, seed)
    err = np.abs(B - ref).max()
    say("  steps %d / %d, max |dB| %.2e" % (it, it_ref, err))
    assert it == it_ref
    assert np.isfinite(B).all()
    assert err <= TOL * max(1.0, np.abs(ref).max())


def test_noalloc_two_calls_second_smaller(lib):
    """Two calls in a row on the shared array, the second with smaller sizes (the array
    keeps the first call's contents)."""
    check(130, 70, 300, seed=1)
    check(40, 30, 100, seed=2)


def test_noalloc_sliced_transform_then_smaller(lib):
    """Sizes whose transform intermediates exceed the array: the spinor rows run in
    slices; then a smaller call."""
    check(250, 150, 300, seed=3)
    check(6, 4, 10, seed=4)


def test_noalloc_rejects_sizes_beyond_the_array(lib):
    """naux = 2000 needs 384 MB of Newton-Schulz matrices: NOMEM before any device work."""
    import torch
    from paper_2103_08473_amd import exacc
    buf = torch.zeros(16, dtype=torch.complex128, device="cuda")
    V = torch.zeros(16, dtype=torch.float64, device="cuda")
    L = exacc.load()
    st = L.exacc_df_factors_noalloc(4, 2, 2000, buf.data_ptr(), buf.data_ptr(), V.data_ptr(),
                                    buf.data_ptr(), None, None)
    assert st == exacc.ERR_NOMEM
    assert b"scratch" in L.exacc_last_error()
