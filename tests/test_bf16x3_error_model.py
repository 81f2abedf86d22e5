"""Error model of the split-BF16 (hi*hi + hi*lo + lo*hi) complex product, emulated on the CPU.

BF16 keeps 8 significant bits.  With hi = bf16(x) and lo = bf16(x - hi),
|x - hi - lo| <= 2^-17 |x| and the dropped lo*lo' term is <= 2^-16 |x||x'|,
so each real product carries a relative error of order 2^-16 ~ 1.5e-5 and a
sum of K products with random signs a relative error ~ 2^-16 (FP32
accumulation adds ~2^-24 sqrt(K)).  The GPU tests bound the BF16x3 residual
by 1e-4 of its largest entry; this test checks that the emulated product of
the same construction (3-multiplication complex form) stays well inside that
bound at the ladder's K, and that plain BF16 would not.
"""
import numpy as np


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float32."""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (b + 0x7FFF + ((b >> 16) & 1)) >> 16 << 16
    return (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)


def split(x):
    hi = bf16_round(x)
    lo = bf16_round(np.asarray(x, np.float32) - hi)
    return hi.astype(np.float64), lo.astype(np.float64)


def gemm_bf16x3(A, B):
    """Complex A @ B with 3-multiplication products of split-BF16 operands."""
    def prod(x, y):
        xh, xl = split(x)
        yh, yl = split(y)
        return xh @ yh + xh @ yl + xl @ yh
    Ar, Ai = A.real.astype(np.float32), A.imag.astype(np.float32)
    Br, Bi = B.real.astype(np.float32), B.imag.astype(np.float32)
    t1, t2 = prod(Ar, Br), prod(Ai, Bi)
    t3 = prod(Ar + Ai, Br + Bi)
    return (t1 - t2) + 1j * (t3 - t1 - t2)


def test_split_is_exact_to_2_pow_minus_16():
    x = np.random.default_rng(0).normal(size=100000).astype(np.float32)
    hi, lo = split(x)
    rel = np.abs(x - hi - lo) / np.abs(x)
    assert rel.max() <= 2.0 ** -16
    assert np.abs(hi - bf16_round(hi)).max() == 0 and np.abs(lo - bf16_round(lo)).max() == 0


def test_bf16x3_product_error_at_ladder_K():
    rng = np.random.default_rng(1)
    M, N, K = 24, 24, 1200
    A = rng.normal(size=(M, K)) + 1j * rng.normal(size=(M, K))
    B = rng.normal(size=(K, N)) + 1j * rng.normal(size=(K, N))
    exact = A @ B
    got = gemm_bf16x3(A, B)
    rel = np.abs(got - exact).max() / np.abs(exact).max()
    plain = (bf16_round(A.real).astype(np.float64) + 1j * bf16_round(A.imag)) @ \
            (bf16_round(B.real).astype(np.float64) + 1j * bf16_round(B.imag))
    rel_plain = np.abs(plain - exact).max() / np.abs(exact).max()
    assert rel < 1e-4 / 5          # well inside the GPU tests' bound
    assert rel_plain > 10 * rel    # the compensation is what buys the accuracy
