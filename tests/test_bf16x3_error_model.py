"""Error model of the split-BF16 (hi*hi + hi*lo + lo*hi) complex product, emulated on the CPU.

BF16 keeps 8 significant bits.  With hi = bf16(x) and lo = bf16(x - hi),
|x - hi - lo| <= 2^-17 |x| and the dropped lo*lo' term is <= 2^-16 |x||x'|,
so each real product carries a relative error of order 2^-16 ~ 1.5e-5 and a
sum of K products with random signs a relative error ~ 2^-16 (FP32
accumulation adds ~2^-24 sqrt(K)).  The GPU tests bound the BF16x3 residual
by 1e-4 of its largest entry.  This test emulates the arithmetic the BF16x3
kernels run: the four-multiplication complex product (re = rr - ii,
im = ri + ir), each real product as three bf16 matrix products issued in the
order lo*hi', hi*lo', hi*hi', one 32-wide k block at a time, every block's dot
product rounded into an FP32 accumulator (the products of two bf16 values are
exact in FP32), and re formed as an FP32 difference at the end.
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


KB = 32  # k values per matrix-core step (v_mfma_f32_16x16x32_bf16)


def gemm_bf16x3_4m(A, B):
    """Complex A @ B as the BF16x3 kernels form it: 4M complex product, per-k-block FP32
    accumulation of the split products lo*hi', hi*lo', hi*hi'."""
    Ar, Ai = (split(A.real.astype(np.float32)), split(A.imag.astype(np.float32)))
    Br, Bi = (split(B.real.astype(np.float32)), split(B.imag.astype(np.float32)))
    M, K = A.shape
    N = B.shape[1]
    accR = np.zeros((M, N), np.float32)
    accN = np.zeros((M, N), np.float32)
    accI = np.zeros((M, N), np.float32)

    def mma3(acc, x, y, k0, k1):
        (xh, xl), (yh, yl) = x, y
        for p, q in ((xl, yh), (xh, yl), (xh, yh)):
            blk = p[:, k0:k1] @ q[k0:k1, :]          # exact: bf16 x bf16 products
            acc = (acc.astype(np.float64) + blk).astype(np.float32)
        return acc

    for k0 in range(0, K, KB):
        k1 = min(K, k0 + KB)
        accR = mma3(accR, Ar, Br, k0, k1)
        accN = mma3(accN, Ai, Bi, k0, k1)
        accI = mma3(accI, Ar, Bi, k0, k1)
        accI = mma3(accI, Ai, Br, k0, k1)
    re = (accR - accN).astype(np.float64)
    return re + 1j * accI.astype(np.float64)


def test_split_is_exact_to_2_pow_minus_16():
    x = np.random.default_rng(0).normal(size=100000).astype(np.float32)
    hi, lo = split(x)
    rel = np.abs(x - hi - lo) / np.abs(x)
    assert rel.max() <= 2.0 ** -16
    assert np.abs(hi - bf16_round(hi)).max() == 0 and np.abs(lo - bf16_round(lo)).max() == 0


def test_bf16x3_product_error_at_ladder_K():
    """K = naux = 1200 (the tile build at 40/360/1200)."""
    rng = np.random.default_rng(1)
    M, N, K = 24, 24, 1200
    A = rng.normal(size=(M, K)) + 1j * rng.normal(size=(M, K))
    B = rng.normal(size=(K, N)) + 1j * rng.normal(size=(K, N))
    exact = A @ B
    got = gemm_bf16x3_4m(A, B)
    rel = np.abs(got - exact).max() / np.abs(exact).max()
    plain = (bf16_round(A.real).astype(np.float64) + 1j * bf16_round(A.imag)) @ \
            (bf16_round(B.real).astype(np.float64) + 1j * bf16_round(B.imag))
    rel_plain = np.abs(plain - exact).max() / np.abs(exact).max()
    assert rel < 1e-4 / 5          # well inside the GPU tests' bound
    assert rel_plain > 10 * rel    # the compensation is what buys the accuracy


def test_bf16x3_product_error_at_contraction_K():
    """A long sum (the ladder contraction runs K = P_v = 64,620 at 40/360/1200; here 8192)
    still stays inside the bound: the FP32 accumulator adds ~2^-24 per k block."""
    rng = np.random.default_rng(2)
    M, N, K = 8, 8, 8192
    A = rng.normal(size=(M, K)) + 1j * rng.normal(size=(M, K))
    B = rng.normal(size=(K, N)) + 1j * rng.normal(size=(K, N))
    exact = A @ B
    rel = np.abs(gemm_bf16x3_4m(A, B) - exact).max() / np.abs(exact).max()
    assert rel < 1e-4 / 5
