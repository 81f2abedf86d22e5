// Complex GEMM-like tensor contraction (GETT) on CDNA4 matrix cores.
//
// One workgroup (4 waves of 64 lanes) owns a BM x BN tile of C; two
// workgroups per CU (two waves per SIMD) hide LDS and barrier latency.
// Operand tiles of BK = 16 complex columns are staged through LDS as three
// real planes, k-major: re, im and re+im, so each 16x16x4 MFMA fragment is
// read with unit stride.  Complex products use the three-multiplication
// (Gauss) form: T1 = re*re, T2 = im*im, T3 = (re+im)(re+im) accumulate in
// three MFMA accumulators and C = (T1 - T2) + i (T3 - T1 - T2) at the end,
// 3 real MFMAs per complex multiply-add instead of 4.  Global loads for the
// next k-tile are issued into registers before the MFMAs of the current one
// (single LDS buffer, register prefetch).  Operand addresses come from the composite
// (outer, inner) index maps of Gett<R>, so permuted and strided tensors are
// contracted in place without transposes in HBM.
#include "common.h"

namespace exacc {

template <typename R>
struct MF;
template <>
struct MF<double> {
  typedef double4_t acc_t;
  __device__ static acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // accumulator element r of a lane holds row lane/16 + 4r, column lane%16
  __device__ static int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct MF<float> {
  typedef float4_t acc_t;
  __device__ static acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // accumulator element r of a lane holds row 4*(lane/16) + r, column lane%16
  __device__ static int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <typename R>
struct C2 {
  R x, y;
};

__device__ __forceinline__ int64_t cmap(int x, int in, int64_t so, int64_t si) {
  const int q = x / in;
  const int r = x - q * in;
  return (int64_t)q * so + (int64_t)r * si;
}

template <typename R>
__device__ __forceinline__ C2<R> ldc(const R* p, int64_t off) {
  // interleaved complex: one aligned 2-element load
  typedef R v2 __attribute__((ext_vector_type(2)));
  v2 t = *reinterpret_cast<const v2*>(p + 2 * off);
  C2<R> c;
  c.x = t.x;
  c.y = t.y;
  return c;
}

template <typename R, int BM, int BN, bool AKF, bool BKF, int KIND>
__global__ __launch_bounds__(256, 2) void gett_kernel(Gett<R> g) {
  constexpr int BK = 16;
  constexpr int LA = BM + 1;  // odd row pitch: conflict-free k-major stores
  constexpr int LB = BN + 1;
  constexpr int NA = BM * BK / 256;  // complex elements per thread per tile
  constexpr int NB = BN * BK / 256;
  constexpr int TM = BM / 32;  // 16x16 blocks per wave along m
  constexpr int TN = BN / 32;
  typedef typename MF<R>::acc_t acc_t;

  __shared__ R sA[3][BK][LA];  // re, im, re + im
  __shared__ R sB[3][BK][LB];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int wm = w & 1, wn = w >> 1;

  const int tiles_m = (g.M + BM - 1) / BM;
  const int bid = blockIdx.x;
  const int tm = bid % tiles_m;
  const int tn = bid / tiles_m;
  const int m0 = tm * BM, n0 = tn * BN;
  const int64_t batch = blockIdx.y;
  const R* __restrict__ A = g.A + 2 * batch * g.a_b;
  const R* __restrict__ B = g.B + 2 * batch * g.b_b;

  const int kb = blockIdx.z * g.kslice;
  const int ke = (g.K - kb) < g.kslice ? g.K : kb + g.kslice;

  // ---- per-thread loader geometry
  int64_t a_off[AKF ? NA : 1];
  bool a_ok[AKF ? NA : 1];
  int a_kk = 0, a_mm = 0, a_kq = 0;
  if (AKF) {
    a_kk = tid % BK;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int m = m0 + tid / BK + 16 * q;
      a_ok[q] = m < g.M;
      a_off[q] = a_ok[q] ? cmap(m, g.m_in, g.a_mo, g.a_mi) : 0;
    }
  } else {
    a_mm = tid % BM;
    a_kq = tid / BM;
    const int m = m0 + a_mm;
    a_ok[0] = m < g.M;
    a_off[0] = a_ok[0] ? cmap(m, g.m_in, g.a_mo, g.a_mi) : 0;
  }
  int64_t b_off[BKF ? NB : 1];
  bool b_ok[BKF ? NB : 1];
  int b_kk = 0, b_nn = 0, b_kq = 0;
  if (BKF) {
    b_kk = tid % BK;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int n = n0 + tid / BK + 16 * q;
      b_ok[q] = n < g.N;
      b_off[q] = b_ok[q] ? cmap(n, g.n_in, g.b_no, g.b_ni) : 0;
    }
  } else {
    b_nn = tid % BN;
    b_kq = tid / BN;
    const int n = n0 + b_nn;
    b_ok[0] = n < g.N;
    b_off[0] = b_ok[0] ? cmap(n, g.n_in, g.b_no, g.b_ni) : 0;
  }

  C2<R> ra[NA], rb[NB];
  const R sa = g.conj_a ? R(-1) : R(1);
  const R sb = g.conj_b ? R(-1) : R(1);

  auto load = [&](int k0) {
    if (AKF) {
      const int k = k0 + a_kk;
      const bool kv = k < ke;
      const int64_t ko = kv ? cmap(k, g.k_in, g.a_ko, g.a_ki) : 0;
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        if (kv && a_ok[q]) {
          ra[q] = ldc(A, a_off[q] + ko);
        } else {
          ra[q].x = R(0);
          ra[q].y = R(0);
        }
      }
    } else {
      constexpr int KS = 256 / BM;
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        const int k = k0 + a_kq + KS * q;
        if (k < ke && a_ok[0]) {
          ra[q] = ldc(A, a_off[0] + cmap(k, g.k_in, g.a_ko, g.a_ki));
        } else {
          ra[q].x = R(0);
          ra[q].y = R(0);
        }
      }
    }
    if (BKF) {
      const int k = k0 + b_kk;
      const bool kv = k < ke;
      const int64_t ko = kv ? cmap(k, g.k_in, g.b_ko, g.b_ki) : 0;
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        if (kv && b_ok[q]) {
          rb[q] = ldc(B, b_off[q] + ko);
        } else {
          rb[q].x = R(0);
          rb[q].y = R(0);
        }
      }
    } else {
      constexpr int KS = 256 / BN;
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int k = k0 + b_kq + KS * q;
        if (k < ke && b_ok[0]) {
          rb[q] = ldc(B, b_off[0] + cmap(k, g.k_in, g.b_ko, g.b_ki));
        } else {
          rb[q].x = R(0);
          rb[q].y = R(0);
        }
      }
    }
  };

  auto store = [&]() {
    if (AKF) {
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        const int m = tid / BK + 16 * q;
        sA[0][a_kk][m] = ra[q].x;
        sA[1][a_kk][m] = sa * ra[q].y;
        sA[2][a_kk][m] = ra[q].x + sa * ra[q].y;
      }
    } else {
      constexpr int KS = 256 / BM;
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        const int k = a_kq + KS * q;
        sA[0][k][a_mm] = ra[q].x;
        sA[1][k][a_mm] = sa * ra[q].y;
        sA[2][k][a_mm] = ra[q].x + sa * ra[q].y;
      }
    }
    if (BKF) {
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int n = tid / BK + 16 * q;
        sB[0][b_kk][n] = rb[q].x;
        sB[1][b_kk][n] = sb * rb[q].y;
        sB[2][b_kk][n] = rb[q].x + sb * rb[q].y;
      }
    } else {
      constexpr int KS = 256 / BN;
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int k = b_kq + KS * q;
        sB[0][k][b_nn] = rb[q].x;
        sB[1][k][b_nn] = sb * rb[q].y;
        sB[2][k][b_nn] = rb[q].x + sb * rb[q].y;
      }
    }
  };

  // accR, accI, accS hold T1 = sum re*re, T2 = sum im*im, T3 = sum (re+im)(re+im)
  acc_t accR[TM][TN], accI[TM][TN], accS[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      accR[i][j] = acc_t{0, 0, 0, 0};
      accI[i][j] = acc_t{0, 0, 0, 0};
      accS[i][j] = acc_t{0, 0, 0, 0};
    }

  const int nk = ke > kb ? (ke - kb + BK - 1) / BK : 0;
  if (nk > 0) {
    load(kb);
    store();
  }
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) load(kb + (kt + 1) * BK);
#pragma unroll
    for (int s = 0; s < BK / 4; ++s) {
      const int kr = 4 * s + (lane >> 4);
      R ar[TM], ai[TM], as[TM], br[TN], bi[TN], bs[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int m = wm * (BM / 2) + 16 * i + (lane & 15);
        ar[i] = sA[0][kr][m];
        ai[i] = sA[1][kr][m];
        as[i] = sA[2][kr][m];
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int n = wn * (BN / 2) + 16 * j + (lane & 15);
        br[j] = sB[0][kr][n];
        bi[j] = sB[1][kr][n];
        bs[j] = sB[2][kr][n];
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          accR[i][j] = MF<R>::mma(ar[i], br[j], accR[i][j]);
          accI[i][j] = MF<R>::mma(ai[i], bi[j], accI[i][j]);
          accS[i][j] = MF<R>::mma(as[i], bs[j], accS[i][j]);
        }
    }
    __syncthreads();
    if (kt + 1 < nk) {
      store();
      __syncthreads();
    }
  }

  // complex result: re = T1 - T2, im = T3 - T1 - T2
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const acc_t t1 = accR[i][j], t2 = accI[i][j];
      accR[i][j] = t1 - t2;
      accI[i][j] = accS[i][j] - t1 - t2;
    }

  // ---- epilogue (output layout of the 16x16 block per MF<R>::row)
  R* __restrict__ Cb = g.C + 2 * batch * g.c_b;
  if (gridDim.z > 1) {  // split-K: raw partial sums, reduced by gett_splitk_reduce
    R* __restrict__ W = g.ws + 2 * (((int64_t)blockIdx.z * gridDim.y + batch) * g.M) * g.N;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int col = n0 + wn * (BN / 2) + 16 * j + (lane & 15);
        if (col >= g.N) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm * (BM / 2) + 16 * i + MF<R>::row(lane, r);
          if (row >= g.M) continue;
          const int64_t off = 2 * ((int64_t)row * g.N + col);
          W[off] = accR[i][j][r];
          W[off + 1] = accI[i][j][r];
        }
      }
    return;
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int col = n0 + wn * (BN / 2) + 16 * j + (lane & 15);
      if (col >= g.N) continue;
      const int64_t co = cmap(col, g.n_in, g.c_no, g.c_ni);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * (BM / 2) + 16 * i + MF<R>::row(lane, r);
        if (row >= g.M) continue;
        const int64_t off = 2 * (co + cmap(row, g.m_in, g.c_mo, g.c_mi));
        const R xr = accR[i][j][r], xi = accI[i][j][r];
        R yr = g.alpha_re * xr - g.alpha_im * xi;
        R yi = g.alpha_re * xi + g.alpha_im * xr;
        if (g.accumulate) {
          yr += Cb[off];
          yi += Cb[off + 1];
        }
        Cb[off] = yr;
        Cb[off + 1] = yi;
      }
    }
}

// C[b](m, n) = alpha * sum_z ws[z][b][m][n] (+ C), fixed summation order.
template <typename R>
__global__ __launch_bounds__(256) void gett_splitk_reduce(Gett<R> g, int nz, int nb) {
  const int64_t MN = (int64_t)g.M * g.N, tot = MN * nb;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < tot; t += (int64_t)gridDim.x * 256) {
    const int64_t b = t / MN, mn = t - b * MN;
    const int m = (int)(mn / g.N), n = (int)(mn - (int64_t)m * g.N);
    R sr = 0, si = 0;
    for (int z = 0; z < nz; ++z) {
      const R* w = g.ws + 2 * (((int64_t)z * nb + b) * MN + mn);
      sr += w[0];
      si += w[1];
    }
    R* c = g.C + 2 * (b * g.c_b + cmap(m, g.m_in, g.c_mo, g.c_mi) + cmap(n, g.n_in, g.c_no, g.c_ni));
    R yr = g.alpha_re * sr - g.alpha_im * si;
    R yi = g.alpha_re * si + g.alpha_im * sr;
    if (g.accumulate) {
      yr += c[0];
      yi += c[1];
    }
    c[0] = yr;
    c[1] = yi;
  }
}

static thread_local void* g_ws = nullptr;
static thread_local size_t g_ws_bytes = 0;
void set_gett_workspace(void* p, size_t bytes) {
  g_ws = p;
  g_ws_bytes = bytes;
}

template <typename R, int BM, int BN, int KIND>
static void launch_cfg(const Gett<R>& g, hipStream_t s) {
  const int tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
  const bool akf = (g.a_ki == 1) || !(g.a_mi == 1);
  const bool bkf = (g.b_ki == 1) || !(g.b_ni == 1);
  for (int64_t b0 = 0; b0 < g.nbatch; b0 += 65535) {
    Gett<R> h = g;
    const int nb = (int)((g.nbatch - b0) < 65535 ? (g.nbatch - b0) : 65535);
    h.A = g.A + 2 * b0 * g.a_b;
    h.B = g.B + 2 * b0 * g.b_b;
    h.C = g.C + 2 * b0 * g.c_b;
    // split K when the output alone gives too few workgroups to fill the chip
    int nz = 1;
    h.kslice = g.K > 0 ? g.K : 1;
    const int64_t wgs = (int64_t)tiles * nb;
    if (g_ws && wgs < 1024 && g.K >= 1024) {
      int64_t want = (1024 + wgs - 1) / wgs;
      want = want < (g.K + 255) / 256 ? want : (g.K + 255) / 256;  // >= 256 k per slice
      const int64_t per = (int64_t)g.M * g.N * nb * 2 * (int64_t)sizeof(R);
      const int64_t cap = per > 0 ? (int64_t)(g_ws_bytes / per) : 0;
      if (want > cap) want = cap;
      if (want > 1024) want = 1024;
      if (want >= 2) {
        int64_t ks = (g.K + want - 1) / want;
        ks = (ks + 15) / 16 * 16;
        nz = (int)((g.K + ks - 1) / ks);
        h.kslice = (int)ks;
        h.ws = (R*)g_ws;
      }
    }
    dim3 grid(tiles, nb, nz), block(256);
    if (akf && bkf)
      hipLaunchKernelGGL((gett_kernel<R, BM, BN, true, true, KIND>), grid, block, 0, s, h);
    else if (akf)
      hipLaunchKernelGGL((gett_kernel<R, BM, BN, true, false, KIND>), grid, block, 0, s, h);
    else if (bkf)
      hipLaunchKernelGGL((gett_kernel<R, BM, BN, false, true, KIND>), grid, block, 0, s, h);
    else
      hipLaunchKernelGGL((gett_kernel<R, BM, BN, false, false, KIND>), grid, block, 0, s, h);
    HIPCHECK(hipGetLastError());
    if (nz > 1) {
      const int64_t tot = (int64_t)g.M * g.N * nb;
      int64_t blocks = (tot + 255) / 256;
      if (blocks > 65535 * 8) blocks = 65535 * 8;
      hipLaunchKernelGGL(gett_splitk_reduce<R>, dim3((unsigned)blocks), dim3(256), 0, s, h, nz, nb);
      HIPCHECK(hipGetLastError());
    }
  }
}


// ---------------------------------------------------------------------------
// BF16x3 complex GETT for operands that are K-contiguous FP32 complex (the
// particle-ladder tile build and contraction and the ring contractions in the
// BF16x3 precision mode).  Each FP32 value x is split as hi = bf16(x),
// lo = bf16(x - hi); a real product is hi*hi' + hi*lo' + lo*hi' (lo*lo'
// dropped), accumulated in FP32 by v_mfma_f32_16x16x32_bf16.  The loader splits
// re and im of each operand into four bf16 planes in LDS ([plane][row][k], k
// contiguous: one 16-byte read per lane per fragment).  Complex products take
// the four-multiplication form here (3 x 4 = 12 MFMAs per 16x16 block per
// k-step of 32): with four planes instead of six the LDS bytes read per MFMA
// halve, which is what bounds this kernel.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void split_bf16(float x, unsigned short& hi, unsigned short& lo) {
  const __bf16 h = (__bf16)x;                 // round to nearest even
  const __bf16 l = (__bf16)(x - (float)h);
  hi = __builtin_bit_cast(unsigned short, h);
  lo = __builtin_bit_cast(unsigned short, l);
}

__device__ __forceinline__ float4_t mma3(bf16x8_t ah, bf16x8_t al, bf16x8_t bh, bf16x8_t bl,
                                         float4_t c) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
}

template <int KIND>
__global__ __launch_bounds__(256, 2) void gett_bf16x3_kernel(Gett<float> g) {
  constexpr int BM = 64, BN = 64, BK = 32;
  constexpr int PK = BK + 8;  // row pitch in bf16 (16-byte aligned rows)
  // planes: 0 re_hi, 1 re_lo, 2 im_hi, 3 im_lo
  __shared__ __attribute__((aligned(16))) unsigned short sA[4][BM][PK];
  __shared__ __attribute__((aligned(16))) unsigned short sB[4][BN][PK];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w & 1, wn = w >> 1;
  const int tiles_m = (g.M + BM - 1) / BM;
  const int tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
  const int m0 = tm * BM, n0 = tn * BN;
  const int64_t batch = blockIdx.y;
  const float* __restrict__ A = g.A + 2 * batch * g.a_b;
  const float* __restrict__ B = g.B + 2 * batch * g.b_b;
  const int kb = blockIdx.z * g.kslice;
  const int ke = (g.K - kb) < g.kslice ? g.K : kb + g.kslice;

  // loader: thread handles k pair (2*(tid%16), +1) of rows tid/16 + 16*q, q < 4
  const int kp = 2 * (tid % 16);
  int64_t aoff[4], boff[4];
  bool aok[4], bok[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int m = m0 + tid / 16 + 16 * q, n = n0 + tid / 16 + 16 * q;
    aok[q] = m < g.M;
    bok[q] = n < g.N;
    aoff[q] = aok[q] ? cmap(m, g.m_in, g.a_mo, g.a_mi) : 0;
    boff[q] = bok[q] ? cmap(n, g.n_in, g.b_no, g.b_ni) : 0;
  }
  typedef float f4v __attribute__((ext_vector_type(4)));
  f4v ra[4], rb[4];
  const float sa = g.conj_a ? -1.f : 1.f, sb = g.conj_b ? -1.f : 1.f;
  auto load = [&](int k0) {
    const int k = k0 + kp;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      // two consecutive complex (k, k+1); K-contiguous operands, k even, K may be odd
      f4v va = {0.f, 0.f, 0.f, 0.f}, vb = {0.f, 0.f, 0.f, 0.f};
      if (aok[q]) {
        if (k + 1 < ke) {
          va = *reinterpret_cast<const f4v*>(A + 2 * (aoff[q] + k));
        } else if (k < ke) {
          va.x = A[2 * (aoff[q] + k)];
          va.y = A[2 * (aoff[q] + k) + 1];
        }
      }
      if (bok[q]) {
        if (k + 1 < ke) {
          vb = *reinterpret_cast<const f4v*>(B + 2 * (boff[q] + k));
        } else if (k < ke) {
          vb.x = B[2 * (boff[q] + k)];
          vb.y = B[2 * (boff[q] + k) + 1];
        }
      }
      ra[q] = va;
      rb[q] = vb;
    }
  };
  auto put = [&](unsigned short (*s)[BM][PK], int row, f4v v, float sg) {
    // v = (re0, im0, re1, im1) at k = kp, kp + 1
    unsigned short h0, l0, h1, l1;
    split_bf16(v.x, h0, l0);
    split_bf16(v.z, h1, l1);
    *reinterpret_cast<unsigned int*>(&s[0][row][kp]) = h0 | ((unsigned)h1 << 16);
    *reinterpret_cast<unsigned int*>(&s[1][row][kp]) = l0 | ((unsigned)l1 << 16);
    split_bf16(sg * v.y, h0, l0);
    split_bf16(sg * v.w, h1, l1);
    *reinterpret_cast<unsigned int*>(&s[2][row][kp]) = h0 | ((unsigned)h1 << 16);
    *reinterpret_cast<unsigned int*>(&s[3][row][kp]) = l0 | ((unsigned)l1 << 16);
  };
  auto store = [&]() {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      put(sA, tid / 16 + 16 * q, ra[q], sa);
      put(sB, tid / 16 + 16 * q, rb[q], sb);
    }
  };

  // accR = sum re*re - im*im, accI = sum re*im + im*re for the wave's 2x2 16x16 blocks;
  // -im*im is accumulated as (-im_A) * im_B via a negated-A pass
  float4_t accR[2][2], accN[2][2], accI[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      accR[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
      accN[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
      accI[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
    }

  const int nk = ke > kb ? (ke - kb + BK - 1) / BK : 0;
  if (nk > 0) {
    load(kb);
    store();
  }
  __syncthreads();
  const int kq = 8 * (lane >> 4);  // this lane's 8 consecutive k in a fragment
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) load(kb + (kt + 1) * BK);
    bf16x8_t arh[2], arl[2], aih[2], ail[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int r = wm * 32 + 16 * i + (lane & 15);
      arh[i] = *reinterpret_cast<const bf16x8_t*>(&sA[0][r][kq]);
      arl[i] = *reinterpret_cast<const bf16x8_t*>(&sA[1][r][kq]);
      aih[i] = *reinterpret_cast<const bf16x8_t*>(&sA[2][r][kq]);
      ail[i] = *reinterpret_cast<const bf16x8_t*>(&sA[3][r][kq]);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = wn * 32 + 16 * j + (lane & 15);
      const bf16x8_t brh = *reinterpret_cast<const bf16x8_t*>(&sB[0][c][kq]);
      const bf16x8_t brl = *reinterpret_cast<const bf16x8_t*>(&sB[1][c][kq]);
      const bf16x8_t bih = *reinterpret_cast<const bf16x8_t*>(&sB[2][c][kq]);
      const bf16x8_t bil = *reinterpret_cast<const bf16x8_t*>(&sB[3][c][kq]);
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        accR[i][j] = mma3(arh[i], arl[i], brh, brl, accR[i][j]);
        accN[i][j] = mma3(aih[i], ail[i], bih, bil, accN[i][j]);
        accI[i][j] = mma3(arh[i], arl[i], bih, bil, accI[i][j]);
        accI[i][j] = mma3(aih[i], ail[i], brh, brl, accI[i][j]);
      }
    }
    __syncthreads();
    if (kt + 1 < nk) {
      store();
      __syncthreads();
    }
  }

  // complex result re = accR - accN, im = accI; 16x16 f32 layout: row 4*(lane/16)+r
  float* __restrict__ Cb = g.C + 2 * batch * g.c_b;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn * 32 + 16 * j + (lane & 15);
      if (col >= g.N) continue;
      const int64_t co = cmap(col, g.n_in, g.c_no, g.c_ni);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 32 + 16 * i + 4 * (lane >> 4) + r;
        if (row >= g.M) continue;
        const float xr = accR[i][j][r] - accN[i][j][r], xi = accI[i][j][r];
        const int64_t off = 2 * (co + cmap(row, g.m_in, g.c_mo, g.c_mi));
        float yr = g.alpha_re * xr - g.alpha_im * xi;
        float yi = g.alpha_re * xi + g.alpha_im * xr;
        if (g.accumulate) {
          yr += Cb[off];
          yi += Cb[off + 1];
        }
        Cb[off] = yr;
        Cb[off + 1] = yi;
      }
    }
}

template <int KIND>
static void launch_bf16x3(const Gett<float>& g, hipStream_t s) {
  const int tiles = ((g.M + 63) / 64) * ((g.N + 63) / 64);
  for (int64_t b0 = 0; b0 < g.nbatch; b0 += 65535) {
    Gett<float> h = g;
    const int nb = (int)((g.nbatch - b0) < 65535 ? (g.nbatch - b0) : 65535);
    h.A = g.A + 2 * b0 * g.a_b;
    h.B = g.B + 2 * b0 * g.b_b;
    h.C = g.C + 2 * b0 * g.c_b;
    h.kslice = g.K > 0 ? g.K : 1;
    h.ws = nullptr;
    hipLaunchKernelGGL((gett_bf16x3_kernel<KIND>), dim3(tiles, nb, 1), dim3(256), 0, s, h);
    HIPCHECK(hipGetLastError());
  }
}

template <typename R>
void launch_gett(const Gett<R>& g, int kind_in, hipStream_t s) {
  int kind = kind_in;
  if (g.M <= 0 || g.N <= 0 || g.nbatch <= 0) return;
  if ((int64_t)((g.M + 63) / 64) * ((g.N + 63) / 64) > 0x7fffffffLL)
    raise(-1, "contraction too large for one launch");
  // BF16x3 kinds: only for FP32 operands that are K-contiguous in both A and B
  // (16-byte loads of two complex values: even row strides and 16-byte aligned bases)
  const bool kcontig = g.k_in == g.K && g.a_ki == 1 && g.b_ki == 1 && g.a_mo % 2 == 0 &&
                       g.a_mi % 2 == 0 && g.b_no % 2 == 0 && g.b_ni % 2 == 0 &&
                       g.a_b % 2 == 0 && g.b_b % 2 == 0 &&
                       reinterpret_cast<uintptr_t>(g.A) % 16 == 0 &&
                       reinterpret_cast<uintptr_t>(g.B) % 16 == 0;
  if (kind == GETT_LADDER_BUILD_BF16X3 || kind == GETT_LADDER_CONTRACT_BF16X3 ||
      kind == GETT_RING_BF16X3) {
    if constexpr (sizeof(R) == sizeof(float)) {
      if (kcontig) {
        if (kind == GETT_LADDER_BUILD_BF16X3)
          launch_bf16x3<GETT_LADDER_BUILD_BF16X3>(g, s);
        else if (kind == GETT_LADDER_CONTRACT_BF16X3)
          launch_bf16x3<GETT_LADDER_CONTRACT_BF16X3>(g, s);
        else
          launch_bf16x3<GETT_RING_BF16X3>(g, s);
        return;
      }
    }
    kind = (kind == GETT_LADDER_BUILD_BF16X3)     ? GETT_LADDER_BUILD
           : (kind == GETT_LADDER_CONTRACT_BF16X3) ? GETT_LADDER_CONTRACT
                                                   : GETT_RING;
  }
  switch (kind) {
    case GETT_LADDER_BUILD: launch_cfg<R, 64, 64, GETT_LADDER_BUILD>(g, s); break;
    case GETT_LADDER_CONTRACT: launch_cfg<R, 64, 64, GETT_LADDER_CONTRACT>(g, s); break;
    case GETT_RING: launch_cfg<R, 64, 64, GETT_RING>(g, s); break;
    default: launch_cfg<R, 64, 64, GETT_GENERIC>(g, s); break;
  }
}

template void launch_gett<double>(const Gett<double>&, int, hipStream_t);
template void launch_gett<float>(const Gett<float>&, int, hipStream_t);

}  // namespace exacc
