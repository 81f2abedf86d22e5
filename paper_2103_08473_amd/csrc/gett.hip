// Complex GEMM-like tensor contraction (GETT) on CDNA4 matrix cores.
//
// One workgroup (4 waves of 64 lanes) owns a BM x BN tile of C; two
// workgroups per CU (two waves per SIMD) hide LDS and barrier latency.
// Operand tiles of BK complex columns (16 in production) are staged through
// LDS as two real planes, k-major (re, im), so each 16x16x4 MFMA fragment is
// read with unit stride; the re+im operand of the Gauss product is formed in
// registers.  Complex products use the three-multiplication (Gauss) form:
// T1 = re*re, T2 = im*im, T3 = (re+im)(re+im) accumulate in three MFMA
// accumulators and C = (T1 - T2) + i (T3 - T1 - T2) at the end, 3 real MFMAs
// per complex multiply-add instead of 4.  Global loads for the next k-tile
// are issued into registers before the MFMAs of the current one and written
// to the second LDS buffer after them (one barrier per k-tile).  Operand
// addresses come from the composite (outer, inner) index maps of Gett<R>, so
// permuted and strided tensors are contracted in place without transposes in
// HBM.
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

template <typename R, int BM, int BN, int BK, bool DB, bool AKF, bool BKF, int KIND>
__global__ __launch_bounds__(256, 2) void gett_kernel(Gett<R> g) {
  constexpr int NBUF = DB ? 2 : 1;  // DB: double-buffered LDS, one barrier per k-tile
  constexpr int RS = 256 / BK;      // tile rows per loader pass (k-fast operands)
  constexpr int LA = BM + 1;  // odd row pitch: conflict-free k-major stores
  constexpr int LB = BN + 1;
  constexpr int NA = BM * BK / 256;  // complex elements per thread per tile
  constexpr int NB = BN * BK / 256;
  constexpr int TM = BM / 32;  // 16x16 blocks per wave along m
  constexpr int TN = BN / 32;
  typedef typename MF<R>::acc_t acc_t;

  // [buffer][re, im][k][m]: two buffers, one barrier per k-tile
  __shared__ R sA[NBUF][2][BK][LA];
  __shared__ R sB[NBUF][2][BK][LB];

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

  // ---- per-thread loader geometry.  Rows past M (columns past N) are clamped
  // to the last valid one: they feed only output rows (columns) that are never
  // stored, so no load needs a row check.  Only the ragged last k-tile checks k.
  int64_t a_off[AKF ? NA : 1];
  int a_kk = 0, a_mm = 0, a_kq = 0;
  if (AKF) {
    a_kk = tid % BK;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int m = min(m0 + tid / BK + RS * q, g.M - 1);
      a_off[q] = cmap(m, g.m_in, g.a_mo, g.a_mi);
    }
  } else {
    a_mm = tid % BM;
    a_kq = tid / BM;
    a_off[0] = cmap(min(m0 + a_mm, g.M - 1), g.m_in, g.a_mo, g.a_mi);
  }
  int64_t b_off[BKF ? NB : 1];
  int b_kk = 0, b_nn = 0, b_kq = 0;
  if (BKF) {
    b_kk = tid % BK;
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int n = min(n0 + tid / BK + RS * q, g.N - 1);
      b_off[q] = cmap(n, g.n_in, g.b_no, g.b_ni);
    }
  } else {
    b_nn = tid % BN;
    b_kq = tid / BN;
    b_off[0] = cmap(min(n0 + b_nn, g.N - 1), g.n_in, g.b_no, g.b_ni);
  }

  C2<R> ra[NA], rb[NB];
  const R sa = g.conj_a ? R(-1) : R(1);
  const R sb = g.conj_b ? R(-1) : R(1);

  // CHECK: the k-tile may be ragged (k >= ke reads as zero)
  auto load_t = [&](int k0, auto check) {
    constexpr bool CHECK = decltype(check)::value;
    if (AKF) {
      const int k = k0 + a_kk;
      const bool kv = !CHECK || k < ke;
      const int64_t ko = kv ? cmap(k, g.k_in, g.a_ko, g.a_ki) : 0;
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        if (kv) {
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
        if (!CHECK || k < ke) {
          ra[q] = ldc(A, a_off[0] + cmap(k, g.k_in, g.a_ko, g.a_ki));
        } else {
          ra[q].x = R(0);
          ra[q].y = R(0);
        }
      }
    }
    if (BKF) {
      const int k = k0 + b_kk;
      const bool kv = !CHECK || k < ke;
      const int64_t ko = kv ? cmap(k, g.k_in, g.b_ko, g.b_ki) : 0;
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        if (kv) {
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
        if (!CHECK || k < ke) {
          rb[q] = ldc(B, b_off[0] + cmap(k, g.k_in, g.b_ko, g.b_ki));
        } else {
          rb[q].x = R(0);
          rb[q].y = R(0);
        }
      }
    }
  };
  auto load = [&](int k0) {
    if (k0 + BK <= ke)
      load_t(k0, std::false_type{});
    else
      load_t(k0, std::true_type{});
  };

  auto store = [&](int buf) {
    if (AKF) {
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        const int m = tid / BK + RS * q;
        sA[buf][0][a_kk][m] = ra[q].x;
        sA[buf][1][a_kk][m] = sa * ra[q].y;
      }
    } else {
      constexpr int KS = 256 / BM;
#pragma unroll
      for (int q = 0; q < NA; ++q) {
        const int k = a_kq + KS * q;
        sA[buf][0][k][a_mm] = ra[q].x;
        sA[buf][1][k][a_mm] = sa * ra[q].y;
      }
    }
    if (BKF) {
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int n = tid / BK + RS * q;
        sB[buf][0][b_kk][n] = rb[q].x;
        sB[buf][1][b_kk][n] = sb * rb[q].y;
      }
    } else {
      constexpr int KS = 256 / BN;
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int k = b_kq + KS * q;
        sB[buf][0][k][b_nn] = rb[q].x;
        sB[buf][1][k][b_nn] = sb * rb[q].y;
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
    store(0);
  }
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = DB ? (kt & 1) : 0;
    if (kt + 1 < nk) load(kb + (kt + 1) * BK);
#pragma unroll
    for (int s = 0; s < BK / 4; ++s) {
      const int kr = 4 * s + (lane >> 4);
      R ar[TM], ai[TM], as[TM], br[TN], bi[TN], bs[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int m = wm * (BM / 2) + 16 * i + (lane & 15);
        ar[i] = sA[cur][0][kr][m];
        ai[i] = sA[cur][1][kr][m];
        as[i] = ar[i] + ai[i];
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int n = wn * (BN / 2) + 16 * j + (lane & 15);
        br[j] = sB[cur][0][kr][n];
        bi[j] = sB[cur][1][kr][n];
        bs[j] = br[j] + bi[j];
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
    if (DB) {
      // the other buffer was last read before the previous barrier
      if (kt + 1 < nk) store(cur ^ 1);
      __syncthreads();
    } else {
      __syncthreads();
      if (kt + 1 < nk) {
        store(0);
        __syncthreads();
      }
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
    // long K: slices of >= 256 k up to ~1024 workgroups; outputs of a few tiles (small
    // problems, whose time is the serial k-loop of each workgroup): slices of >= 32 k up to
    // ~256 workgroups
    const bool long_k = wgs < 1024 && g.K >= 1024, few_tiles = wgs < 128 && g.K >= 64;
    if (g_ws && (long_k || few_tiles)) {
      const int64_t kmin = long_k ? 256 : 32;
      const int64_t per = (int64_t)g.M * g.N * nb * 2 * (int64_t)sizeof(R);
      const int64_t cap = per > 0 ? (int64_t)(g_ws_bytes / per) : 0;
      int64_t zmax = (g.K + kmin - 1) / kmin;
      if (zmax > cap) zmax = cap;
      if (zmax > 1024) zmax = 1024;
      int64_t want = 1;
      if (few_tiles && !long_k) {
        want = (256 + wgs - 1) / wgs;
      } else {
        // whole rounds of workgroups (two per CU, 512 at a time): nz slices take
        // ceil(wgs nz / 512) rounds of K / nz each; the smallest nz within 2% of the best
        // rounds / nz
        auto cost = [&](int64_t z) { return (double)((wgs * z + 511) / 512) / (double)z; };
        double best = cost(1);
        for (int64_t z = 2; z <= zmax; ++z) best = cost(z) < best ? cost(z) : best;
        while (want < zmax && cost(want) > 1.02 * best) ++want;
      }
      if (want > zmax) want = zmax;
      if (want >= 2) {
        int64_t ks = (g.K + want - 1) / want;
        ks = (ks + 31) / 32 * 32;  // a multiple of every BK
        nz = (int)((g.K + ks - 1) / ks);
        h.kslice = (int)ks;
        h.ws = (R*)g_ws;
      }
    }
    dim3 grid(tiles, nb, nz), block(256);
    // FP64: BK = 32, one LDS buffer (two barriers per 96 MFMAs); FP32: BK = 16,
    // two buffers.  Both fill 65 KB (FP64) / 33 KB (FP32) of LDS per workgroup.
    constexpr int BK = sizeof(R) == 8 ? 32 : 16;
    constexpr bool DB = sizeof(R) != 8;
    if (akf && bkf)
      hipLaunchKernelGGL((gett_kernel<R, BM, BN, BK, DB, true, true, KIND>), grid, block, 0, s, h);
    else if (akf)
      hipLaunchKernelGGL((gett_kernel<R, BM, BN, BK, DB, true, false, KIND>), grid, block, 0, s, h);
    else if (bkf)
      hipLaunchKernelGGL((gett_kernel<R, BM, BN, BK, DB, false, true, KIND>), grid, block, 0, s, h);
    else
      hipLaunchKernelGGL((gett_kernel<R, BM, BN, BK, DB, false, false, KIND>), grid, block, 0, s, h);
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

// Split two FP32 values into packed bf16 pairs: hi = bf16(x) (round to
// nearest even), lo = bf16(x - hi); element 0 in the low half of each word.
typedef float f2v_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void split_bf16x2(float x0, float x1, unsigned& hi, unsigned& lo) {
  const f2v_t x = {x0, x1};
  hi = __builtin_bit_cast(unsigned, __builtin_convertvector(x, bf16x2_t));
  const f2v_t r = {x0 - __builtin_bit_cast(float, hi << 16),
                   x1 - __builtin_bit_cast(float, hi & 0xffff0000u)};
  lo = __builtin_bit_cast(unsigned, __builtin_convertvector(r, bf16x2_t));
}

__device__ __forceinline__ float4_t mma3(bf16x8_t ah, bf16x8_t al, bf16x8_t bh, bf16x8_t bl,
                                         float4_t c) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
}

// Workgroup index after an optional XCD-aware renumbering: workgroups are
// handed to the 8 XCDs round-robin by id and each XCD has its own L2, so
// consecutive ids (the m-tiles that share one n-panel of B) land on different
// L2s.  The renumbering gives each XCD a contiguous run of logical ids; it is
// a bijection of [0, n), so only the L2 hit rate depends on it.
__device__ __forceinline__ int xcd_tile(int id, int n) {
  const int per = (n + 7) / 8, tall = n % 8 == 0 ? 8 : n % 8;
  const int x = id % 8, l = id / 8;
  return x < tall ? x * per + l : tall * per + (x - tall) * (per - 1) + l;
}

// BM x BN workgroup tile, (BM/32) x (BN/32) waves of 32 x 32 outputs each.  A16: operand
// rows and bases are 16-byte aligned (one 16-byte load per k pair); otherwise each k pair
// is read as two 8-byte complex values.
template <int KIND, int BM, int BN, bool XCD, bool A16>
__global__ __launch_bounds__(64 * (BM / 32) * (BN / 32), (BM * BN == 64 * 64) ? 2 : 1) void
gett_bf16x3_kernel(Gett<float> g) {
  constexpr int BK = 32;
  constexpr int WM = BM / 32, T = 64 * (BM / 32) * (BN / 32);
  constexpr int QA = BM * 16 / T, QB = BN * 16 / T, RS = T / 16;
  constexpr int PK = BK + 8;  // row pitch in bf16 (16-byte aligned rows)
  // planes: 0 re_hi, 1 re_lo, 2 im_hi, 3 im_lo
  __shared__ __attribute__((aligned(16))) unsigned short sA[4][BM][PK];
  __shared__ __attribute__((aligned(16))) unsigned short sB[4][BN][PK];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w % WM, wn = w / WM;
  const int tiles_m = (g.M + BM - 1) / BM;
  const int tile = XCD ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
  const int tm = tile % tiles_m, tn = tile / tiles_m;
  const int m0 = tm * BM, n0 = tn * BN;
  const int64_t batch = blockIdx.y;
  const float* __restrict__ A = g.A + 2 * batch * g.a_b;
  const float* __restrict__ B = g.B + 2 * batch * g.b_b;
  const int kb = blockIdx.z * g.kslice;
  const int ke = (g.K - kb) < g.kslice ? g.K : kb + g.kslice;

  // loader: thread handles the k pair (kp, kp + 1), kp = 2*(tid%16), of tile
  // rows tid/16 + RS*q.  Rows past M (columns past N) are clamped to the last
  // valid one: they feed only output rows (columns) that are never stored, so
  // their values do not matter, and no load needs a row check.
  const int kp = 2 * (tid % 16);
  const float* pa[QA];
  const float* pb[QB];
#pragma unroll
  for (int q = 0; q < QA; ++q) {
    const int m = min(m0 + tid / 16 + RS * q, g.M - 1);
    pa[q] = A + 2 * (cmap(m, g.m_in, g.a_mo, g.a_mi) + kb + kp);
  }
#pragma unroll
  for (int q = 0; q < QB; ++q) {
    const int n = min(n0 + tid / 16 + RS * q, g.N - 1);
    pb[q] = B + 2 * (cmap(n, g.n_in, g.b_no, g.b_ni) + kb + kp);
  }
  typedef float f4v __attribute__((ext_vector_type(4)));
  f4v ra[QA], rb[QB];
  const int klen = ke - kb;
  auto ld2 = [](const float* p) -> f4v {  // complex values k, k + 1 at p
    if constexpr (A16) {
      return *reinterpret_cast<const f4v*>(p);
    } else {
      const f2v_t u = *reinterpret_cast<const f2v_t*>(p);
      const f2v_t w = *reinterpret_cast<const f2v_t*>(p + 2);
      return f4v{u.x, u.y, w.x, w.y};
    }
  };
  auto ld = [&](const float* p, int k0) {
    // two consecutive complex (k, k+1) from k0 + kp; past the slice reads as zero
    const int k = k0 + kp;
    f4v v = {0.f, 0.f, 0.f, 0.f};
    if (k + 1 < klen) {
      v = ld2(p + 2 * k0);
    } else if (k < klen) {
      v.x = p[2 * k0];
      v.y = p[2 * k0 + 1];
    }
    return v;
  };
  auto load = [&](int k0) {  // k0: offset of the tile from kb
    if (k0 + BK <= klen) {   // whole tile inside the slice
#pragma unroll
      for (int q = 0; q < QA; ++q) ra[q] = ld2(pa[q] + 2 * k0);
#pragma unroll
      for (int q = 0; q < QB; ++q) rb[q] = ld2(pb[q] + 2 * k0);
    } else {  // ragged last tile (K may be odd)
#pragma unroll
      for (int q = 0; q < QA; ++q) ra[q] = ld(pa[q], k0);
#pragma unroll
      for (int q = 0; q < QB; ++q) rb[q] = ld(pb[q], k0);
    }
  };
  // sign bits that conjugate an operand (negate both bf16 halves of its imaginary planes)
  const unsigned sga = g.conj_a ? 0x80008000u : 0u, sgb = g.conj_b ? 0x80008000u : 0u;
  auto put = [&](auto& sm, int row, f4v v, unsigned sg) {
    // v = (re0, im0, re1, im1) at k = kp, kp + 1
    unsigned h, l;
    split_bf16x2(v.x, v.z, h, l);
    *reinterpret_cast<unsigned*>(&sm[0][row][kp]) = h;
    *reinterpret_cast<unsigned*>(&sm[1][row][kp]) = l;
    split_bf16x2(v.y, v.w, h, l);
    *reinterpret_cast<unsigned*>(&sm[2][row][kp]) = h ^ sg;
    *reinterpret_cast<unsigned*>(&sm[3][row][kp]) = l ^ sg;
  };
  auto store = [&]() {
#pragma unroll
    for (int q = 0; q < QA; ++q) put(sA, tid / 16 + RS * q, ra[q], sga);
#pragma unroll
    for (int q = 0; q < QB; ++q) put(sB, tid / 16 + RS * q, rb[q], sgb);
  };

  // for the wave's 2x2 16x16 blocks: accR = sum re*re', accN = sum im*im',
  // accI = sum re*im' + im*re'
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
    load(0);
    store();
  }
  __syncthreads();
  const int kq = 8 * (lane >> 4);  // this lane's 8 consecutive k in a fragment
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) load((kt + 1) * BK);
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
  if (gridDim.z > 1) {  // split-K: raw partial sums, reduced by gett_splitk_reduce
    float* __restrict__ W = g.ws + 2 * (((int64_t)blockIdx.z * gridDim.y + batch) * g.M) * g.N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int col = n0 + wn * 32 + 16 * j + (lane & 15);
        if (col >= g.N) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm * 32 + 16 * i + 4 * (lane >> 4) + r;
          if (row >= g.M) continue;
          const int64_t off = 2 * ((int64_t)row * g.N + col);
          W[off] = accR[i][j][r] - accN[i][j][r];
          W[off + 1] = accI[i][j][r];
        }
      }
    return;
  }
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

// ---------------------------------------------------------------------------
// BF16x3 GEMM on pre-split operands.  An operand that many launches read (the
// virtual-virtual density-fitting rows of the particle-ladder tile build) is
// split once into bf16 planes in HBM, so the GEMM loader copies bytes to LDS
// and does no conversion.  Split layout of a row r with K complex values:
// Kp = K rounded up to a multiple of 32 (zero tail); block kb of 8 k values is
// 32 bf16 at r*4*Kp + 32*kb, planes re_hi, re_lo, im_hi, im_lo of 8 k each.
// The split is the same one the loader of gett_bf16x3_kernel applies, and the
// MFMA sequence is the same, so both kernels give bitwise-equal results.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void split_rows_kernel(const float* __restrict__ src, int64_t rows,
                                                         int64_t group, int64_t group_stride,
                                                         int64_t row_stride, int K, int Kp,
                                                         unsigned short* __restrict__ dst) {
  typedef unsigned u4v __attribute__((ext_vector_type(4)));
  const int nkb = Kp / 8;
  const int64_t tot = rows * nkb;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < tot; t += (int64_t)gridDim.x * 256) {
    const int64_t r = t / nkb;
    const int kb = (int)(t - r * nkb);
    const float* p = src + 2 * ((r / group) * group_stride + (r % group) * row_stride);
    float re[8], im[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = 8 * kb + j;
      re[j] = k < K ? p[2 * k] : 0.f;
      im[j] = k < K ? p[2 * k + 1] : 0.f;
    }
    u4v rh, rl, ih, il;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      unsigned h, l;
      split_bf16x2(re[2 * j], re[2 * j + 1], h, l);
      rh[j] = h;
      rl[j] = l;
      split_bf16x2(im[2 * j], im[2 * j + 1], h, l);
      ih[j] = h;
      il[j] = l;
    }
    u4v* q = reinterpret_cast<u4v*>(dst + r * 4 * (int64_t)Kp + 32 * (int64_t)kb);
    q[0] = rh;
    q[1] = rl;
    q[2] = ih;
    q[3] = il;
  }
}

// C[m][n] = sum_k A[m][k] B[n][k] over pre-split rows (row strides 4*Kp bf16), B row of n at
// (n / b_in) * b_outer + n % b_in, C complex FP32 row-major with leading dimension ldc
// (complex elements).  BM x BN workgroup tile, (BM/32) x (BN/32) waves of 32 x 32 outputs each.
template <int BM, int BN, bool XCD>
__global__ __launch_bounds__(64 * (BM / 32) * (BN / 32), (BM * BN == 64 * 64) ? 2 : 1) void
gett_bf16x3_split_kernel(const unsigned short* __restrict__ A, const unsigned short* __restrict__ B, int M,
                         int N, int Kp, float* __restrict__ C, int64_t ldc, int b_in, int64_t b_outer) {
  constexpr int BK = 32;
  constexpr int WM = BM / 32, T = 64 * (BM / 32) * (BN / 32);
  constexpr int QA = BM * 16 / T, QB = BN * 16 / T, RS = T / 16;
  constexpr int CH = 17;  // 16-byte chunks per LDS row: 4 k blocks x 4 planes + 1 pad
  typedef unsigned u4v __attribute__((ext_vector_type(4)));
  __shared__ u4v sA[2][BM][CH];
  __shared__ u4v sB[2][BN][CH];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w % WM, wn = w / WM;
  const int tiles_m = (M + BM - 1) / BM;
  const int tile = XCD ? xcd_tile(blockIdx.x, gridDim.x) : blockIdx.x;
  const int m0 = (tile % tiles_m) * BM, n0 = (tile / tiles_m) * BN;
  const int64_t rs = 4 * (int64_t)Kp;  // bf16 per row

  // loader: chunk tid%16 (k block (tid%16)/4, plane tid%4) of tile rows
  // tid/16 + RS*q; rows past M (N) are clamped: they feed only outputs that
  // are not stored
  const int ch = tid % 16;
  const u4v* pa[QA];
  const u4v* pb[QB];
#pragma unroll
  for (int q = 0; q < QA; ++q)
    pa[q] = reinterpret_cast<const u4v*>(A + min(m0 + tid / 16 + RS * q, M - 1) * rs) + ch;
#pragma unroll
  for (int q = 0; q < QB; ++q) {
    const int n = min(n0 + tid / 16 + RS * q, N - 1);
    const int nq = n / b_in;
    pb[q] = reinterpret_cast<const u4v*>(B + ((int64_t)nq * b_outer + (n - nq * b_in)) * rs) + ch;
  }
  u4v ra[QA], rb[QB];
  auto load = [&](int kt) {  // 16 chunks (256 bytes) per row and k tile
#pragma unroll
    for (int q = 0; q < QA; ++q) ra[q] = pa[q][16 * kt];
#pragma unroll
    for (int q = 0; q < QB; ++q) rb[q] = pb[q][16 * kt];
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < QA; ++q) sA[buf][tid / 16 + RS * q][ch] = ra[q];
#pragma unroll
    for (int q = 0; q < QB; ++q) sB[buf][tid / 16 + RS * q][ch] = rb[q];
  };

  float4_t accR[2][2], accN[2][2], accI[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      accR[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
      accN[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
      accI[i][j] = float4_t{0.f, 0.f, 0.f, 0.f};
    }

  const int nk = Kp / BK;
  if (nk > 0) {
    load(0);
    store(0);
  }
  __syncthreads();
  const int kc = 4 * (lane >> 4);  // this lane's k block (8 k values) in a fragment
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) load(kt + 1);
    bf16x8_t arh[2], arl[2], aih[2], ail[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int r = wm * 32 + 16 * i + (lane & 15);
      arh[i] = __builtin_bit_cast(bf16x8_t, sA[cur][r][kc + 0]);
      arl[i] = __builtin_bit_cast(bf16x8_t, sA[cur][r][kc + 1]);
      aih[i] = __builtin_bit_cast(bf16x8_t, sA[cur][r][kc + 2]);
      ail[i] = __builtin_bit_cast(bf16x8_t, sA[cur][r][kc + 3]);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = wn * 32 + 16 * j + (lane & 15);
      const bf16x8_t brh = __builtin_bit_cast(bf16x8_t, sB[cur][c][kc + 0]);
      const bf16x8_t brl = __builtin_bit_cast(bf16x8_t, sB[cur][c][kc + 1]);
      const bf16x8_t bih = __builtin_bit_cast(bf16x8_t, sB[cur][c][kc + 2]);
      const bf16x8_t bil = __builtin_bit_cast(bf16x8_t, sB[cur][c][kc + 3]);
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        accR[i][j] = mma3(arh[i], arl[i], brh, brl, accR[i][j]);
        accN[i][j] = mma3(aih[i], ail[i], bih, bil, accN[i][j]);
        accI[i][j] = mma3(arh[i], arl[i], bih, bil, accI[i][j]);
        accI[i][j] = mma3(aih[i], ail[i], brh, brl, accI[i][j]);
      }
    }
    // the other buffer was last read before the previous barrier
    if (kt + 1 < nk) store(cur ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn * 32 + 16 * j + (lane & 15);
      if (col >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm * 32 + 16 * i + 4 * (lane >> 4) + r;
        if (row >= M) continue;
        float* c = C + 2 * ((int64_t)row * ldc + col);
        c[0] = accR[i][j][r] - accN[i][j][r];
        c[1] = accI[i][j][r];
      }
    }
}

int bf16x3_split_k(int K) { return (K + 31) / 32 * 32; }

void split_rows_bf16x3(const float* src, int64_t rows, int64_t group, int64_t group_stride,
                       int64_t row_stride, int K, unsigned short* dst, hipStream_t s) {
  if (rows <= 0 || K <= 0) return;
  const int Kp = bf16x3_split_k(K);
  const int64_t tot = rows * (Kp / 8);
  int64_t blocks = (tot + 255) / 256;
  if (blocks > 65535 * 8) blocks = 65535 * 8;
  hipLaunchKernelGGL(split_rows_kernel, dim3((unsigned)blocks), dim3(256), 0, s, src, rows,
                     group > 0 ? group : 1, group_stride, row_stride, K, Kp, dst);
  HIPCHECK(hipGetLastError());
}

void gemm_bf16x3_split(const unsigned short* A, const unsigned short* B, int M, int N, int K, float* C,
                       int64_t ldc, hipStream_t s, int b_in, int64_t b_outer) {
  if (M <= 0 || N <= 0) return;
  if (b_in <= 0) {  // B rows contiguous
    b_in = N;
    b_outer = N;
  }
  // 128 x 128 tiles (16 waves, one workgroup per CU) in XCD order: 1.22x the
  // 64 x 64 tiles in plain order on the ladder tile build, bitwise equal
  constexpr int BM = 128, BN = 128;
  const int64_t tiles = (int64_t)((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  if (tiles > 0x7fffffffLL) raise(-1, "contraction too large for one launch");
  hipLaunchKernelGGL((gett_bf16x3_split_kernel<BM, BN, true>), dim3((unsigned)tiles),
                     dim3(64 * (BM / 32) * (BN / 32)), 0, s, A, B, M, N, bf16x3_split_k(K), C, ldc,
                     b_in, b_outer);
  HIPCHECK(hipGetLastError());
}

template <int KIND, bool A16>
static void launch_bf16x3(const Gett<float>& g, hipStream_t s) {
  // 128 x 128 tiles in XCD order: 1.37x (contraction) and 1.25x (ring) the
  // 64 x 64 tiles in plain order, bitwise equal
  constexpr int BM = 128, BN = 128, BK = 32;
  const int tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
  for (int64_t b0 = 0; b0 < g.nbatch; b0 += 65535) {
    Gett<float> h = g;
    const int nb = (int)((g.nbatch - b0) < 65535 ? (g.nbatch - b0) : 65535);
    h.A = g.A + 2 * b0 * g.a_b;
    h.B = g.B + 2 * b0 * g.b_b;
    h.C = g.C + 2 * b0 * g.c_b;
    h.kslice = g.K > 0 ? g.K : 1;
    h.ws = nullptr;
    // split K when the output gives too few workgroups for whole rounds over the CUs (one
    // 16-wave workgroup per CU): with nz slices the launch takes ceil(wgs nz / 256) rounds
    // of K / nz each, so nz is the smallest count within 2% of the best rounds / nz, taken
    // when it saves at least 10%; slices of >= 1024 k, a multiple of BK (keeps the 16-byte
    // alignment of the k-pair loads), fixed-order reduction
    int nz = 1;
    const int64_t wgs = (int64_t)tiles * nb;
    if (g_ws && wgs < 1024 && g.K >= 2048) {
      const int64_t per = (int64_t)g.M * g.N * nb * 2 * (int64_t)sizeof(float);
      const int64_t cap = per > 0 ? (int64_t)(g_ws_bytes / per) : 0;
      int64_t zmax = g.K / 1024;
      if (zmax > cap) zmax = cap;
      if (zmax > 32) zmax = 32;
      auto cost = [&](int64_t z) { return (double)((wgs * z + 255) / 256) / (double)z; };
      double best = cost(1);
      for (int64_t z = 2; z <= zmax; ++z) best = cost(z) < best ? cost(z) : best;
      int64_t want = 1;
      while (want < zmax && cost(want) > 1.02 * best) ++want;
      if (cost(want) > 0.9 * cost(1)) want = 1;  // under 10% to gain: no split
      if (want >= 2) {
        int64_t ks = (g.K + want - 1) / want;
        ks = (ks + BK - 1) / BK * BK;
        nz = (int)((g.K + ks - 1) / ks);
        h.kslice = (int)ks;
        h.ws = (float*)g_ws;
      }
    }
    hipLaunchKernelGGL((gett_bf16x3_kernel<KIND, BM, BN, true, A16>), dim3(tiles, nb, nz),
                       dim3(64 * (BM / 32) * (BN / 32)), 0, s, h);
    HIPCHECK(hipGetLastError());
    if (nz > 1) {
      const int64_t tot = (int64_t)g.M * g.N * nb;
      int64_t blocks = (tot + 255) / 256;
      if (blocks > 65535 * 8) blocks = 65535 * 8;
      hipLaunchKernelGGL(gett_splitk_reduce<float>, dim3((unsigned)blocks), dim3(256), 0, s, h, nz, nb);
      HIPCHECK(hipGetLastError());
    }
  }
}

template <typename R>
void launch_gett(const Gett<R>& g, int kind_in, hipStream_t s) {
  int kind = kind_in;
  if (g.M <= 0 || g.N <= 0 || g.nbatch <= 0) return;
  if ((int64_t)((g.M + 63) / 64) * ((g.N + 63) / 64) > 0x7fffffffLL)
    raise(-1, "contraction too large for one launch");
  // BF16x3 kinds: only for FP32 operands that are K-contiguous in both A and B; 16-byte
  // loads of two complex values where row strides are even and bases 16-byte aligned
  const bool kcontig = g.k_in == g.K && g.a_ki == 1 && g.b_ki == 1;
  const bool a16 = g.a_mo % 2 == 0 && g.a_mi % 2 == 0 && g.b_no % 2 == 0 && g.b_ni % 2 == 0 &&
                   g.a_b % 2 == 0 && g.b_b % 2 == 0 && reinterpret_cast<uintptr_t>(g.A) % 16 == 0 &&
                   reinterpret_cast<uintptr_t>(g.B) % 16 == 0;
  if (kind == GETT_LADDER_BUILD_BF16X3 || kind == GETT_LADDER_CONTRACT_BF16X3 ||
      kind == GETT_RING_BF16X3) {
    if constexpr (sizeof(R) == sizeof(float)) {
      if (kcontig) {
        if (kind == GETT_LADDER_BUILD_BF16X3)
          a16 ? launch_bf16x3<GETT_LADDER_BUILD_BF16X3, true>(g, s)
              : launch_bf16x3<GETT_LADDER_BUILD_BF16X3, false>(g, s);
        else if (kind == GETT_LADDER_CONTRACT_BF16X3)
          a16 ? launch_bf16x3<GETT_LADDER_CONTRACT_BF16X3, true>(g, s)
              : launch_bf16x3<GETT_LADDER_CONTRACT_BF16X3, false>(g, s);
        else
          a16 ? launch_bf16x3<GETT_RING_BF16X3, true>(g, s) : launch_bf16x3<GETT_RING_BF16X3, false>(g, s);
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
