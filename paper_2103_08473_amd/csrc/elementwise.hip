// HBM-bound kernels of the CCSD iteration: packing of antisymmetric pairs,
// tau formation, operand permutes for the ring contractions, the residual
// assembly fused with the denominator (Jacobi) step, DIIS vector operations,
// the energy, and fixed-order (deterministic, atomic-free) reductions.
#include "common.h"

namespace exacc {

namespace {

constexpr int TB = 256;

struct z {
  double x, y;
};
// complex element i of an interleaved array of T (float or double), widened to double
template <typename T>
__device__ __forceinline__ z ld(const T* p, int64_t i) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2 t = *reinterpret_cast<const v2*>(p + 2 * i);
  return z{(double)t.x, (double)t.y};
}
// store complex element i, rounded to T (round to nearest even)
template <typename T>
__device__ __forceinline__ void st(T* p, int64_t i, z v) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2 t;
  t.x = (T)v.x;
  t.y = (T)v.y;
  *reinterpret_cast<v2*>(p + 2 * i) = t;
}
__device__ __forceinline__ z add(z a, z b) { return z{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ z sub(z a, z b) { return z{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ z mul(z a, z b) { return z{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ z scal(double s, z a) { return z{s * a.x, s * a.y}; }

// (p, q), p < q, from the packed index x of pairs over m (row-major by p).
__device__ __forceinline__ void pair_of(int64_t x, int m, int& p, int& q) {
  const double tm = 2.0 * m - 1.0;
  int a = (int)floor((tm - sqrt(tm * tm - 8.0 * (double)x)) * 0.5);
  if (a < 0) a = 0;
  // exact correction for rounding at row boundaries
  while (a > 0 && (int64_t)a * m - (int64_t)a * (a + 1) / 2 > x) --a;
  while ((int64_t)(a + 1) * m - (int64_t)(a + 1) * (a + 2) / 2 <= x) ++a;
  p = a;
  q = (int)(x - ((int64_t)a * m - (int64_t)a * (a + 1) / 2)) + a + 1;
}
__device__ __forceinline__ int64_t pidx(int p, int q, int m) {
  return (int64_t)p * m - (int64_t)p * (p + 1) / 2 + (q - p - 1);
}

inline int nblocks(int64_t n, int cap = 65535 * 8) {
  int64_t b = (n + TB - 1) / TB;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

// ------------------------------------------------------------------ B staging
__global__ void transpose_B_kernel(const double* __restrict__ B, double* __restrict__ Bt, int64_t X,
                                   int64_t nn) {
  __shared__ double tr[32][33], ti[32][33];
  const int64_t q0 = (int64_t)blockIdx.x * 32, P0 = (int64_t)blockIdx.y * 32;
  const int tx = threadIdx.x, ty = threadIdx.y;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int64_t P = P0 + r, q = q0 + tx;
    if (P < X && q < nn) {
      z v = ld(B, P * nn + q);
      tr[r][tx] = v.x;
      ti[r][tx] = v.y;
    }
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t q = q0 + r, P = P0 + tx;
    if (P < X && q < nn) st(Bt, q * X + P, z{tr[tx][r], ti[tx][r]});
  }
}

// out3 = {max |B - B^H|, max |B|, number of non-finite entries}
__global__ void check_B_kernel(const double* __restrict__ B, int64_t X, int n,
                               double* __restrict__ part) {
  double mh = 0, mb = 0, nf = 0;
  const int64_t nn = (int64_t)n * n, tot = X * nn;
  for (int64_t t = (int64_t)blockIdx.x * TB + threadIdx.x; t < tot; t += (int64_t)gridDim.x * TB) {
    const int64_t P = t / nn, r = t - P * nn;
    const int p = (int)(r / n), q = (int)(r - (int64_t)p * n);
    z a = ld(B, t), b = ld(B, P * nn + (int64_t)q * n + p);
    if (!isfinite(a.x) || !isfinite(a.y)) nf += 1;
    const double dh = fmax(fabs(a.x - b.x), fabs(a.y + b.y));
    mh = fmax(mh, dh);
    mb = fmax(mb, fmax(fabs(a.x), fabs(a.y)));
  }
  __shared__ double s[3][TB];
  s[0][threadIdx.x] = mh;
  s[1][threadIdx.x] = mb;
  s[2][threadIdx.x] = nf;
  __syncthreads();
  for (int w = TB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s[0][threadIdx.x] = fmax(s[0][threadIdx.x], s[0][threadIdx.x + w]);
      s[1][threadIdx.x] = fmax(s[1][threadIdx.x], s[1][threadIdx.x + w]);
      s[2][threadIdx.x] += s[2][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x + 0] = s[0][0];
    part[3 * blockIdx.x + 1] = s[1][0];
    part[3 * blockIdx.x + 2] = s[2][0];
  }
}

__global__ void check_B_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double a = 0, b = 0, c = 0;
    for (int i = 0; i < nb; ++i) {
      a = fmax(a, part[3 * i]);
      b = fmax(b, part[3 * i + 1]);
      c += part[3 * i + 2];
    }
    out[0] = a;
    out[1] = b;
    out[2] = c;
  }
}

// ------------------------------------------------------------------ packing
template <typename T>
__global__ void pack_last2_kernel(T* __restrict__ out, const T* __restrict__ in,
                                  const int* __restrict__ rowmap, int64_t rows, int m,
                                  int64_t in_row_stride) {
  const int64_t P = (int64_t)m * (m - 1) / 2, tot = rows * P;
  for (int64_t t = (int64_t)blockIdx.x * TB + threadIdx.x; t < tot; t += (int64_t)gridDim.x * TB) {
    const int64_t r = t / P, x = t - r * P;
    int a, b;
    pair_of(x, m, a, b);
    const int64_t rr = rowmap ? rowmap[r] : r;
    st(out, t, ld(in, rr * in_row_stride + (int64_t)a * m + b));
  }
}

// T2 (full), TAU (full) and packed tau from t1 and packed t2.
template <typename T>
__global__ void unpack_tau_kernel(const double* __restrict__ t1, const double* __restrict__ t2p,
                                  T* __restrict__ T2, T* __restrict__ TAU, T* __restrict__ taup, int o,
                                  int v) {
  const int64_t vv = (int64_t)v * v, tot = (int64_t)o * o * vv, Pv = (int64_t)v * (v - 1) / 2;
  for (int64_t t = (int64_t)blockIdx.x * TB + threadIdx.x; t < tot; t += (int64_t)gridDim.x * TB) {
    const int64_t ij = t / vv, ab = t - ij * vv;
    const int i = (int)(ij / o), j = (int)(ij - (int64_t)i * o);
    const int a = (int)(ab / v), b = (int)(ab - (int64_t)a * v);
    z val{0, 0};
    if (i != j && a != b) {
      const int pi = i < j ? i : j, pj = i < j ? j : i;
      const int pa = a < b ? a : b, pb = a < b ? b : a;
      const double sg = ((i < j) == (a < b)) ? 1.0 : -1.0;
      val = scal(sg, ld(t2p, pidx(pi, pj, o) * Pv + pidx(pa, pb, v)));
    }
    st(T2, t, val);
    const z tt = sub(mul(ld(t1, (int64_t)i * v + a), ld(t1, (int64_t)j * v + b)),
                     mul(ld(t1, (int64_t)j * v + a), ld(t1, (int64_t)i * v + b)));
    const z tau = add(val, tt);
    st(TAU, t, tau);
    if (i < j && a < b) st(taup, pidx(i, j, o) * Pv + pidx(a, b, v), tau);
  }
}

// Tq[b][j][k][c] = T2[j][k][c][b];  Xp[b][j][k][c] = 1/2 Tq + t1[k][b] t1[j][c]
// (- t1r[k][b] t1r[j][c] when t1r is given: the operands of a difference T2 - T2_ref)
template <typename T>
__global__ void ring_operands_kernel(const T* __restrict__ T2, const double* __restrict__ t1,
                                     T* __restrict__ Tq, T* __restrict__ Xp, int o, int v,
                                     const double* __restrict__ t1r) {
  __shared__ double tr[32][33], ti[32][33];
  const int b0 = blockIdx.x * 32, c0 = blockIdx.y * 32;
  const int64_t jk = blockIdx.z;
  const int j = (int)(jk / o), k = (int)(jk - (int64_t)j * o);
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int64_t vv = (int64_t)v * v, oo = (int64_t)o * o;
  for (int r = ty; r < 32; r += 8) {
    const int c = c0 + r, b = b0 + tx;
    if (c < v && b < v) {
      z x = ld(T2, jk * vv + (int64_t)c * v + b);
      tr[r][tx] = x.x;
      ti[r][tx] = x.y;
    }
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int b = b0 + r, c = c0 + tx;
    if (c < v && b < v) {
      const z q{tr[tx][r], ti[tx][r]};
      const int64_t off = ((int64_t)b * oo + jk) * v + c;
      st(Tq, off, q);
      z p = mul(ld(t1, (int64_t)k * v + b), ld(t1, (int64_t)j * v + c));
      if (t1r) p = sub(p, mul(ld(t1r, (int64_t)k * v + b), ld(t1r, (int64_t)j * v + c)));
      st(Xp, off, add(scal(0.5, q), p));
    }
  }
}

// Cf[i][j][b][k] = conj(Vooov[i][j][k][b]) + sign(i,j) Cp[(min,max)][b][k]
template <typename T>
__global__ void expand_c_kernel(const T* __restrict__ Vooov, const T* __restrict__ Cp,
                                T* __restrict__ Cf, int o, int v) {
  const int64_t tot = (int64_t)o * o * v * o;
  for (int64_t t = (int64_t)blockIdx.x * TB + threadIdx.x; t < tot; t += (int64_t)gridDim.x * TB) {
    int64_t r = t;
    const int k = (int)(r % o);
    r /= o;
    const int b = (int)(r % v);
    r /= v;
    const int j = (int)(r % o);
    const int i = (int)(r / o);
    z x = ld(Vooov, (((int64_t)i * o + j) * o + k) * v + b);
    x.y = -x.y;
    if (i != j) {
      const int p = i < j ? i : j, q = i < j ? j : i;
      z c = ld(Cp, (pidx(p, q, o) * v + b) * o + k);
      x = (i < j) ? add(x, c) : sub(x, c);
    }
    st(Cf, t, x);
  }
}

// W[b'][x=(c<d)] = Ta[c][b'][d] - Ta[d][b'][c] (row stride ldw).  One block per (b', c-tile,
// d-tile) with c-tile <= d-tile: both Ta tiles are read along their contiguous last index
// and the second is transposed through LDS, so every global access is coalesced.
template <typename T>
__global__ void ladder_antisym_kernel(const T* __restrict__ Ta, T* __restrict__ W, int nb, int v,
                                      int64_t ldw) {
  __shared__ double tr[32][33], ti[32][33];
  const int ntile = (v + 31) / 32;
  // blockIdx.x enumerates tile pairs (tc <= td) row-major
  int tc = 0, rem = blockIdx.x;
  while (rem >= ntile - tc) {
    rem -= ntile - tc;
    ++tc;
  }
  const int td = tc + rem;
  const int64_t bp = blockIdx.y;
  const int c0 = 32 * tc, d0 = 32 * td;
  const int tx = threadIdx.x, ty = threadIdx.y;  // 32 x 8
  // stage Ta[d][b'][c] for d in d-tile, c in c-tile (contiguous in c) as [c - c0][d - d0]
  for (int r = ty; r < 32; r += 8) {
    const int d = d0 + r, c = c0 + tx;
    if (d < v && c < v) {
      const z q = ld(Ta, ((int64_t)d * nb + bp) * v + c);
      tr[tx][r] = q.x;
      ti[tx][r] = q.y;
    }
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int c = c0 + r, d = d0 + tx;
    if (c < v && d < v && c < d) {
      const z p = ld(Ta, ((int64_t)c * nb + bp) * v + d);
      const z q{tr[r][tx], ti[r][tx]};
      st(W, bp * ldw + pidx(c, d, v), sub(p, q));
    }
  }
}

// All rows at once: W[(a<b)][(c<d)] = T[a][c][b][d] - T[a][d][b][c] from the full product
// T[a][c][b][d] = sum_P F_ac F_bd (v^4 elements).  blockIdx.z = a, blockIdx.y = b - a - 1
// (blocks past the row's last b exit), blockIdx.x = (c-tile <= d-tile) pair; the second T
// tile is transposed through LDS as in ladder_antisym_kernel.
template <typename T>
__global__ void ladder_antisym_all_kernel(const T* __restrict__ Tf, T* __restrict__ W, int v) {
  __shared__ double tr[32][33], ti[32][33];
  const int a = blockIdx.z, b = a + 1 + (int)blockIdx.y;
  if (b >= v) return;
  const int ntile = (v + 31) / 32;
  int tc = 0, rem = blockIdx.x;
  while (rem >= ntile - tc) {
    rem -= ntile - tc;
    ++tc;
  }
  const int td = tc + rem;
  const int c0 = 32 * tc, d0 = 32 * td;
  const int tx = threadIdx.x, ty = threadIdx.y;  // 32 x 8
  const int64_t vv = (int64_t)v * v;
  const T* Ta = Tf + 2 * ((int64_t)a * v * vv + (int64_t)b * v);  // [c][d] at c * v^2 + d
  // stage T[a][d][b][c] for d in d-tile, c in c-tile (contiguous in c) as [c - c0][d - d0]
  for (int r = ty; r < 32; r += 8) {
    const int d = d0 + r, c = c0 + tx;
    if (d < v && c < v) {
      const z q = ld(Ta, (int64_t)d * vv + c);
      tr[tx][r] = q.x;
      ti[tx][r] = q.y;
    }
  }
  __syncthreads();
  const int64_t row = pidx(a, b, v), Pv = (int64_t)v * (v - 1) / 2;
  for (int r = ty; r < 32; r += 8) {
    const int c = c0 + r, d = d0 + tx;
    if (c < v && d < v && c < d) {
      const z p = ld(Ta, (int64_t)c * vv + d);
      const z q{tr[r][tx], ti[r][tx]};
      st(W, row * Pv + pidx(c, d, v), sub(p, q));
    }
  }
}

// Wt[y][x] = W[x][col0 + y] for x < rows, y < ncols (32 x 32 tiles through LDS: reads along
// W rows and writes along Wt rows are both coalesced).
template <typename T>
__global__ void transpose_tail_kernel(const T* __restrict__ W, int64_t rows, int64_t ldw, int64_t col0,
                                      int64_t ncols, T* __restrict__ Wt, int64_t ldt) {
  __shared__ double tr[32][33], ti[32][33];
  const int64_t x0 = 32 * (int64_t)blockIdx.y, y0 = 32 * (int64_t)blockIdx.x;
  const int tx = threadIdx.x, ty = threadIdx.y;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int64_t x = x0 + r, y = y0 + tx;
    if (x < rows && y < ncols) {
      const z q = ld(W, x * ldw + col0 + y);
      tr[r][tx] = q.x;
      ti[r][tx] = q.y;
    }
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t y = y0 + r, x = x0 + tx;
    if (x < rows && y < ncols) st(Wt, y * ldt + x, z{tr[tx][r], ti[tx][r]});
  }
}

// Residual assembly + Jacobi step for the doubles (packed i<j, a<b).
template <typename T>
__global__ void assemble_t2_kernel(const T* __restrict__ Znp, const T* __restrict__ Z,
                                   const T* __restrict__ R,
                                   const double* __restrict__ Vp, const double* __restrict__ t2p,
                                   const double* __restrict__ eps, int o, int v, double shift,
                                   double* __restrict__ xt, double* __restrict__ e,
                                   double* __restrict__ s2, double* __restrict__ part) {
  const int64_t Po = (int64_t)o * (o - 1) / 2, Pv = (int64_t)v * (v - 1) / 2, tot = Po * Pv;
  const int64_t vv = (int64_t)v * v;
  double acc = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * TB + threadIdx.x; t < tot; t += (int64_t)gridDim.x * TB) {
    const int64_t p = t / Pv, x = t - p * Pv;
    int i, j, a, b;
    pair_of(p, o, i, j);
    pair_of(x, v, a, b);
    const int64_t ijab = ((int64_t)i * o + j) * vv + (int64_t)a * v + b;
    const int64_t ijba = ((int64_t)i * o + j) * vv + (int64_t)b * v + a;
    const int64_t jiab = ((int64_t)j * o + i) * vv + (int64_t)a * v + b;
    const int64_t jiba = ((int64_t)j * o + i) * vv + (int64_t)b * v + a;
    // Znp, R and Vp may be null (CC2 doubles: Z holds the whole T1-dressed <ab||ij>)
    z s = ld(Z, ijab);
    if (Znp) s = add(s, ld(Znp, t));
    if (R) s = add(s, add(sub(ld(R, ijab), ld(R, jiab)), sub(ld(R, jiba), ld(R, ijba))));
    if (Vp) {
      const z g = ld(Vp, t);
      s.x += g.x;
      s.y -= g.y;
    }
    const z tt = ld(t2p, t);
    const double D = eps[o + a] + eps[o + b] - eps[i] - eps[j];
    s = add(s, scal(D, tt));
    if (s2) {
      st(s2, ijab, s);
      st(s2, jiba, s);
      st(s2, ijba, scal(-1.0, s));
      st(s2, jiab, scal(-1.0, s));
    } else {
      const z dl = scal(-1.0 / (D + 2.0 * shift), s);
      st(e, t, dl);
      st(xt, t, add(tt, dl));
      acc += dl.x * dl.x + dl.y * dl.y;
    }
  }
  __shared__ double sh[TB];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = TB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && part) part[blockIdx.x] = sh[0];
}

template <typename T>
__global__ void assemble_t1_kernel(const T* __restrict__ S1, const double* __restrict__ t1,
                                   const double* __restrict__ eps, int o, int v, double shift,
                                   int frozen, double* __restrict__ xt, double* __restrict__ e,
                                   double* __restrict__ s1, double* __restrict__ part) {
  const int64_t tot = (int64_t)o * v;
  double acc = 0.0;
  for (int64_t t = threadIdx.x; t < tot; t += TB) {
    const int i = (int)(t / v), a = (int)(t - (int64_t)i * v);
    const double D = eps[o + a] - eps[i];
    const z tt = ld(t1, t);
    const z s = add(ld(S1, t), scal(D, tt));
    if (s1) {
      st(s1, t, s);
    } else {
      // frozen (CCD): no T1 equation, the step is zero and t1 stays as it is (zero)
      const z dl = frozen ? scal(0.0, s) : scal(-1.0 / (D + shift), s);
      st(e, t, dl);
      st(xt, t, add(tt, dl));
      acc += dl.x * dl.x + dl.y * dl.y;
    }
  }
  __shared__ double sh[TB];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = TB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && part) part[0] = sh[0];
}

// out[w] = sum_b partial[b*width + w], fixed order, one block.
__global__ void reduce_sum_kernel(const double* __restrict__ partial, int n, int width,
                                  double* __restrict__ out) {
  __shared__ double sh[TB];
  for (int w = 0; w < width; ++w) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < n; b += TB) acc += partial[(int64_t)b * width + w];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = TB / 2; s > 0; s >>= 1) {
      if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[w] = sh[0];
    __syncthreads();
  }
}

constexpr int MAXV = 16;
struct Ptrs {
  const double* p[MAXV];
};
struct Coefs {
  double re[MAXV], im[MAXV];
};

// partial[blk][k] = sum_i conj(es[k][i]) e[i]   (complex, k < m)
__global__ void dot_many_kernel(Ptrs es, int m, const double* __restrict__ e, int64_t len,
                                double* __restrict__ part) {
  double ar[MAXV], ai[MAXV];
#pragma unroll
  for (int k = 0; k < MAXV; ++k) ar[k] = ai[k] = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * TB + threadIdx.x; t < len; t += (int64_t)gridDim.x * TB) {
    const z y = ld(e, t);
#pragma unroll
    for (int k = 0; k < MAXV; ++k) {
      if (k < m) {
        const z x = ld(es.p[k], t);
        ar[k] += x.x * y.x + x.y * y.y;
        ai[k] += x.x * y.y - x.y * y.x;
      }
    }
  }
  __shared__ double sh[TB];
  for (int k = 0; k < m; ++k) {
    for (int c = 0; c < 2; ++c) {
      sh[threadIdx.x] = c ? ai[k] : ar[k];
      __syncthreads();
      for (int s = TB / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
      }
      if (threadIdx.x == 0) part[((int64_t)blockIdx.x * m + k) * 2 + c] = sh[0];
      __syncthreads();
    }
  }
}

__global__ void lincomb_kernel(double* __restrict__ x, Ptrs xs, Coefs c, int m, int64_t len) {
  for (int64_t t = (int64_t)blockIdx.x * TB + threadIdx.x; t < len; t += (int64_t)gridDim.x * TB) {
    z acc{0, 0};
    for (int k = 0; k < m; ++k) acc = add(acc, mul(z{c.re[k], c.im[k]}, ld(xs.p[k], t)));
    st(x, t, acc);
  }
}

// E partial = sum_{i<j,a<b} <ij||ab> (t_ij^ab + t_i^a t_j^b - t_j^a t_i^b)
__global__ void energy_kernel(const double* __restrict__ Vp, const double* __restrict__ t2p,
                              const double* __restrict__ t1, int o, int v,
                              double* __restrict__ part) {
  const int64_t Po = (int64_t)o * (o - 1) / 2, Pv = (int64_t)v * (v - 1) / 2, tot = Po * Pv;
  double er = 0, ei = 0;
  for (int64_t t = (int64_t)blockIdx.x * TB + threadIdx.x; t < tot; t += (int64_t)gridDim.x * TB) {
    const int64_t p = t / Pv, x = t - p * Pv;
    int i, j, a, b;
    pair_of(p, o, i, j);
    pair_of(x, v, a, b);
    const z tau = add(ld(t2p, t), sub(mul(ld(t1, (int64_t)i * v + a), ld(t1, (int64_t)j * v + b)),
                                      mul(ld(t1, (int64_t)j * v + a), ld(t1, (int64_t)i * v + b))));
    const z g = mul(ld(Vp, t), tau);
    er += g.x;
    ei += g.y;
  }
  __shared__ double sr[TB], si[TB];
  sr[threadIdx.x] = er;
  si[threadIdx.x] = ei;
  __syncthreads();
  for (int s = TB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sr[threadIdx.x] += sr[threadIdx.x + s];
      si[threadIdx.x] += si[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sr[0];
    part[2 * blockIdx.x + 1] = si[0];
  }
}

__global__ void unpack_full_kernel(const double* __restrict__ t2p, double* __restrict__ t2, int o,
                                   int v) {
  const int64_t vv = (int64_t)v * v, tot = (int64_t)o * o * vv, Pv = (int64_t)v * (v - 1) / 2;
  for (int64_t t = (int64_t)blockIdx.x * TB + threadIdx.x; t < tot; t += (int64_t)gridDim.x * TB) {
    const int64_t ij = t / vv, ab = t - ij * vv;
    const int i = (int)(ij / o), j = (int)(ij - (int64_t)i * o);
    const int a = (int)(ab / v), b = (int)(ab - (int64_t)a * v);
    z val{0, 0};
    if (i != j && a != b) {
      const int pi = i < j ? i : j, pj = i < j ? j : i;
      const int pa = a < b ? a : b, pb = a < b ? b : a;
      const double sg = ((i < j) == (a < b)) ? 1.0 : -1.0;
      val = scal(sg, ld(t2p, pidx(pi, pj, o) * Pv + pidx(pa, pb, v)));
    }
    st(t2, t, val);
  }
}

// t2[i][j][a][b] = FP32 of the full antisymmetric t2 - t2_ref, from their packed forms
// (the difference is formed in FP64)
__global__ void unpack_diff_kernel(const double* __restrict__ t2p, const double* __restrict__ r2p,
                                   float* __restrict__ t2, int o, int v) {
  const int64_t vv = (int64_t)v * v, tot = (int64_t)o * o * vv, Pv = (int64_t)v * (v - 1) / 2;
  for (int64_t t = (int64_t)blockIdx.x * TB + threadIdx.x; t < tot; t += (int64_t)gridDim.x * TB) {
    const int64_t ij = t / vv, ab = t - ij * vv;
    const int i = (int)(ij / o), j = (int)(ij - (int64_t)i * o);
    const int a = (int)(ab / v), b = (int)(ab - (int64_t)a * v);
    z val{0, 0};
    if (i != j && a != b) {
      const int pi = i < j ? i : j, pj = i < j ? j : i;
      const int pa = a < b ? a : b, pb = a < b ? b : a;
      const double sg = ((i < j) == (a < b)) ? 1.0 : -1.0;
      const int64_t q = pidx(pi, pj, o) * Pv + pidx(pa, pb, v);
      val = scal(sg, sub(ld(t2p, q), ld(r2p, q)));
    }
    st(t2, t, val);
  }
}

// out = a - b, n reals
__global__ void sub_kernel(const double* __restrict__ a, const double* __restrict__ b,
                           double* __restrict__ out, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * TB + threadIdx.x; t < n; t += (int64_t)gridDim.x * TB)
    out[t] = a[t] - b[t];
}

__global__ void pack_amp_kernel(const double* __restrict__ t2, double* __restrict__ x2, int o,
                                int v) {
  const int64_t Po = (int64_t)o * (o - 1) / 2, Pv = (int64_t)v * (v - 1) / 2, tot = Po * Pv;
  for (int64_t t = (int64_t)blockIdx.x * TB + threadIdx.x; t < tot; t += (int64_t)gridDim.x * TB) {
    const int64_t p = t / Pv, x = t - p * Pv;
    int i, j, a, b;
    pair_of(p, o, i, j);
    pair_of(x, v, a, b);
    st(x2, t, ld(t2, (((int64_t)i * o + j) * v + a) * v + b));
  }
}

// dst[r][k] = conj(src[r * src_stride + k]), k < len (complex elements)
__global__ void conj_rows_kernel(double* __restrict__ dst, const double* __restrict__ src, int64_t rows,
                                 int64_t src_stride, int64_t len) {
  const int64_t tot = rows * len;
  for (int64_t t = (int64_t)blockIdx.x * TB + threadIdx.x; t < tot; t += (int64_t)gridDim.x * TB) {
    const int64_t r = t / len, k = t - r * len;
    z x = ld(src, r * src_stride + k);
    x.y = -x.y;
    st(dst, t, x);
  }
}

// Lambda one-body density (App. E) from its pieces, gamma[p][q] = <{q+ p}>:
//   oo [i][j] = -Go[j][i] - M[j][i]      (M[i][m] = sum_e l1[m][e] t1[i][e])
//   ov [i][a] = l1[i][a]
//   vo [a][i] = Dvo[i][a]
//   vv [a][b] = -Gv[b][a] + N[a][b]      (N[a][b] = sum_m t1[m][a] l1[m][b])
__global__ void lambda_density_kernel(const double* __restrict__ Go, const double* __restrict__ M,
                                      const double* __restrict__ l1, const double* __restrict__ Dvo,
                                      const double* __restrict__ Gv, const double* __restrict__ N,
                                      int o, int v, double* __restrict__ g) {
  const int n = o + v;
  const int64_t tot = (int64_t)n * n;
  for (int64_t t = (int64_t)blockIdx.x * TB + threadIdx.x; t < tot; t += (int64_t)gridDim.x * TB) {
    const int p = (int)(t / n), q = (int)(t - (int64_t)p * n);
    z x;
    if (p < o && q < o) {
      const int64_t ji = (int64_t)q * o + p;
      x = scal(-1.0, add(ld(Go, ji), ld(M, ji)));
    } else if (p < o) {
      x = ld(l1, (int64_t)p * v + (q - o));
    } else if (q < o) {
      x = ld(Dvo, (int64_t)q * v + (p - o));
    } else {
      const int a = p - o, b = q - o;
      x = sub(ld(N, (int64_t)a * v + b), ld(Gv, (int64_t)b * v + a));
    }
    st(g, t, x);
  }
}

__global__ void cast_kernel(const double* __restrict__ in, float* __restrict__ out, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * TB + threadIdx.x; t < n; t += (int64_t)gridDim.x * TB)
    out[t] = (float)in[t];
}

// out = FP32(a - b), n reals (the difference is formed in FP64, then rounded)
__global__ void diff_cast_kernel(const double* __restrict__ a, const double* __restrict__ b,
                                 float* __restrict__ out, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * TB + threadIdx.x; t < n; t += (int64_t)gridDim.x * TB)
    out[t] = (float)(a[t] - b[t]);
}

// y += a (+ c, promoted to FP64, when c is given), n reals
__global__ void add2_kernel(double* __restrict__ y, const double* __restrict__ a, const float* __restrict__ c,
                            int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * TB + threadIdx.x; t < n; t += (int64_t)gridDim.x * TB)
    y[t] += c ? a[t] + (double)c[t] : a[t];
}

}  // namespace

// ------------------------------------------------------------------ launchers
void k_conj_rows(double* dst, const double* src, int64_t rows, int64_t src_stride, int64_t len,
                 hipStream_t s) {
  const int64_t tot = rows * len;
  if (tot <= 0) return;
  hipLaunchKernelGGL(conj_rows_kernel, dim3(nblocks(tot)), dim3(TB), 0, s, dst, src, rows, src_stride, len);
  HIPCHECK(hipGetLastError());
}
void k_lambda_density(const double* Go, const double* M, const double* l1, const double* Dvo,
                      const double* Gv, const double* N, int o, int v, double* gamma, hipStream_t s) {
  const int64_t tot = (int64_t)(o + v) * (o + v);
  hipLaunchKernelGGL(lambda_density_kernel, dim3(nblocks(tot)), dim3(TB), 0, s, Go, M, l1, Dvo, Gv, N, o,
                     v, gamma);
  HIPCHECK(hipGetLastError());
}
void k_cast(const double* in, float* out, int64_t nreal, hipStream_t s) {
  if (nreal <= 0) return;
  hipLaunchKernelGGL(cast_kernel, dim3(nblocks(nreal)), dim3(TB), 0, s, in, out, nreal);
  HIPCHECK(hipGetLastError());
}
void k_diff_cast(const double* a, const double* b, float* out, int64_t nreal, hipStream_t s) {
  if (nreal <= 0) return;
  hipLaunchKernelGGL(diff_cast_kernel, dim3(nblocks(nreal)), dim3(TB), 0, s, a, b, out, nreal);
  HIPCHECK(hipGetLastError());
}
void k_add2(double* y, const double* a, const float* c, int64_t nreal, hipStream_t s) {
  if (nreal <= 0) return;
  hipLaunchKernelGGL(add2_kernel, dim3(nblocks(nreal)), dim3(TB), 0, s, y, a, c, nreal);
  HIPCHECK(hipGetLastError());
}
void k_transpose_B(const double* B, double* Bt, int64_t X, int64_t nn, hipStream_t s) {
  dim3 grid((unsigned)((nn + 31) / 32), (unsigned)((X + 31) / 32)), block(32, 8);
  hipLaunchKernelGGL(transpose_B_kernel, grid, block, 0, s, B, Bt, X, nn);
  HIPCHECK(hipGetLastError());
}

void k_check_B(const double* B, int64_t X, int n, double* out3, double* scratch, hipStream_t s) {
  const int nb = 1024;
  hipLaunchKernelGGL(check_B_kernel, dim3(nb), dim3(TB), 0, s, B, X, n, scratch);
  HIPCHECK(hipGetLastError());
  hipLaunchKernelGGL(check_B_final, dim3(1), dim3(64), 0, s, scratch, nb, out3);
  HIPCHECK(hipGetLastError());
}

template <typename T>
void k_pack_last2(T* out, const T* in, const int* rowmap, int64_t rows, int m, int64_t in_row_stride,
                  hipStream_t s) {
  const int64_t tot = rows * ((int64_t)m * (m - 1) / 2);
  if (tot <= 0) return;
  hipLaunchKernelGGL(pack_last2_kernel<T>, dim3(nblocks(tot)), dim3(TB), 0, s, out, in, rowmap, rows,
                     m, in_row_stride);
  HIPCHECK(hipGetLastError());
}

template <typename T>
void k_unpack_tau(const double* t1, const double* t2p, T* T2, T* TAU, T* taup, int o, int v,
                  hipStream_t s) {
  const int64_t tot = (int64_t)o * o * v * v;
  hipLaunchKernelGGL(unpack_tau_kernel<T>, dim3(nblocks(tot)), dim3(TB), 0, s, t1, t2p, T2, TAU, taup,
                     o, v);
  HIPCHECK(hipGetLastError());
}

template <typename T>
void k_ring_operands(const T* T2, const double* t1, T* Tq, T* Xp, int o, int v, hipStream_t s,
                     const double* t1r) {
  const int64_t oo = (int64_t)o * o;
  if (oo > 65535) raise(-5, "nocc too large for ring operand permute");
  dim3 grid((v + 31) / 32, (v + 31) / 32, (unsigned)oo), block(32, 8);
  hipLaunchKernelGGL(ring_operands_kernel<T>, grid, block, 0, s, T2, t1, Tq, Xp, o, v, t1r);
  HIPCHECK(hipGetLastError());
}

template <typename T>
void k_expand_c(const T* Vooov, const T* Cp, T* Cf, int o, int v, hipStream_t s) {
  const int64_t tot = (int64_t)o * o * o * v;
  hipLaunchKernelGGL(expand_c_kernel<T>, dim3(nblocks(tot)), dim3(TB), 0, s, Vooov, Cp, Cf, o, v);
  HIPCHECK(hipGetLastError());
}

template <typename T>
void k_ladder_antisym(const T* Ta, T* W, int nb, int v, int64_t ldw, hipStream_t s) {
  if (nb <= 0 || v < 2) return;
  const int nt = (v + 31) / 32;
  if (nb > 65535) raise(-5, "ladder row too long");
  dim3 grid((unsigned)(nt * (nt + 1) / 2), (unsigned)nb), block(32, 8);
  hipLaunchKernelGGL(ladder_antisym_kernel<T>, grid, block, 0, s, Ta, W, nb, v, ldw);
  HIPCHECK(hipGetLastError());
}

template <typename T>
void k_ladder_antisym_all(const T* Tf, T* W, int v, hipStream_t s) {
  if (v < 2) return;
  const int nt = (v + 31) / 32;
  if (v > 65535) raise(-5, "ladder too wide");
  dim3 grid((unsigned)(nt * (nt + 1) / 2), (unsigned)(v - 1), (unsigned)(v - 1)), block(32, 8);
  hipLaunchKernelGGL(ladder_antisym_all_kernel<T>, grid, block, 0, s, Tf, W, v);
  HIPCHECK(hipGetLastError());
}

template <typename T>
void k_transpose_tail(const T* W, int64_t rows, int64_t ldw, int64_t col0, int64_t ncols, T* Wt,
                      int64_t ldt, hipStream_t s) {
  if (rows <= 0 || ncols <= 0) return;
  const int64_t gx = (ncols + 31) / 32, gy = (rows + 31) / 32;
  if (gx > 0x7fffffffLL || gy > 65535) raise(-5, "ladder tail too large to transpose");
  hipLaunchKernelGGL(transpose_tail_kernel<T>, dim3((unsigned)gx, (unsigned)gy), dim3(32, 8), 0, s, W,
                     rows, ldw, col0, ncols, Wt, ldt);
  HIPCHECK(hipGetLastError());
}

int assemble_t2_blocks(int64_t npairs) { return nblocks(npairs, 4096); }
int dot_many_blocks(int64_t len) { return nblocks(len, 2048); }
int energy_blocks(int64_t npairs) { return nblocks(npairs, 2048); }

template <typename T>
void k_assemble_t2(const T* Znp, const T* Z, const T* R, const double* Voovv_p, const double* t2p,
                   const double* eps, int o, int v, double shift, double* xt, double* e,
                   double* s2_full, double* partial, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(assemble_t2_kernel<T>, dim3(nblk), dim3(TB), 0, s, Znp, Z, R, Voovv_p, t2p, eps,
                     o, v, shift, xt, e, s2_full, partial);
  HIPCHECK(hipGetLastError());
}

// T1-dressed virtual-occupied DF factor (CC2 doubles): Vt[a][i][P] holds
// sum_c B^P_ac t_i^c on entry and B^P_ai + sum_c B^P_ac t_i^c - Q[a][i][P] on exit,
// with Q^P_ai = sum_k t_k^a (B^P_ki + sum_d B^P_kd t_i^d); Bt is [p][q][P].
template <typename T>
__global__ void dress_vo_kernel(T* __restrict__ Vt, const T* __restrict__ Bt, const T* __restrict__ Q,
                                int o, int v, int n, int X) {
  const int64_t tot = (int64_t)v * o * X;
  for (int64_t t = (int64_t)blockIdx.x * TB + threadIdx.x; t < tot; t += (int64_t)gridDim.x * TB) {
    const int64_t ai = t / X, P = t - ai * X;
    const int a = (int)(ai / o), i = (int)(ai - (int64_t)a * o);
    const z b = ld(Bt, ((int64_t)(o + a) * n + i) * X + P);
    st(Vt, t, add(ld(Vt, t), sub(b, ld(Q, t))));
  }
}

template <typename T>
void k_dress_vo(T* Vt, const T* Bt, const T* Q, int o, int v, int n, int X, hipStream_t s) {
  const int64_t tot = (int64_t)v * o * X;
  if (tot <= 0) return;
  hipLaunchKernelGGL(dress_vo_kernel<T>, dim3(nblocks(tot)), dim3(TB), 0, s, Vt, Bt, Q, o, v, n, X);
  HIPCHECK(hipGetLastError());
}

// Perturbative triples (App. C), a batch of occupied triples (i0 + y, j, k), y < ni,
// i0 + ni <= j < k, with W = We + Wm held packed: We[y][(a<b)][c] (the sum over e,
// antisymmetric in (a, b)) and Wm[y][a][(b<c)] (the sum over m, antisymmetric in (b, c)),
// Pv v each, and the full T2 [i][j][a][b].  W~, Z~ and Y~ are fully antisymmetric in
// (a, b, c), so only a < b < c is evaluated, with weight 6:
//   W~ = W[a,b,c] + W[b,c,a] + W[c,a,b]
//      = We(ab,c) + We(bc,a) - We(ac,b) + Wm(a,bc) - Wm(b,ac) + Wm(c,ab)
//   Z~ = Z(a,b,c) + Z(c,a,b) + Z(b,c,a),  Z(a,b,c) = <ab||ij> t_k^c + <ab||jk> t_i^c
//        + <ab||ki> t_j^c with <ab||xy> = conj(<xy||ab>) from Voovv [x][y][a][b]
//   Y~ = Y(a,b,c) + Y(c,a,b) + Y(b,c,a),  Y(a,b,c) = (1/3) sum over the permutations p
//        of (i,j,k) of sign(p) t_p1^a t_p2^b t_p3^c + t_ij^ab t_k^c + t_jk^ab t_i^c
//        + t_ki^ab t_j^c
//   e4 += -6 |W~|^2 / D,  e5 += -6 Re(conj(Z~) W~) / D,  ey += 6 Re(conj(Y~) W~),
//   D = e_a + e_b + e_c - e_i - e_j - e_k.
// One workgroup per triple of 8-wide virtual tiles (tA <= tB <= tC).  Staged in LDS, each
// read with its contiguous index fastest (every global read coalesced): the six 8x8x8 cubes
// of packed values that W~ needs on (A, B, C); the 8x8 blocks of <xy||pq> and t_xy^pq for
// the three occupied pairs (ij, jk, ki) and the three virtual tile pairs (AB, CA, BC) that
// Z~ and Y~ read; and t_x^p for x in (i, j, k) on the three tiles.  Then each thread
// evaluates its a < b < c points.  Block partial sums (e4, e5, ey) to
// part[4 * (y * gridDim.x + block)].
__global__ void triples_energy_kernel(const double* __restrict__ Web, const double* __restrict__ Wmb,
                                      const double* __restrict__ Voovv,
                                      const double* __restrict__ T2, const double* __restrict__ t1,
                                      const double* __restrict__ eps, int i0, int j, int k, int o, int v,
                                      double* __restrict__ part) {
  const int64_t vv = (int64_t)v * v, Pv = (int64_t)v * (v - 1) / 2;
  const int i = i0 + (int)blockIdx.y;
  const double* __restrict__ We = Web + 2 * (int64_t)blockIdx.y * Pv * v;
  const double* __restrict__ Wm = Wmb + 2 * (int64_t)blockIdx.y * Pv * v;
  // packed parts at p < q (p, q, r < v)
  auto Ep = [&](int p, int q, int r) { return ld(We, pidx(p, q, v) * v + r); };
  auto Mp = [&](int r, int p, int q) { return ld(Wm, (int64_t)r * Pv + pidx(p, q, v)); };
  // tile triple of this workgroup
  const int nt = (v + 7) / 8;
  int rem = (int)blockIdx.x, ta = 0;
  while (rem >= (nt - ta) * (nt - ta + 1) / 2) {
    rem -= (nt - ta) * (nt - ta + 1) / 2;
    ++ta;
  }
  int tb = ta;
  while (rem >= nt - tb) {
    rem -= nt - tb;
    ++tb;
  }
  const int tc = tb + rem;
  const int a0 = 8 * ta, b0 = 8 * tb, c0 = 8 * tc;
  // cube q at LDS index (x * 8 + y) * 8 + w holds its value for (a, b, c) = (a0+x, b0+y, c0+w);
  // entries whose pair is not p < q (unused by a < b < c) are zero
  __shared__ double qr[6][512], qi[6][512];
  for (int e = threadIdx.x; e < 512; e += TB) {
    const int u = e >> 6, m = (e >> 3) & 7, f = e & 7;  // f fastest
    z g[6];
    int at[6];
    // 0: We(ab, c), c fastest;  3: Wm(a, bc), c fastest;  4: Wm(b, ac), c fastest
    {
      const int a = a0 + u, b = b0 + m, c = c0 + f;
      const bool in = a < v && b < v && c < v;
      g[0] = (in && a < b) ? Ep(a, b, c) : z{0, 0};
      g[3] = (in && b < c) ? Mp(a, b, c) : z{0, 0};
      g[4] = (in && a < c) ? Mp(b, a, c) : z{0, 0};
      at[0] = at[3] = at[4] = (u * 8 + m) * 8 + f;
    }
    // 1: We(bc, a), a fastest
    {
      const int b = b0 + u, c = c0 + m, a = a0 + f;
      g[1] = (a < v && b < v && c < v && b < c) ? Ep(b, c, a) : z{0, 0};
      at[1] = (f * 8 + u) * 8 + m;
    }
    // 2: We(ac, b), b fastest;  5: Wm(c, ab), b fastest
    {
      const int a = a0 + u, c = c0 + m, b = b0 + f;
      const bool in = a < v && b < v && c < v;
      g[2] = (in && a < c) ? Ep(a, c, b) : z{0, 0};
      g[5] = (in && a < b) ? Mp(c, a, b) : z{0, 0};
      at[2] = at[5] = (u * 8 + f) * 8 + m;
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      qr[q][at[q]] = g[q].x;
      qi[q][at[q]] = g[q].y;
    }
  }
  // block 3 p + r, cell 8 row + col: <pair p||tile pair r> (conjugated) and t_(pair p)^(tile pair
  // r); pairs p = (ij, jk, ki), tile pairs r = (AB, CA, BC) as (row, col); t1s[x][8 tile + w]
  // = t_x^(tile start + w) for x = (i, j, k), tiles (A, B, C)
  __shared__ double vr[9][64], vi[9][64], sr[9][64], si[9][64], t1r[3][24], t1i[3][24];
  const int xs[3] = {i, j, k};
  for (int e = threadIdx.x; e < 9 * 64; e += TB) {
    const int blk = e >> 6, cell = e & 63, r = cell >> 3, c = cell & 7;
    const int p = blk / 3, role = blk - 3 * p;
    const int x = xs[p], y = xs[p == 2 ? 0 : p + 1];
    const int row = (role == 0 ? a0 : role == 1 ? c0 : b0) + r;
    const int col = (role == 0 ? b0 : role == 1 ? a0 : c0) + c;
    z g{0, 0}, h{0, 0};
    if (row < v && col < v) {
      const int64_t off = ((int64_t)x * o + y) * vv + (int64_t)row * v + col;
      g = ld(Voovv, off);
      h = ld(T2, off);
    }
    vr[blk][cell] = g.x;
    vi[blk][cell] = -g.y;
    sr[blk][cell] = h.x;
    si[blk][cell] = h.y;
  }
  for (int e = threadIdx.x; e < 72; e += TB) {
    const int xi = e / 24, q = e - 24 * xi, tile = q >> 3, w = q & 7;
    const int col = (tile == 0 ? a0 : tile == 1 ? b0 : c0) + w;
    const z g = col < v ? ld(t1, (int64_t)xs[xi] * v + col) : z{0, 0};
    t1r[xi][q] = g.x;
    t1i[xi][q] = g.y;
  }
  __syncthreads();
  auto T1 = [&](int x, int q) { return z{t1r[x][q], t1i[x][q]}; };
  auto Vs = [&](int blk, int cell) { return z{vr[blk][cell], vi[blk][cell]}; };
  auto Ts = [&](int blk, int cell) { return z{sr[blk][cell], si[blk][cell]}; };
  // Z(p, q, r) and Y(p, q, r) for (p, q, r) one of (a, b, c), (c, a, b), (b, c, a): tile pair
  // `role` of (p, q), its cell, and the t1s columns qp, qq, qr of p, q, r
  auto Zr = [&](int role, int cell, int qr_) {
    z r = mul(Vs(role, cell), T1(2, qr_));
    r = add(r, mul(Vs(3 + role, cell), T1(0, qr_)));
    return add(r, mul(Vs(6 + role, cell), T1(1, qr_)));
  };
  auto Yr = [&](int role, int cell, int qp, int qq, int qr_) {
    z d = mul(mul(T1(0, qp), T1(1, qq)), T1(2, qr_));
    d = sub(d, mul(mul(T1(1, qp), T1(0, qq)), T1(2, qr_)));
    d = add(d, mul(mul(T1(1, qp), T1(2, qq)), T1(0, qr_)));
    d = sub(d, mul(mul(T1(2, qp), T1(1, qq)), T1(0, qr_)));
    d = add(d, mul(mul(T1(2, qp), T1(0, qq)), T1(1, qr_)));
    d = sub(d, mul(mul(T1(0, qp), T1(2, qq)), T1(1, qr_)));
    z r = scal(1.0 / 3.0, d);
    r = add(r, mul(Ts(role, cell), T1(2, qr_)));
    r = add(r, mul(Ts(3 + role, cell), T1(0, qr_)));
    return add(r, mul(Ts(6 + role, cell), T1(1, qr_)));
  };
  double e4 = 0, e5 = 0, ey = 0;
  const double eo = eps[i] + eps[j] + eps[k];
  for (int e = threadIdx.x; e < 512; e += TB) {
    const int x = e >> 6, y = (e >> 3) & 7, w = e & 7;
    const int a = a0 + x, b = b0 + y, c = c0 + w;
    if (!(c < v && a < b && b < c)) continue;
    const z wt{qr[0][e] + qr[1][e] - qr[2][e] + qr[3][e] - qr[4][e] + qr[5][e],
               qi[0][e] + qi[1][e] - qi[2][e] + qi[3][e] - qi[4][e] + qi[5][e]};
    const int qa = x, qb = 8 + y, qc = 16 + w;
    const z zz = add(Zr(0, x * 8 + y, qc), add(Zr(1, w * 8 + x, qb), Zr(2, y * 8 + w, qa)));
    const z yy = add(Yr(0, x * 8 + y, qa, qb, qc),
                     add(Yr(1, w * 8 + x, qc, qa, qb), Yr(2, y * 8 + w, qb, qc, qa)));
    const double D = eps[o + a] + eps[o + b] + eps[o + c] - eo;
    e4 -= 6.0 * (wt.x * wt.x + wt.y * wt.y) / D;
    e5 -= 6.0 * (zz.x * wt.x + zz.y * wt.y) / D;
    ey += 6.0 * (yy.x * wt.x + yy.y * wt.y);
  }
  __shared__ double s4[TB], s5[TB], sy[TB];
  s4[threadIdx.x] = e4;
  s5[threadIdx.x] = e5;
  sy[threadIdx.x] = ey;
  __syncthreads();
  for (int s = TB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      s4[threadIdx.x] += s4[threadIdx.x + s];
      s5[threadIdx.x] += s5[threadIdx.x + s];
      sy[threadIdx.x] += sy[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t q = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    part[4 * q] = s4[0];
    part[4 * q + 1] = s5[0];
    part[4 * q + 2] = sy[0];
  }
}

// Acat[y][a][t][m] = conj(<x_t y_t||m a>) for the two sums over m of a triples batch whose
// excitation elements depend on i = i0 + y: t = 0 -> <k i||m a>, t = 1 -> <i j||m a>
// (Vooov [x][y][m][a])
__global__ void triples_acat_kernel(const double* __restrict__ Vooov, int i0, int ni, int j, int k,
                                    int o, int v, double* __restrict__ out) {
  const int64_t tot = (int64_t)ni * v * 2 * o;
  for (int64_t t = (int64_t)blockIdx.x * TB + threadIdx.x; t < tot; t += (int64_t)gridDim.x * TB) {
    const int m = (int)(t % o);
    int64_t r = t / o;
    const int tt = (int)(r % 2);
    r /= 2;
    const int a = (int)(r % v);
    const int y = (int)(r / v);
    const int i = i0 + y;
    const int x0 = tt == 0 ? k : i, y0 = tt == 0 ? i : j;
    const z g = ld(Vooov, (((int64_t)x0 * o + y0) * o + m) * v + a);
    st(out, t, z{g.x, -g.y});
  }
}

// One block per triple of the batch: the nblk partials in a fixed order, to
// out[4 * (((i0 + y) * o + j) * o + k)] (three values).
__global__ void triples_reduce_kernel(const double* __restrict__ part, int nblk, int i0, int j, int k,
                                      int o, double* __restrict__ out) {
  __shared__ double s4[TB], s5[TB], sy[TB];
  const double* p = part + 4 * (int64_t)blockIdx.x * nblk;
  double a = 0, b = 0, c = 0;
  for (int q = threadIdx.x; q < nblk; q += TB) {
    a += p[4 * q];
    b += p[4 * q + 1];
    c += p[4 * q + 2];
  }
  s4[threadIdx.x] = a;
  s5[threadIdx.x] = b;
  sy[threadIdx.x] = c;
  __syncthreads();
  for (int s = TB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      s4[threadIdx.x] += s4[threadIdx.x + s];
      s5[threadIdx.x] += s5[threadIdx.x + s];
      sy[threadIdx.x] += sy[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t idx = ((int64_t)(i0 + blockIdx.x) * o + j) * o + k;
    out[4 * idx] = s4[0];
    out[4 * idx + 1] = s5[0];
    out[4 * idx + 2] = sy[0];
  }
}

// Fill and copy of nbytes (a multiple of 8) with 16-byte or 8-byte vector stores: the
// stream-ordered zero and device-to-device copy of the iteration, as kernels so that a
// captured iteration graph holds kernel nodes only.
template <typename V>
__global__ void fill_zero_kernel(V* __restrict__ p, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * TB + threadIdx.x; t < n; t += (int64_t)gridDim.x * TB) p[t] = V{};
}
template <typename V>
__global__ void copy_words_kernel(V* __restrict__ d, const V* __restrict__ src, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * TB + threadIdx.x; t < n; t += (int64_t)gridDim.x * TB) d[t] = src[t];
}

void k_zero_bytes(void* p, int64_t nbytes, hipStream_t s) {
  if (nbytes <= 0) return;
  typedef unsigned u4 __attribute__((ext_vector_type(4)));
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  if (reinterpret_cast<uintptr_t>(p) % 16 == 0 && nbytes % 16 == 0) {
    const int64_t n = nbytes / 16;
    hipLaunchKernelGGL(fill_zero_kernel<u4>, dim3(nblocks(n)), dim3(TB), 0, s, (u4*)p, n);
  } else {
    const int64_t n = nbytes / 8;
    hipLaunchKernelGGL(fill_zero_kernel<u2>, dim3(nblocks(n)), dim3(TB), 0, s, (u2*)p, n);
  }
  HIPCHECK(hipGetLastError());
}

void k_copy_bytes(void* d, const void* src, int64_t nbytes, hipStream_t s) {
  if (nbytes <= 0) return;
  typedef unsigned u4 __attribute__((ext_vector_type(4)));
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  if (reinterpret_cast<uintptr_t>(d) % 16 == 0 && reinterpret_cast<uintptr_t>(src) % 16 == 0 &&
      nbytes % 16 == 0) {
    const int64_t n = nbytes / 16;
    hipLaunchKernelGGL(copy_words_kernel<u4>, dim3(nblocks(n)), dim3(TB), 0, s, (u4*)d, (const u4*)src, n);
  } else {
    const int64_t n = nbytes / 8;
    hipLaunchKernelGGL(copy_words_kernel<u2>, dim3(nblocks(n)), dim3(TB), 0, s, (u2*)d, (const u2*)src, n);
  }
  HIPCHECK(hipGetLastError());
}

void k_triples_acat(const double* Vooov, int i0, int ni, int j, int k, int o, int v, double* out,
                    hipStream_t s) {
  const int64_t tot = (int64_t)ni * v * 2 * o;
  if (tot <= 0) return;
  hipLaunchKernelGGL(triples_acat_kernel, dim3(nblocks(tot)), dim3(TB), 0, s, Vooov, i0, ni, j, k, o, v, out);
  HIPCHECK(hipGetLastError());
}

int triples_blocks(int v) {
  const int64_t nt = (v + 7) / 8;
  return (int)(nt * (nt + 1) * (nt + 2) / 6);
}

void k_triples_energy(const double* We, const double* Wm, const double* Voovv, const double* T2,
                      const double* t1, const double* eps, int i0, int ni, int j, int k, int o, int v,
                      double* partial, int nblk, double* out, hipStream_t s) {
  if (ni <= 0) return;
  hipLaunchKernelGGL(triples_energy_kernel, dim3(nblk, ni), dim3(TB), 0, s, We, Wm, Voovv, T2, t1, eps, i0,
                     j, k, o, v, partial);
  HIPCHECK(hipGetLastError());
  hipLaunchKernelGGL(triples_reduce_kernel, dim3(ni), dim3(TB), 0, s, partial, nblk, i0, j, k, o, out);
  HIPCHECK(hipGetLastError());
}

template <typename T>
void k_assemble_t1(const T* S1, const double* t1, const double* eps, int o, int v, double shift,
                   bool frozen, double* xt, double* e, double* s1_full, double* partial, hipStream_t s) {
  hipLaunchKernelGGL(assemble_t1_kernel<T>, dim3(1), dim3(TB), 0, s, S1, t1, eps, o, v, shift,
                     frozen ? 1 : 0, xt, e, s1_full, partial);
  HIPCHECK(hipGetLastError());
}

void k_reduce_sum(const double* partial, int n, int width, double* out, hipStream_t s) {
  hipLaunchKernelGGL(reduce_sum_kernel, dim3(1), dim3(TB), 0, s, partial, n, width, out);
  HIPCHECK(hipGetLastError());
}

void k_dot_many(const double* const* es, int m, const double* e, int64_t len, double* partial,
                int nblk, hipStream_t s) {
  if (m > MAXV) raise(-1, "DIIS subspace larger than 16");
  Ptrs p{};
  for (int k = 0; k < m; ++k) p.p[k] = es[k];
  hipLaunchKernelGGL(dot_many_kernel, dim3(nblk), dim3(TB), 0, s, p, m, e, len, partial);
  HIPCHECK(hipGetLastError());
}

void k_lincomb(double* x, const double* const* xs, const cplx* c, int m, int64_t len, hipStream_t s) {
  if (m > MAXV) raise(-1, "DIIS subspace larger than 16");
  Ptrs p{};
  Coefs cc{};
  for (int k = 0; k < m; ++k) {
    p.p[k] = xs[k];
    cc.re[k] = c[k].re;
    cc.im[k] = c[k].im;
  }
  hipLaunchKernelGGL(lincomb_kernel, dim3(nblocks(len, 8192)), dim3(TB), 0, s, x, p, cc, m, len);
  HIPCHECK(hipGetLastError());
}

void k_energy(const double* Voovv_p, const double* t2p, const double* t1, int o, int v,
              double* partial, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(energy_kernel, dim3(nblk), dim3(TB), 0, s, Voovv_p, t2p, t1, o, v, partial);
  HIPCHECK(hipGetLastError());
}

void k_unpack_full(const double* t1, const double* t2p, double* t1_out, double* t2_out, int o, int v,
                   hipStream_t s) {
  (void)t1;
  (void)t1_out;
  const int64_t tot = (int64_t)o * o * v * v;
  hipLaunchKernelGGL(unpack_full_kernel, dim3(nblocks(tot)), dim3(TB), 0, s, t2p, t2_out, o, v);
  HIPCHECK(hipGetLastError());
}

void k_unpack_diff(const double* t2p, const double* r2p, float* t2_out, int o, int v, hipStream_t s) {
  const int64_t tot = (int64_t)o * o * v * v;
  if (tot <= 0) return;
  hipLaunchKernelGGL(unpack_diff_kernel, dim3(nblocks(tot)), dim3(TB), 0, s, t2p, r2p, t2_out, o, v);
  HIPCHECK(hipGetLastError());
}

void k_sub(const double* a, const double* b, double* out, int64_t nreal, hipStream_t s) {
  if (nreal <= 0) return;
  hipLaunchKernelGGL(sub_kernel, dim3(nblocks(nreal)), dim3(TB), 0, s, a, b, out, nreal);
  HIPCHECK(hipGetLastError());
}

void k_pack_amplitudes(const double* t1, const double* t2, double* x, int o, int v, hipStream_t s) {
  (void)t1;
  const int64_t tot = ((int64_t)o * (o - 1) / 2) * ((int64_t)v * (v - 1) / 2);
  if (tot <= 0) return;
  hipLaunchKernelGGL(pack_amp_kernel, dim3(nblocks(tot)), dim3(TB), 0, s, t2, x, o, v);
  HIPCHECK(hipGetLastError());
}

#define EXACC_INST(T)                                                                          \
  template void k_pack_last2<T>(T*, const T*, const int*, int64_t, int, int64_t, hipStream_t);   \
  template void k_unpack_tau<T>(const double*, const double*, T*, T*, T*, int, int, hipStream_t); \
  template void k_ring_operands<T>(const T*, const double*, T*, T*, int, int, hipStream_t,       \
                                   const double*);                                               \
  template void k_expand_c<T>(const T*, const T*, T*, int, int, hipStream_t);                    \
  template void k_ladder_antisym<T>(const T*, T*, int, int, int64_t, hipStream_t);               \
  template void k_ladder_antisym_all<T>(const T*, T*, int, hipStream_t);                          \
  template void k_transpose_tail<T>(const T*, int64_t, int64_t, int64_t, int64_t, T*, int64_t,       \
                                    hipStream_t);                                                 \
  template void k_assemble_t2<T>(const T*, const T*, const T*, const double*, const double*,     \
                                 const double*, int, int, double, double*, double*, double*,     \
                                 double*, int, hipStream_t);                                      \
  template void k_assemble_t1<T>(const T*, const double*, const double*, int, int, double, bool, \
                                 double*, double*, double*, double*, hipStream_t);               \
  template void k_dress_vo<T>(T*, const T*, const T*, int, int, int, int, hipStream_t);
EXACC_INST(double)
EXACC_INST(float)
#undef EXACC_INST

}  // namespace exacc
