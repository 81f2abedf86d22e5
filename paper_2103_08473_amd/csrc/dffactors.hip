// Density-fitting factors from AO three-index integrals, the step before the CC
// iteration (robust fitting; the paper's Introduction names density fitting and
// Cholesky decomposition for the integral tensor, its Performance section the cost of
// the AO->MO transformation):
//
//   B^P_pq = sum_Q [V^-1/2]_PQ sum_{mu nu} conj(C_mu p) (mu nu|Q) C_nu q.
//
// V^-1/2 comes from the coupled Newton-Schulz iteration (Higham, Functions of
// Matrices, 2008, the coupled Newton-Schulz iteration for the matrix square root),
// which needs only matrix products and therefore runs on the same MFMA GETT as
// everything else: with A = V / c (c = max row sum of |V| >= the largest eigenvalue,
// so the spectrum of A lies in (0, 1]), Y_0 = A, Z_0 = I,
//   P_k = Z_k Y_k,  T_k = (3 I - P_k) / 2,  Y_{k+1} = Y_k T_k,  Z_{k+1} = T_k Z_k,
// Z_k -> A^-1/2 quadratically once ||I - P_k|| is small; V^-1/2 = Z / sqrt(c).  The two
// transform GEMMs and the metric GEMM then give B.
#include <algorithm>
#include <cmath>
#include <utility>
#include <vector>

#include "common.h"
#include "einsum.h"

namespace exacc {
namespace {

constexpr int kTB = 256;

inline int nblk(int64_t n, int cap = 4096) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + kTB - 1) / kTB, cap));
}

// out[i] = sum_j |V[i][j]|
__global__ void row_abs_sum_kernel(const double* __restrict__ V, int X, double* __restrict__ out) {
  for (int i = blockIdx.x * kTB + threadIdx.x; i < X; i += gridDim.x * kTB) {
    double s = 0.0;
    for (int j = 0; j < X; ++j) s += fabs(V[(int64_t)i * X + j]);
    out[i] = s;
  }
}

// A = V * inv_c (complex, zero imaginary part), Z = I
__global__ void ns_init_kernel(const double* __restrict__ V, int X, double inv_c, double* __restrict__ A,
                               double* __restrict__ Z) {
  const int64_t tot = (int64_t)X * X;
  for (int64_t t = (int64_t)blockIdx.x * kTB + threadIdx.x; t < tot; t += (int64_t)gridDim.x * kTB) {
    const int64_t i = t / X, j = t - i * X;
    A[2 * t] = V[t] * inv_c;
    A[2 * t + 1] = 0.0;
    Z[2 * t] = (i == j) ? 1.0 : 0.0;
    Z[2 * t + 1] = 0.0;
  }
}

// T = (3 I - P) / 2 and per-block partial sums of |I - P|^2
__global__ void ns_step_kernel(const double* __restrict__ P, int X, double* __restrict__ T,
                               double* __restrict__ part) {
  const int64_t tot = (int64_t)X * X;
  double acc = 0.0;
  for (int64_t t = (int64_t)blockIdx.x * kTB + threadIdx.x; t < tot; t += (int64_t)gridDim.x * kTB) {
    const int64_t i = t / X, j = t - i * X;
    const double d = (i == j) ? 1.0 : 0.0;
    const double pr = P[2 * t], pi = P[2 * t + 1];
    acc += (d - pr) * (d - pr) + pi * pi;
    T[2 * t] = 0.5 * (3.0 * d - pr);
    T[2 * t + 1] = -0.5 * pi;
  }
  __shared__ double sh[kTB];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kTB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Device buffers of one call, freed on every exit path.
struct Pool {
  std::vector<void*> mem;
  std::vector<AllocRange> ranges;
  ~Pool() {
    for (void* p : mem) (void)hipFree(p);
    set_alloc_registry(nullptr, 0);
    set_gett_workspace(nullptr, 0);
  }
  double* alloc(size_t bytes) {
    void* p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(bytes, 16)) != hipSuccess) {
      (void)hipGetLastError();
      raise(-2, "DF factors: device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    mem.push_back(p);
    ranges.push_back({p, std::max<size_t>(bytes, 16)});
    set_alloc_registry(ranges.data(), (int)ranges.size());
    return (double*)p;
  }
  void add(const void* p, size_t bytes) {
    ranges.push_back({p, bytes});
    set_alloc_registry(ranges.data(), (int)ranges.size());
  }
};

}  // namespace

int df_factors_impl(int m, int n, int X, const double* C, const double* J, const double* V, double* B,
                    bool on_device, hipStream_t s) {
  const cplx ONE{1.0, 0.0};
  Pool pool;
  const size_t bC = (size_t)m * n * 16, bJ = (size_t)X * m * m * 16, bV = (size_t)X * X * 8,
               bB = (size_t)X * n * n * 16, bXX = (size_t)X * X * 16;
  const double *Cd = C, *Jd = J, *Vd = V;
  double* Bd = B;
  if (on_device) {
    pool.add(C, bC);
    pool.add(J, bJ);
    pool.add(V, bV);
    pool.add(B, bB);
  } else {
    double* c = pool.alloc(bC);
    double* j = pool.alloc(bJ);
    double* v = pool.alloc(bV);
    HIPCHECK(hipMemcpyAsync(c, C, bC, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(j, J, bJ, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(v, V, bV, hipMemcpyHostToDevice, s));
    Cd = c;
    Jd = j;
    Vd = v;
    Bd = pool.alloc(bB);
  }
  double* Y = pool.alloc(bXX);
  double* Z = pool.alloc(bXX);
  double* P = pool.alloc(bXX);
  double* T = pool.alloc(bXX);
  double* Y2 = pool.alloc(bXX);
  double* Z2 = pool.alloc(bXX);
  double* T1 = pool.alloc((size_t)X * n * m * 16);
  double* M = pool.alloc((size_t)X * n * n * 16);
  const int nb = nblk((int64_t)X * X);
  double* part = pool.alloc((size_t)(std::max(nb, X) + 8) * 8);
  double* red = pool.alloc(64);
  const size_t wsb = (size_t)64 << 20;
  set_gett_workspace(pool.alloc(wsb), wsb);
  std::vector<double> host(std::max(X, 2));

  // scale: c = max_i sum_j |V_ij| bounds the spectrum of the symmetric V from above
  hipLaunchKernelGGL(row_abs_sum_kernel, dim3(nblk(X, 1024)), dim3(kTB), 0, s, Vd, X, part);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipMemcpyAsync(host.data(), part, (size_t)X * 8, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  double c = 0.0;
  for (int i = 0; i < X; ++i) c = std::max(c, host[i]);
  if (!(c > 0.0) || !std::isfinite(c)) raise(-1, "DF factors: metric is zero or not finite");
  hipLaunchKernelGGL(ns_init_kernel, dim3(nb), dim3(kTB), 0, s, Vd, X, 1.0 / c, Y, Z);
  HIPCHECK(hipGetLastError());

  auto XXv = [&](double* p) { return view(p, {X, X}); };
  int iters = 0;
  bool done = false;
  for (; iters < 200 && !done; ++iters) {
    contract(s, "ab,bc->ac", ONE, XXv(Z), XXv(Y), false, XXv(P));
    hipLaunchKernelGGL(ns_step_kernel, dim3(nb), dim3(kTB), 0, s, P, X, T, part);
    HIPCHECK(hipGetLastError());
    k_reduce_sum(part, nb, 1, red, s);
    HIPCHECK(hipMemcpyAsync(host.data(), red, 8, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    const double r = std::sqrt(host[0]);
    if (!std::isfinite(r) || r > 1e3 * X) break;
    // quadratic phase: one more step takes the error to ~r^2 (rounding level)
    if (r < 1e-8) done = true;
    contract(s, "ab,bc->ac", ONE, XXv(Y), XXv(T), false, XXv(Y2));
    contract(s, "ab,bc->ac", ONE, XXv(T), XXv(Z), false, XXv(Z2));
    std::swap(Y, Y2);
    std::swap(Z, Z2);
  }
  if (!done)
    raise(-1, "DF factors: the inverse square root iteration did not converge (metric not positive "
              "definite or too ill-conditioned)");

  // (pq|Q) = sum_mu nu conj(C_mu p) (mu nu|Q) C_nu q, then B = V^-1/2 (pq|Q)
  contract(s, "mp,Qmn->Qpn", ONE, conj(view(const_cast<double*>(Cd), {m, n})),
           view(const_cast<double*>(Jd), {X, m, m}), false, view(T1, {X, n, m}));
  contract(s, "Qpn,nq->Qpq", ONE, view(T1, {X, n, m}), view(const_cast<double*>(Cd), {m, n}), false,
           view(M, {X, n, n}));
  contract(s, "PQ,Qx->Px", cplx{1.0 / std::sqrt(c), 0.0}, XXv(Z), view(M, {X, (int64_t)n * n}), false,
           view(Bd, {X, (int64_t)n * n}));
  if (!on_device) HIPCHECK(hipMemcpyAsync(B, Bd, bB, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  return iters;
}

}  // namespace exacc
