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
#include <mutex>
#include <string>
#include <utility>

#include "../../include/exacc.h"

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

// max over part[0..n) into out[0] (one workgroup; max is exact in any order)
__global__ void max_kernel(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double sh[kTB];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += kTB) m = fmax(m, part[i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = kTB / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

inline size_t up256(size_t b) { return (b + 255) / 256 * 256; }

// Bytes of the temporaries that do not depend on the slice width: the reduction
// scalars and partials and the six naux x naux Newton-Schulz matrices.
size_t fixed_bytes(int X) {
  const int64_t nb = nblk((int64_t)X * X);
  return up256(256) + up256((size_t)(std::max<int64_t>(nb, X) + 8) * 8) +
         6 * up256((size_t)X * X * 16);
}
// Bytes of the two transform intermediates for a slice of ps spinor rows p.
size_t slice_bytes(int m, int n, int X, int ps) {
  return up256((size_t)X * ps * m * 16) + up256((size_t)X * ps * n * 16);
}

// Bump allocation inside one device region that the caller owns.
struct Carve {
  char* base;
  size_t cap, used = 0;
  double* take(size_t bytes) {
    const size_t b = up256(std::max<size_t>(bytes, 16));
    if (used + b > cap) raise(-2, "DF factors: scratch region exhausted");
    double* p = reinterpret_cast<double*>(base + used);
    used += b;
    return p;
  }
};

// The planner's extent check and the split-K workspace are per thread; restore both.
struct PlannerState {
  AllocRange r[6];
  int n = 0;
  void add(const void* p, size_t bytes) {
    r[n++] = {p, bytes};
    set_alloc_registry(r, n);
  }
  ~PlannerState() {
    set_alloc_registry(nullptr, 0);
    set_gett_workspace(nullptr, 0);
  }
};

// B from device C, J, V with every temporary inside [base, base + cap): the fixed part,
// the transform intermediates for slices of ps spinor rows (the widest that fits, at most
// nspinor) and a split-K workspace of what is left, at most ws_cap.  Returns the
// Newton-Schulz step count.  Nothing in the region needs to start at zero: every
// temporary is written before it is read.
int df_core(int m, int n, int X, const double* Cd, const double* Jd, const double* Vd, double* Bd,
            hipStream_t s, char* base, size_t cap, size_t ws_cap) {
  const cplx ONE{1.0, 0.0};
  const size_t fixed = fixed_bytes(X);
  if (fixed + slice_bytes(m, n, X, 1) > cap) raise(-2, "DF factors: scratch region too small");
  int ps = n;
  while (ps > 1 && fixed + slice_bytes(m, n, X, ps) > cap) ps = std::max(1, ps / 2);
  PlannerState ps_state;
  ps_state.add(Cd, (size_t)m * n * 16);
  ps_state.add(Jd, (size_t)X * m * m * 16);
  ps_state.add(Vd, (size_t)X * X * 8);
  ps_state.add(Bd, (size_t)X * n * n * 16);
  ps_state.add(base, cap);
  Carve cv{base, cap};
  const int nb = nblk((int64_t)X * X);
  double* red = cv.take(256);
  double* part = cv.take((size_t)(std::max(nb, X) + 8) * 8);
  double* Y = cv.take((size_t)X * X * 16);
  double* Z = cv.take((size_t)X * X * 16);
  double* P = cv.take((size_t)X * X * 16);
  double* T = cv.take((size_t)X * X * 16);
  double* Y2 = cv.take((size_t)X * X * 16);
  double* Z2 = cv.take((size_t)X * X * 16);
  double* T1 = cv.take((size_t)X * ps * m * 16);
  double* M = cv.take((size_t)X * ps * n * 16);
  const size_t left = cap > cv.used ? (cap - cv.used) / 256 * 256 : 0;
  const size_t wsb = std::min(left, ws_cap);
  set_gett_workspace(wsb >= (1u << 20) ? cv.take(wsb) : nullptr, wsb >= (1u << 20) ? wsb : 0);
  double h1 = 0.0;

  // scale: c = max_i sum_j |V_ij| bounds the spectrum of the symmetric V from above
  hipLaunchKernelGGL(row_abs_sum_kernel, dim3(nblk(X, 1024)), dim3(kTB), 0, s, Vd, X, part);
  HIPCHECK(hipGetLastError());
  hipLaunchKernelGGL(max_kernel, dim3(1), dim3(kTB), 0, s, part, X, red);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipMemcpyAsync(&h1, red, 8, hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  const double c = h1;
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
    HIPCHECK(hipMemcpyAsync(&h1, red, 8, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
    const double r = std::sqrt(h1);
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

  // per slice of spinor rows p: (pq|Q) = sum_mu nu conj(C_mu p) (mu nu|Q) C_nu q, then
  // B[P][p][q] = sum_Q [V^-1/2]_PQ (pq|Q)
  const int64_t nn = (int64_t)n * n;
  for (int p0 = 0; p0 < n; p0 += ps) {
    const int pn = std::min(ps, n - p0);
    contract(s, "mp,Qmn->Qpn", ONE, conj(sview(const_cast<double*>(Cd) + 2 * p0, {m, pn}, {n, 1})),
             view(const_cast<double*>(Jd), {X, m, m}), false, view(T1, {X, pn, m}));
    contract(s, "Qpn,nq->Qpq", ONE, view(T1, {X, pn, m}), view(const_cast<double*>(Cd), {m, n}), false,
             view(M, {X, pn, n}));
    contract(s, "PQ,Qx->Px", cplx{1.0 / std::sqrt(c), 0.0}, XXv(Z), view(M, {X, (int64_t)pn * n}), false,
             sview(Bd + 2 * (int64_t)p0 * n, {X, (int64_t)pn * n}, {nn, 1}));
  }
  HIPCHECK(hipStreamSynchronize(s));
  return iters;
}

// Device memory of one allocating call, freed on every exit path.
struct Owned {
  void* p[5] = {};
  ~Owned() {
    for (void* q : p)
      if (q) (void)hipFree(q);
  }
  char* alloc(int k, size_t bytes) {
    if (hipMalloc(&p[k], std::max<size_t>(bytes, 16)) != hipSuccess) {
      (void)hipGetLastError();
      p[k] = nullptr;
      raise(-2, "DF factors: device allocation of " + std::to_string(bytes) + " bytes failed");
    }
    return static_cast<char*>(p[k]);
  }
};

// Temporaries of exacc_df_factors_noalloc: one array per GPU, held from library
// load to process end.  Host code never passes the symbol itself to a kernel; it
// uses the device address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[EXACC_DF_SCRATCH_BYTES];
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

char* scratch_address() {
  int dev = 0;
  HIPCHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) raise(-1, "DF factors (no allocation): device ordinal beyond 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = p;
  }
  return static_cast<char*>(g_scratch_ptr[dev]);
}

}  // namespace

int df_factors_impl(int m, int n, int X, const double* C, const double* J, const double* V, double* B,
                    bool on_device, hipStream_t s) {
  Owned own;
  const size_t bC = (size_t)m * n * 16, bJ = (size_t)X * m * m * 16, bV = (size_t)X * X * 8,
               bB = (size_t)X * n * n * 16;
  const double *Cd = C, *Jd = J, *Vd = V;
  double* Bd = B;
  if (!on_device) {
    char* c = own.alloc(0, bC);
    char* j = own.alloc(1, bJ);
    char* v = own.alloc(2, bV);
    HIPCHECK(hipMemcpyAsync(c, C, bC, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(j, J, bJ, hipMemcpyHostToDevice, s));
    HIPCHECK(hipMemcpyAsync(v, V, bV, hipMemcpyHostToDevice, s));
    Cd = reinterpret_cast<double*>(c);
    Jd = reinterpret_cast<double*>(j);
    Vd = reinterpret_cast<double*>(v);
    Bd = reinterpret_cast<double*>(own.alloc(3, bB));
  }
  // every temporary in one region: the whole spinor range in one slice and a 64 MiB
  // split-K workspace
  const size_t wsb = (size_t)64 << 20;
  const size_t cap = fixed_bytes(X) + slice_bytes(m, n, X, n) + wsb;
  char* region = own.alloc(4, cap);
  const int iters = df_core(m, n, X, Cd, Jd, Vd, Bd, s, region, cap, wsb);
  if (!on_device) {
    HIPCHECK(hipMemcpyAsync(B, Bd, bB, hipMemcpyDeviceToHost, s));
    HIPCHECK(hipStreamSynchronize(s));
  }
  return iters;
}

int df_factors_noalloc_impl(int m, int n, int X, const double* C, const double* J, const double* V,
                            double* B, hipStream_t s) {
  const size_t need = fixed_bytes(X) + slice_bytes(m, n, X, 1);
  if (need > (size_t)EXACC_DF_SCRATCH_BYTES)
    raise(-2, "DF factors (no allocation): naux = " + std::to_string(X) + ", nao = " + std::to_string(m) +
                  ", nspinor = " + std::to_string(n) + " need " + std::to_string(need) +
                  " bytes of scratch, above the static " + std::to_string((size_t)EXACC_DF_SCRATCH_BYTES));
  char* base = scratch_address();
  return df_core(m, n, X, C, J, V, B, s, base, (size_t)EXACC_DF_SCRATCH_BYTES, (size_t)64 << 20);
}

}  // namespace exacc
