// Shared declarations of the exacc HIP library (device kernels + host driver).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

namespace exacc {

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));

struct cplx {
  double re, im;
};

// Error raised inside the library; mapped to a status code at the C ABI.
struct Error {
  int status;
  std::string msg;
};

[[noreturn]] void raise(int status, const std::string& msg);
void hip_check(hipError_t e, const char* what, const char* file, int line);
#define HIPCHECK(x) ::exacc::hip_check((x), #x, __FILE__, __LINE__)

// ---------------------------------------------------------------------------
// GETT: C[b](m, n) = alpha * sum_k opA(A[b](m, k)) * opB(B[b](k, n)) (+ C[b](m, n))
// Each of m, n, k is a composite index split into (outer, inner):
//   offset(x) = (x / x_in) * x_so + (x % x_in) * x_si      (complex elements)
// which covers any contraction whose index groups merge into two strided
// levels per operand (the host planner in einsum.cpp finds the split).
// ---------------------------------------------------------------------------
template <typename R>
struct Gett {
  int M, N, K, nbatch;
  int m_in, n_in, k_in;
  int64_t a_mo, a_mi, a_ko, a_ki, a_b;
  int64_t b_ko, b_ki, b_no, b_ni, b_b;
  int64_t c_mo, c_mi, c_no, c_ni, c_b;
  int conj_a, conj_b, accumulate;
  R alpha_re, alpha_im;
  const R* A;  // interleaved complex
  const R* B;
  R* C;
  int kslice;  // split-K: workgroup z covers k in [z*kslice, min(K, (z+1)*kslice))
  R* ws;       // split-K partial sums [z][batch][m][n] (unscaled)
};

// Scratch the calling thread's GETT launches may use for split-K partials.
void set_gett_workspace(void* p, size_t bytes);

enum GettKind {
  GETT_GENERIC = 0,
  GETT_LADDER_BUILD = 1,
  GETT_LADDER_CONTRACT = 2,
  GETT_RING = 3,
  GETT_LADDER_BUILD_BF16X3 = 4,     // FP32 operands, BF16x3 products (falls back to FP32 MFMA
  GETT_LADDER_CONTRACT_BF16X3 = 5,  // when an operand is not K-contiguous)
  GETT_RING_BF16X3 = 6
};

template <typename R>
void launch_gett(const Gett<R>& g, int kind, hipStream_t s);

// BF16x3 on pre-split operands (layout in gett.hip): K rounded up to the split
// width; split `rows` rows of K complex FP32 values (row r at src +
// (r / group) * group_stride + (r % group) * row_stride complex elements) into
// dst, 4 * bf16x3_split_k(K) bf16 per row; C[m][n] = sum_k A[m][k] B[n][k].
int bf16x3_split_k(int K);
void split_rows_bf16x3(const float* src, int64_t rows, int64_t group, int64_t group_stride,
                       int64_t row_stride, int K, unsigned short* dst, hipStream_t s);
// B row of column n: (n / b_in) * b_outer + n % b_in (b_in <= 0: row n)
void gemm_bf16x3_split(const unsigned short* A, const unsigned short* B, int M, int N, int K, float* C,
                       int64_t ldc, hipStream_t s, int b_in = 0, int64_t b_outer = 0);

// ---------------------------------------------------------------------------
// Bandwidth kernels (elementwise.hip).  Sizes in elements; complex arrays are
// interleaved (re, im).  Packed pair index of (p<q) over m: p*m - p(p+1)/2 + q-p-1.
// ---------------------------------------------------------------------------
void k_transpose_B(const double* B, double* Bt, int64_t X, int64_t nn, hipStream_t s);
void k_check_B(const double* B, int64_t X, int n, double* out3, double* scratch, hipStream_t s);
template <typename T>
void k_pack_last2(T* out, const T* in, const int* rowmap, int64_t rows, int m, int64_t in_row_stride,
                  hipStream_t s);
template <typename T>
void k_unpack_tau(const double* t1, const double* t2p, T* T2, T* TAU, T* taup, int o, int v,
                  hipStream_t s);
// Tq[b][j][k][c] = T2[j][k][c][b], Xp = Tq / 2 + t1[k][b] t1[j][c] (- t1r[k][b] t1r[j][c])
template <typename T>
void k_ring_operands(const T* T2, const double* t1, T* Tq, T* Xp, int o, int v, hipStream_t s,
                     const double* t1r = nullptr);
template <typename T>
void k_expand_c(const T* Vooov, const T* Cp, T* Cf, int o, int v, hipStream_t s);
// W[b'][(c<d)] = Ta[c][b'][d] - Ta[d][b'][c] over c, d < v, rows of W ldw apart
template <typename T>
void k_ladder_antisym(const T* Ta, T* W, int nb, int v, int64_t ldw, hipStream_t s);
// W[(a<b)][(c<d)] = Tf[a][c][b][d] - Tf[a][d][b][c] for all a < b (Tf: v^4, W: P_v x P_v)
template <typename T>
void k_ladder_antisym_all(const T* Tf, T* W, int v, hipStream_t s);
// Wt[y][x] = W[x][col0 + y], x < rows, y < ncols (row strides ldw, ldt)
template <typename T>
void k_transpose_tail(const T* W, int64_t rows, int64_t ldw, int64_t col0, int64_t ncols, T* Wt,
                      int64_t ldt, hipStream_t s);
// S2 pieces of type T are summed in FP64 with the FP64 driver <ab||ij> and the
// diagonal Fock part; writes the Jacobi step (or the full residual into s2_full).
template <typename T>
void k_assemble_t2(const T* Znp, const T* Z, const T* R, const double* Voovv_p, const double* t2p,
                   const double* eps, int o, int v, double shift, double* xt, double* e,
                   double* s2_full, double* partial, int nblk, hipStream_t s);
template <typename T>
void k_assemble_t1(const T* S1, const double* t1, const double* eps, int o, int v, double shift,
                   bool frozen, double* xt, double* e, double* s1_full, double* partial, hipStream_t s);
// CC2: Vt[a][i][P] += B^P_ai - Q[a][i][P] (the T1-dressed vo DF factor; Bt is [p][q][P])
template <typename T>
void k_dress_vo(T* Vt, const T* Bt, const T* Q, int o, int v, int n, int X, hipStream_t s);
// perturbative triples: (e4, e5, ey) of the occupied triples (i0 + y, j, k), y < ni, from
// the packed parts We[y][(a<b)][c], Wm[y][a][(b<c)] of W and the full T2; written to
// out[4 * (((i0 + y) * o + j) * o + k)]
int triples_blocks(int v);
// zero nbytes at p / copy nbytes from src to d (nbytes a multiple of 8, pointers 8-byte aligned)
void k_zero_bytes(void* p, int64_t nbytes, hipStream_t s);
void k_copy_bytes(void* d, const void* src, int64_t nbytes, hipStream_t s);
// Acat[y][a][t][m] = conj(<x_t y_t||m a>), (x_0, y_0) = (k, i0 + y), (x_1, y_1) = (i0 + y, j)
void k_triples_acat(const double* Vooov, int i0, int ni, int j, int k, int o, int v, double* out,
                    hipStream_t s);
void k_triples_energy(const double* We, const double* Wm, const double* Voovv, const double* T2,
                      const double* t1, const double* eps, int i0, int ni, int j, int k, int o, int v,
                      double* partial, int nblk, double* out, hipStream_t s);
// FP64 -> FP32, round to nearest even, nreal reals
// DF factors B[X][n][n] from C [m][n], J [X][m][m] (complex) and the real metric V [X][X]
// (all device pointers when on_device, else host); returns the Newton-Schulz step count
int df_factors_impl(int m, int n, int X, const double* C, const double* J, const double* V, double* B,
                    bool on_device, hipStream_t s);
// The same from device pointers with every temporary in the library's static per-GPU
// scratch array (no device allocation); raises NOMEM when the sizes need more than it holds
int df_factors_noalloc_impl(int m, int n, int X, const double* C, const double* J, const double* V,
                            double* B, hipStream_t s);
// dst[r][k] = conj(src[r * src_stride + k]) (complex elements)
void k_conj_rows(double* dst, const double* src, int64_t rows, int64_t src_stride, int64_t len,
                 hipStream_t s);
// Lambda one-body density [n][n] from Go [o][o], M [o][o], l1 [o][v], Dvo [o][v], Gv [v][v], N [v][v]
void k_lambda_density(const double* Go, const double* M, const double* l1, const double* Dvo,
                      const double* Gv, const double* N, int o, int v, double* gamma, hipStream_t s);
void k_cast(const double* in, float* out, int64_t nreal, hipStream_t s);
// out = FP32(a - b), y += a + FP64(c) (c may be null), nreal reals
void k_diff_cast(const double* a, const double* b, float* out, int64_t nreal, hipStream_t s);
void k_add2(double* y, const double* a, const float* c, int64_t nreal, hipStream_t s);
int assemble_t2_blocks(int64_t npairs);
void k_reduce_sum(const double* partial, int n, int width, double* out, hipStream_t s);
void k_dot_many(const double* const* es, int m, const double* e, int64_t len, double* partial,
                int nblk, hipStream_t s);
int dot_many_blocks(int64_t len);
void k_lincomb(double* x, const double* const* xs, const cplx* c, int m, int64_t len,
               hipStream_t s);
void k_energy(const double* Voovv_p, const double* t2p, const double* t1, int o, int v,
              double* partial, int nblk, hipStream_t s);
int energy_blocks(int64_t npairs);
void k_unpack_full(const double* t1, const double* t2p, double* t1_out, double* t2_out, int o,
                   int v, hipStream_t s);
void k_pack_amplitudes(const double* t1, const double* t2, double* x, int o, int v,
                       hipStream_t s);
// t2_out [o][o][v][v] FP32 = the full antisymmetric t2p - r2p (packed inputs, FP64 difference)
void k_unpack_diff(const double* t2p, const double* r2p, float* t2_out, int o, int v, hipStream_t s);
// out = a - b (FP64), nreal reals
void k_sub(const double* a, const double* b, double* out, int64_t nreal, hipStream_t s);

}  // namespace exacc
