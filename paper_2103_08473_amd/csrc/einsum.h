// Host planner: maps a two-operand einsum specification onto one GETT launch
// (or a short host loop of them) without moving data.
#pragma once
#include <cstdint>
#include <initializer_list>

#include "common.h"

namespace exacc {

// A strided view of a complex tensor; dims and strides in complex elements.
template <typename R>
struct TV {
  R* p = nullptr;
  int nd = 0;
  int64_t dim[8] = {};
  int64_t str[8] = {};
  bool conj = false;
};

// Row-major contiguous view of p with the given dims.
template <typename R>
TV<R> view(R* p, std::initializer_list<int64_t> dims) {
  TV<R> t;
  t.p = p;
  t.nd = (int)dims.size();
  int k = 0;
  for (int64_t d : dims) t.dim[k++] = d;
  int64_t s = 1;
  for (int i = t.nd - 1; i >= 0; --i) {
    t.str[i] = s;
    s *= t.dim[i];
  }
  return t;
}

// Explicitly strided view.
template <typename R>
TV<R> sview(R* p, std::initializer_list<int64_t> dims, std::initializer_list<int64_t> strides) {
  TV<R> t;
  t.p = p;
  t.nd = (int)dims.size();
  int k = 0;
  for (int64_t d : dims) t.dim[k++] = d;
  k = 0;
  for (int64_t s : strides) t.str[k++] = s;
  return t;
}

template <typename R>
TV<R> conj(TV<R> t) {
  t.conj = !t.conj;
  return t;
}

// Device allocations the calling thread may address: every operand of
// contract() must lie inside one of them (checked on the host before launch).
struct AllocRange {
  const void* base;
  size_t bytes;
};
void set_alloc_registry(const AllocRange* r, int n);

// C = alpha * einsum(spec, A, B) (+ C if accumulate).  spec is "ab,bc->ac":
// every label of C must occur in A or B; labels in A and B but not C are
// summed; labels in all three are a batch.  Throws on unsupported layouts.
template <typename R>
void contract(hipStream_t s, const char* spec, cplx alpha, const TV<R>& A, const TV<R>& B,
              bool accumulate, const TV<R>& C, int kind = GETT_GENERIC);

}  // namespace exacc
