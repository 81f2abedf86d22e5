// Host planner for contract(): groups the einsum labels into batch / m / n / k,
// and finds for each group an order and a split point so that every operand
// carrying the group addresses it as (outer, inner) with one stride per level.
#include "einsum.h"

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

namespace exacc {

namespace {

struct Lab {
  char c;
  int64_t dim;
  int64_t str[3];  // stride in A, B, C (0 if absent)
  bool in[3];
};

struct Comp {
  int64_t size = 1, in = 1;
  int64_t so[3] = {0, 0, 0}, si[3] = {0, 0, 0};
  int score = -1;
};

// Merge an ordered run of labels for operand t; true if one stride suffices.
bool merge(const std::vector<const Lab*>& run, int t, int64_t& stride, int64_t& size) {
  size = 1;
  stride = 0;
  if (run.empty()) return true;
  for (size_t i = 0; i + 1 < run.size(); ++i)
    if (run[i]->str[t] != run[i + 1]->str[t] * run[i + 1]->dim) return false;
  stride = run.back()->str[t];
  for (auto* l : run) size *= l->dim;
  return true;
}

Comp best_comp(std::vector<const Lab*> g, const int* ops, int nops, int fast_pref) {
  Comp best;
  if (g.empty()) {
    best.score = 0;
    return best;
  }
  std::sort(g.begin(), g.end(), [](const Lab* a, const Lab* b) { return a->c < b->c; });
  do {
    for (size_t sp = 0; sp <= g.size(); ++sp) {
      std::vector<const Lab*> outer(g.begin(), g.begin() + sp), inner(g.begin() + sp, g.end());
      Comp c;
      bool ok = true;
      int64_t osz = 1, isz = 1;
      for (int q = 0; q < nops && ok; ++q) {
        const int t = ops[q];
        int64_t so, si;
        ok = merge(outer, t, so, osz) && merge(inner, t, si, isz);
        c.so[t] = so;
        c.si[t] = si;
      }
      if (!ok) continue;
      c.size = osz * isz;
      c.in = isz;
      if (inner.empty()) {  // single level carried by the outer run
        c.in = c.size;
        for (int q = 0; q < nops; ++q) c.si[ops[q]] = c.so[ops[q]];
      }
      int score = 0;
      for (int q = 0; q < nops; ++q)
        if (c.si[ops[q]] == 1) score += (ops[q] == fast_pref) ? 4 : 2;
      if (c.in == c.size) score += 1;  // no division needed
      if (score > best.score) {
        best = c;
        best.score = score;
      }
    }
  } while (std::next_permutation(g.begin(), g.end(),
                                 [](const Lab* a, const Lab* b) { return a->c < b->c; }));
  return best;
}

thread_local const AllocRange* g_reg = nullptr;
thread_local int g_nreg = 0;

// Highest and lowest element offsets a view can address must fall inside one allocation.
template <typename R>
void check_extent(const TV<R>& t, const char* what, const std::string& sp) {
  if (!g_reg) return;
  int64_t lo = 0, hi = 0;
  for (int i = 0; i < t.nd; ++i) {
    if (t.dim[i] == 0) return;
    const int64_t span = (t.dim[i] - 1) * t.str[i];
    if (span >= 0) hi += span; else lo += span;
  }
  const char* p = reinterpret_cast<const char*>(t.p);
  const char* first = p + 2 * lo * (int64_t)sizeof(R);
  const char* last = p + 2 * (hi + 1) * (int64_t)sizeof(R);
  for (int k = 0; k < g_nreg; ++k) {
    const char* b = reinterpret_cast<const char*>(g_reg[k].base);
    if (first >= b && last <= b + g_reg[k].bytes) return;
  }
  raise(-3, std::string("contract: operand ") + what + " outside its allocation in " + sp);
}

}  // namespace

void set_alloc_registry(const AllocRange* r, int n) {
  g_reg = r;
  g_nreg = n;
}

template <typename R>
static void contract_impl(hipStream_t s, const std::string& la, const std::string& lb,
                          const std::string& lc, cplx alpha, const TV<R>& A, const TV<R>& B,
                          bool accumulate, const TV<R>& C, int kind) {
  const std::string sp = la + "," + lb + "->" + lc;
  const TV<R>* T[3] = {&A, &B, &C};
  const std::string* L[3] = {&la, &lb, &lc};
  std::vector<Lab> labs;
  labs.reserve(16);
  for (int t = 0; t < 3; ++t) {
    if ((int)L[t]->size() != T[t]->nd) raise(-1, "contract: rank mismatch in " + sp);
    for (int i = 0; i < T[t]->nd; ++i) {
      const char ch = (*L[t])[i];
      auto it = std::find_if(labs.begin(), labs.end(), [&](const Lab& l) { return l.c == ch; });
      if (it == labs.end()) {
        Lab l{};
        l.c = ch;
        l.dim = T[t]->dim[i];
        labs.push_back(l);
        it = labs.end() - 1;
      }
      if (it->in[t]) raise(-1, "contract: repeated label in " + sp);
      if (it->dim != T[t]->dim[i]) raise(-1, "contract: dimension mismatch in " + sp);
      it->in[t] = true;
      it->str[t] = T[t]->str[i];
    }
  }
  std::vector<const Lab*> gb, gm, gn, gk;
  for (auto& l : labs) {
    if (l.in[0] && l.in[1] && l.in[2]) gb.push_back(&l);
    else if (l.in[0] && l.in[2]) gm.push_back(&l);
    else if (l.in[1] && l.in[2]) gn.push_back(&l);
    else if (l.in[0] && l.in[1]) gk.push_back(&l);
    else raise(-1, "contract: label in one operand only in " + sp);
  }
  for (auto& l : labs)  // empty output: nothing to do (an empty sum still writes zeros)
    if (l.dim == 0 && l.in[2]) return;

  const int opsM[2] = {0, 2}, opsN[2] = {1, 2}, opsK[2] = {0, 1}, opsB[3] = {0, 1, 2};
  const Comp cm = best_comp(gm, opsM, 2, 0);
  const Comp cn = best_comp(gn, opsN, 2, 1);
  const Comp ck = best_comp(gk, opsK, 2, 0);
  const Comp cb = best_comp(gb, opsB, 3, 2);
  const std::vector<const Lab*>* bad = nullptr;
  if (cm.score < 0) bad = &gm;
  else if (cn.score < 0) bad = &gn;
  else if (cb.score < 0) bad = &gb;
  else if (ck.score < 0) bad = &gk;
  if (bad) {
    // Peel one label of the group into a host loop (a summed label accumulates).
    const Lab* pl = (*bad)[0];
    for (auto* l : *bad)
      if (l->dim < pl->dim) pl = l;
    const char pc = pl->c;
    const int64_t pdim = pl->dim;
    auto drop = [&](const std::string& ls, const TV<R>& t, int64_t val, TV<R>& out, std::string& lo) {
      out = TV<R>();
      out.p = t.p;
      out.conj = t.conj;
      lo.clear();
      for (int i = 0; i < t.nd; ++i) {
        if (ls[i] == pc) {
          out.p = t.p + 2 * val * t.str[i];
        } else {
          out.dim[out.nd] = t.dim[i];
          out.str[out.nd] = t.str[i];
          out.nd++;
          lo.push_back(ls[i]);
        }
      }
    };
    const bool summed = !pl->in[2];
    for (int64_t q = 0; q < pdim; ++q) {
      TV<R> a2, b2, c2;
      std::string la2, lb2, lc2;
      drop(la, A, q, a2, la2);
      drop(lb, B, q, b2, lb2);
      drop(lc, C, q, c2, lc2);
      contract_impl(s, la2, lb2, lc2, alpha, a2, b2, accumulate || (summed && q > 0), c2, kind);
    }
    return;
  }
  if (cm.size > 0x7fffffff || cn.size > 0x7fffffff || ck.size > 0x7fffffff)
    raise(-1, "contract: extent beyond 2^31 in " + sp);

  Gett<R> g{};
  g.M = (int)cm.size;
  g.N = (int)cn.size;
  g.K = (int)ck.size;
  g.m_in = (int)cm.in;
  g.n_in = (int)cn.in;
  g.k_in = (int)ck.in;
  g.a_mo = cm.so[0];
  g.a_mi = cm.si[0];
  g.c_mo = cm.so[2];
  g.c_mi = cm.si[2];
  g.b_no = cn.so[1];
  g.b_ni = cn.si[1];
  g.c_no = cn.so[2];
  g.c_ni = cn.si[2];
  g.a_ko = ck.so[0];
  g.a_ki = ck.si[0];
  g.b_ko = ck.so[1];
  g.b_ki = ck.si[1];
  g.conj_a = A.conj;
  g.conj_b = B.conj;
  g.accumulate = accumulate ? 1 : 0;
  g.alpha_re = (R)alpha.re;
  g.alpha_im = (R)alpha.im;
  // batch: inner level is the launch batch, outer level (if any) a host loop
  const int64_t nouter = cb.size / cb.in;
  g.nbatch = (int)cb.in;
  g.a_b = cb.si[0];
  g.b_b = cb.si[1];
  g.c_b = cb.si[2];
  for (int64_t q = 0; q < nouter; ++q) {
    Gett<R> h = g;
    h.A = A.p + 2 * q * cb.so[0];
    h.B = B.p + 2 * q * cb.so[1];
    h.C = C.p + 2 * q * cb.so[2];
    launch_gett(h, kind, s);
  }
}

template <typename R>
void contract(hipStream_t s, const char* spec, cplx alpha, const TV<R>& A, const TV<R>& B,
              bool accumulate, const TV<R>& C, int kind) {
  std::string sp(spec);
  const size_t comma = sp.find(','), arrow = sp.find("->");
  if (comma == std::string::npos || arrow == std::string::npos || arrow < comma)
    raise(-1, "contract: bad spec " + sp);
  check_extent(A, "A", sp);
  check_extent(B, "B", sp);
  check_extent(C, "C", sp);
  contract_impl(s, sp.substr(0, comma), sp.substr(comma + 1, arrow - comma - 1),
                sp.substr(arrow + 2), alpha, A, B, accumulate, C, kind);
}

template void contract<double>(hipStream_t, const char*, cplx, const TV<double>&, const TV<double>&,
                               bool, const TV<double>&, int);
template void contract<float>(hipStream_t, const char*, cplx, const TV<float>&, const TV<float>&,
                              bool, const TV<float>&, int);

}  // namespace exacc
