// CPU check of the contraction planner (einsum.cpp): launch_gett is replaced by
// a CPU loop with the same semantics, every spec the iteration issues is run
// on small ragged shapes, and the result is compared with a direct loop over
// all label values.  Also checks that every GETT offset stays inside its view.
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <string>
#include <vector>

#include "einsum.h"

namespace exacc {
void raise(int status, const std::string& msg) { throw Error{status, msg}; }
void hip_check(hipError_t, const char*, const char*, int) {}

struct Span {
  const double* lo;
  const double* hi;
};
static std::vector<Span> g_spans;
static int g_bad = 0;
static long g_launches = 0;

static void chk(const double* p) {
  for (auto& s : g_spans)
    if (p >= s.lo && p + 1 < s.hi) return;
  g_bad++;
}

static int64_t cm(int x, int in, int64_t so, int64_t si) { return (int64_t)(x / in) * so + (int64_t)(x % in) * si; }

template <typename R>
void launch_gett(const Gett<R>& g, int, hipStream_t) {
  g_launches++;
  for (int b = 0; b < g.nbatch; ++b)
    for (int m = 0; m < g.M; ++m)
      for (int n = 0; n < g.N; ++n) {
        std::complex<double> acc = 0;
        for (int k = 0; k < g.K; ++k) {
          const R* a = g.A + 2 * (b * g.a_b + cm(m, g.m_in, g.a_mo, g.a_mi) + cm(k, g.k_in, g.a_ko, g.a_ki));
          const R* bb = g.B + 2 * (b * g.b_b + cm(k, g.k_in, g.b_ko, g.b_ki) + cm(n, g.n_in, g.b_no, g.b_ni));
          chk((const double*)a);
          chk((const double*)bb);
          std::complex<double> x(a[0], g.conj_a ? -a[1] : a[1]), y(bb[0], g.conj_b ? -bb[1] : bb[1]);
          acc += x * y;
        }
        R* c = g.C + 2 * (b * g.c_b + cm(m, g.m_in, g.c_mo, g.c_mi) + cm(n, g.n_in, g.c_no, g.c_ni));
        chk((const double*)c);
        std::complex<double> r = std::complex<double>(g.alpha_re, g.alpha_im) * acc;
        if (g.accumulate) r += std::complex<double>(c[0], c[1]);
        c[0] = r.real();
        c[1] = r.imag();
      }
}
template void launch_gett<double>(const Gett<double>&, int, hipStream_t);
template void launch_gett<float>(const Gett<float>&, int, hipStream_t);
}  // namespace exacc

using namespace exacc;
typedef std::complex<double> zc;
typedef std::complex<double> cplx_t;

struct Buf {
  std::vector<double> d;
  explicit Buf(int64_t n) : d(2 * n) {}
  double* p() { return d.data(); }
};

static std::mt19937_64 rng(12345);
static void fill(Buf& b) {
  std::normal_distribution<double> nd;
  for (auto& x : b.d) x = nd(rng);
}

// direct evaluation of C = alpha * sum A B (+ C)
static void naive(const std::string& spec, zc alpha, const TV<double>& A, const TV<double>& B, bool acc,
                  const TV<double>& C) {
  double* out = C.p;
  const size_t comma = spec.find(','), arrow = spec.find("->");
  const std::string la = spec.substr(0, comma), lb = spec.substr(comma + 1, arrow - comma - 1),
                    lc = spec.substr(arrow + 2);
  std::string labels;
  std::map<char, int64_t> dim;
  auto reg = [&](const std::string& l, const TV<double>& t) {
    for (int i = 0; i < t.nd; ++i) {
      if (labels.find(l[i]) == std::string::npos) labels.push_back(l[i]);
      dim[l[i]] = t.dim[i];
    }
  };
  reg(la, A);
  reg(lb, B);
  reg(lc, C);
  auto off = [&](const std::string& l, const TV<double>& t, const std::map<char, int64_t>& v) {
    int64_t o = 0;
    for (int i = 0; i < t.nd; ++i) o += v.at(l[i]) * t.str[i];
    return o;
  };
  // zero or keep C over its own index space
  std::map<char, int64_t> val;
  for (char c : labels) val[c] = 0;
  std::vector<zc> accum;
  // enumerate C index space
  int64_t ctot = 1;
  for (int i = 0; i < C.nd; ++i) ctot *= C.dim[i];
  for (int64_t q = 0; q < ctot; ++q) {
    int64_t r = q;
    for (int i = C.nd - 1; i >= 0; --i) {
      val[lc[i]] = r % C.dim[i];
      r /= C.dim[i];
    }
    const int64_t o = off(lc, C, val);
    if (!acc) {
      out[2 * o] = 0;
      out[2 * o + 1] = 0;
    }
  }
  int64_t tot = 1;
  for (char c : labels) tot *= dim[c];
  for (int64_t q = 0; q < tot; ++q) {
    int64_t r = q;
    for (int i = (int)labels.size() - 1; i >= 0; --i) {
      val[labels[i]] = r % dim[labels[i]];
      r /= dim[labels[i]];
    }
    const double* a = A.p + 2 * off(la, A, val);
    const double* b = B.p + 2 * off(lb, B, val);
    zc x(a[0], A.conj ? -a[1] : a[1]), y(b[0], B.conj ? -b[1] : b[1]);
    const int64_t o = off(lc, C, val);
    zc z = alpha * x * y;
    out[2 * o] += z.real();
    out[2 * o + 1] += z.imag();
  }
}

int main() {
  int fails = 0, cases = 0;
  const int o = 3, v = 5, X = 4, n = o + v;
  const int64_t nX = (int64_t)n * X, Po = o * (o - 1) / 2, Pv = v * (v - 1) / 2;
  Buf Bt(n * nX);
  fill(Bt);
  TV<double> Boo = sview(Bt.p(), {o, o, X}, {nX, X, 1});
  TV<double> Bov = sview(Bt.p() + 2 * (int64_t)o * X, {o, v, X}, {nX, X, 1});
  TV<double> Bvo = sview(Bt.p() + 2 * (int64_t)o * nX, {v, o, X}, {nX, X, 1});
  TV<double> Bvv = sview(Bt.p() + 2 * ((int64_t)o * nX + (int64_t)o * X), {v, v, X}, {nX, X, 1});
  std::vector<Buf*> pool;
  auto mk = [&](std::initializer_list<int64_t> dims) {
    int64_t t = 1;
    for (auto d : dims) t *= d;
    Buf* b = new Buf(t);
    fill(*b);
    pool.push_back(b);
    return view(b->p(), dims);
  };
  auto run = [&](const char* spec, zc alpha, TV<double> A, TV<double> B, bool acc, TV<double> C) {
    cases++;
    g_spans.clear();
    auto add = [&](const double* base, int64_t ncplx) { g_spans.push_back({base, base + 2 * ncplx}); };
    add(Bt.p(), n * nX);
    for (auto* b : pool) add(b->p(), (int64_t)b->d.size() / 2);
    // reference on a copy of C's whole buffer
    Buf* owner = nullptr;
    for (auto* b : pool)
      if (C.p >= b->p() && C.p < b->p() + b->d.size()) owner = b;
    std::vector<double> before = owner->d;
    std::vector<double> ref = owner->d;
    const int64_t shift = C.p - owner->p();
    TV<double> Cr = C;
    Cr.p = ref.data() + shift;
    naive(spec, alpha, A, B, acc, Cr);
    const int bad0 = g_bad;
    try {
      contract(nullptr, spec, cplx{alpha.real(), alpha.imag()}, A, B, acc, C);
    } catch (const Error& e) {
      printf("FAIL %s: planner raised: %s\n", spec, e.msg.c_str());
      fails++;
      return;
    }
    double err = 0, mx = 0;
    for (size_t i = 0; i < ref.size(); ++i) {
      err = std::max(err, std::fabs(ref[i] - owner->d[i]));
      mx = std::max(mx, std::fabs(ref[i]));
    }
    const bool ok = err <= 1e-12 * std::max(1.0, mx) && g_bad == bad0;
    if (!ok) {
      printf("FAIL %s: max err %.3e (scale %.3e), out-of-view accesses %d\n", spec, err, mx, g_bad - bad0);
      fails++;
    }
    (void)before;
  };
  const zc ONE(1, 0), MONE(-1, 0), HALF(0.5, 0), CPX(0.3, -0.7);
  // integral classes
  run("kiP,ljP->klij", ONE, Boo, Boo, false, mk({o, o, o, o}));
  run("kjP,liP->klij", MONE, Boo, Boo, true, mk({o, o, o, o}));
  run("kiP,lcP->klic", ONE, Boo, Bov, false, mk({o, o, o, v}));
  run("kcP,liP->klic", MONE, Bov, Boo, true, mk({o, o, o, v}));
  run("kcP,ldP->klcd", ONE, Bov, Bov, false, mk({o, o, v, v}));
  run("kdP,lcP->klcd", MONE, Bov, Bov, true, mk({o, o, v, v}));
  run("acP,kiP->aikc", ONE, Bvv, Boo, false, mk({v, o, o, v}));
  run("aiP,kcP->aikc", MONE, Bvo, Bov, true, mk({v, o, o, v}));
  {
    const int nb = 2, b0 = 2;
    auto Bc = sview(Bvv.p + 2 * (int64_t)b0 * nX, {nb, v, X}, {nX, X, 1});
    auto tmp = mk({nb, o, v, v});
    run("bcP,kdP->bkcd", ONE, Bc, Bov, false, tmp);
    run("bdP,kcP->bkcd", MONE, Bc, Bov, true, tmp);
  }
  // iteration
  auto t1 = mk({o, v});
  auto T2 = mk({o, o, v, v}), TAU = mk({o, o, v, v});
  auto taup = mk({Po, Pv});
  auto Voovv = mk({o, o, v, v}), Vooov = mk({o, o, o, v}), Vvovo = mk({v, o, o, v});
  auto Hac = mk({v, v}), Gac = mk({v, v}), Hki = mk({o, o}), Gki = mk({o, o}), Hkc = mk({o, v});
  run("klcd,klda->ac", HALF, Voovv, TAU, false, Hac);
  run("klcd,licd->ki", HALF, Voovv, TAU, false, Hki);
  run("klcd,ld->kc", ONE, Voovv, t1, false, Hkc);
  auto y = mk({X});
  run("kdP,kd->P", ONE, Bov, t1, false, y);
  run("acP,P->ac", ONE, Bvv, y, true, Gac);
  auto Zt = mk({v, v, X});
  run("kd,kcP->dcP", ONE, t1, Bov, false, Zt);
  run("adP,dcP->ac", MONE, Bvv, Zt, true, Gac);
  run("klic,lc->ki", MONE, Vooov, t1, true, Gki);
  auto H4 = mk({v, o, o, v}), U = mk({o, o, X}), Vt = mk({v, o, X});
  run("kdP,id->kiP", ONE, Bov, t1, false, U);
  run("acP,ic->aiP", ONE, Bvv, t1, false, Vt);
  run("acP,kiP->aikc", ONE, Bvv, U, true, H4);
  run("aiP,kcP->aikc", MONE, Vt, Bov, true, H4);
  run("klic,la->aikc", MONE, Vooov, t1, true, H4);
  run("aild,klcd->aikc", ONE, mk({v, o, o, v}), Voovv, true, H4);
  auto R = mk({o, o, v, v});
  run("aikc,bjkc->ijab", ONE, H4, mk({v, o, o, v}), false, R);
  run("aiP,bjP->ijab", ONE, Vt, Bvo, true, R);
  auto Zij = mk({o, o, v, v}), Zab = mk({o, o, v, v});
  run("kj,ikab->ijab", ONE, Gki, T2, false, Zij);
  run("ac,ijcb->ijab", ONE, Gac, T2, false, Zab);
  auto Cp = mk({Po, v, o}), Cf = mk({o, o, v, o});
  run("bkx,px->pbk", MONE, mk({v, o, Pv}), taup, false, Cp);
  run("bikc,jc->ijbk", ONE, Vvovo, t1, true, Cf);
  run("bjkc,ic->ijbk", MONE, Vvovo, t1, true, Cf);
  run("ijak,kb->ijab", ONE, Cf, t1, true, Zab);
  auto Af = mk({o, o, o, o});
  run("klic,jc->klij", ONE, Vooov, t1, true, Af);
  run("kljc,ic->klij", MONE, Vooov, t1, true, Af);
  run("klcd,ijcd->klij", HALF, Voovv, TAU, true, Af);
  auto Znp = mk({Po, Pv});
  run("qp,qx->px", ONE, mk({Po, Po}), taup, false, Znp);
  {
    const int a = 1, nb = v - a - 1;
    auto Ba = sview(Bvv.p + 2 * (int64_t)a * nX, {v, X}, {X, 1});
    auto Bb = sview(Bvv.p + 2 * (int64_t)(a + 1) * nX, {nb, v, X}, {nX, X, 1});
    run("cP,bdP->cbd", ONE, Ba, Bb, false, mk({v, nb, v}));
    const int64_t rows = 4, start = 3;
    auto W = mk({rows, Pv});
    auto Zc = sview(Znp.p + 2 * start, {Po, rows}, {Pv, 1});
    run("py,xy->px", ONE, taup, W, true, Zc);
  }
  // Hermitian ladder: the chunk's tile build over c, d >= a0, the forward product over the
  // pair tail and the backward product through conj(W) (K strided) or its transpose
  {
    const int a0 = 1, a = 2, nb = v - a - 1, wv = v - a0;
    const int64_t Pw = (int64_t)wv * (wv - 1) / 2, off = (int64_t)a0 * v - (int64_t)a0 * (a0 + 1) / 2;
    const int64_t rows = 5, nt = Pw - rows;
    auto Ba = sview(Bvv.p + 2 * ((int64_t)a * nX + (int64_t)a0 * X), {wv, X}, {X, 1});
    auto Bb = sview(Bvv.p + 2 * ((int64_t)(a + 1) * nX + (int64_t)a0 * X), {nb, wv, X}, {nX, X, 1});
    run("cP,bdP->cbd", ONE, Ba, Bb, false, mk({wv, nb, wv}));
    auto W = mk({rows, Pw});
    run("py,xy->px", ONE, sview(taup.p + 2 * off, {Po, Pw}, {Pv, 1}), W, true,
        sview(Znp.p + 2 * off, {Po, rows}, {Pv, 1}));
    auto Lc = sview(taup.p + 2 * off, {Po, rows}, {Pv, 1});
    auto Zt = sview(Znp.p + 2 * (off + rows), {Po, nt}, {Pv, 1});
    run("px,xy->py", ONE, Lc, conj(sview(W.p + 2 * rows, {rows, nt}, {Pw, 1})), true, Zt);
    run("px,yx->py", ONE, Lc, conj(mk({nt, rows})), true, Zt);
  }
  auto S1 = mk({o, v}), M1 = mk({o, o}), Y = mk({o, v, X});
  run("ac,ic->ia", ONE, Hac, t1, false, S1);
  run("ki,ka->ia", ONE, Hki, t1, true, S1);
  run("kc,ikac->ia", ONE, Hkc, T2, true, S1);
  run("kc,ic->ki", ONE, Hkc, t1, false, M1);
  run("ki,ka->ia", ONE, M1, t1, true, S1);
  run("ikcd,kdP->icP", ONE, TAU, Bov, false, Y);
  run("icP,acP->ia", ONE, Y, Bvv, true, S1);
  run("klic,klca->ia", HALF, Vooov, TAU, true, S1);
  run("aikc,kc->ia", MONE, Vvovo, t1, true, S1);
  // T2 read through the permuted ring operand Tq[b][i][k][a]; Z and its i<->j / a<->b swapped views
  {
    const int64_t ov = (int64_t)o * v, oov = (int64_t)o * o * v, vv = (int64_t)v * v, ovv = ov * v;
    auto Tq = mk({v, o, o, v});
    auto T2v = sview(Tq.p, {o, o, v, v}, {ov, v, 1, oov});
    auto Zf = mk({o, o, v, v});
    auto Zji = sview(Zf.p, {o, o, v, v}, {vv, ovv, v, 1});
    auto Zba = sview(Zf.p, {o, o, v, v}, {ovv, vv, 1, v});
    run("kj,ikab->ijab", ONE, Gki, T2v, false, Zf);
    run("kj,ikab->ijab", MONE, Gki, T2v, true, Zji);
    run("ac,ijcb->ijab", ONE, Gac, T2v, true, Zf);
    run("ac,ijcb->ijab", MONE, Gac, T2v, true, Zba);
    run("ijak,kb->ijab", MONE, Cf, t1, true, Zba);
    run("kc,ikac->ia", ONE, Hkc, T2v, true, S1);
  }
  // <kl||cd> stored [k][c][l][d] (FP32 copy layout)
  {
    auto Vperm = sview(mk({o, v, o, v}).p, {o, o, v, v}, {(int64_t)o * v * v, (int64_t)v, (int64_t)o * v, 1});
    run("kcP,ldP->klcd", ONE, Bov, Bov, false, Vperm);
    run("klcd,klda->ac", HALF, Vperm, TAU, false, Hac);
    run("klcd,licd->ki", HALF, Vperm, TAU, false, Hki);
    run("klcd,ld->kc", ONE, Vperm, t1, false, Hkc);
    run("aild,klcd->aikc", ONE, mk({v, o, o, v}), Vperm, true, H4);
    run("klcd,ijcd->klij", HALF, Vperm, TAU, true, Af);
  }
  // Lambda equations: preparation and residual (views as the library issues them)
  {
    const int64_t ov = (int64_t)o * v, oov = (int64_t)o * o * v, vv = (int64_t)v * v, ovv = ov * v;
    const cplx_t NHALF(-0.5, 0), NQ(-0.25, 0);
    auto U = mk({o, o, X}), Vt = mk({v, o, X});
    auto Tq = mk({v, o, o, v});
    auto T2v = sview(Tq.p, {o, o, v, v}, {ov, v, 1, oov});
    auto Wqb = mk({v, o, o, v});
    auto WqH = sview(Wqb.p, {v, o, o, v}, {1, v, ov, oov});
    run("acP,kiP->aikc", MONE, Bvv, Boo, false, WqH);
    run("aiP,kcP->aikc", ONE, Bvo, Bov, true, WqH);
    run("acP,kiP->aikc", MONE, Bvv, U, true, WqH);
    run("aiP,kcP->aikc", ONE, Vt, Bov, true, WqH);
    run("klic,la->aikc", ONE, Vooov, t1, true, WqH);
    run("aild,klcd->aikc", MONE, mk({v, o, o, v}), Voovv, true, WqH);
    run("aild,klcd->aikc", NHALF, Tq, Voovv, true, WqH);
    auto Wooov = mk({o, o, o, v});
    run("if,mnfe->mnie", ONE, t1, Voovv, true, Wooov);
    auto Cfb = mk({o, o, v, o});
    const int64_t vo = (int64_t)v * o;
    auto Cfji = sview(Cfb.p, {o, o, v, o}, {vo, o * vo, o, 1});
    auto Afb = mk({o, o, o, o});
    run("me,ijbe->ijbm", MONE, Hkc, T2v, true, Cfb);
    run("nb,mnij->ijbm", MONE, t1, Afb, true, Cfb);
    run("mnie,jnbe->ijbm", ONE, Vooov, T2v, true, Cfb);
    run("mnie,jnbe->ijbm", MONE, Vooov, T2v, true, Cfji);
    run("miP,bjP->ijbm", ONE, U, Bvo, true, Cfb);
    run("mjP,biP->ijbm", MONE, Boo, Vt, true, Cfji);
    auto Wt = mk({o, o, o, v});
    run("ie,mnef->mnif", ONE, t1, Voovv, false, Wt);
    run("mnif,njbf->ijbm", MONE, Wt, T2v, true, Cfb);
    auto Bd = mk({v, v, X});
    run("amP,me->aeP", MONE, conj(Bvo), t1, true, Bd);
    // residual
    auto Lq = mk({v, o, o, v});
    auto L2v = sview(Lq.p, {o, o, v, v}, {ov, v, 1, oov});
    auto l1 = mk({o, v});
    auto Gv = mk({v, v}), Go = mk({o, o});
    run("mnef,mnaf->ae", NHALF, T2v, L2v, false, Gv);
    run("mnef,inef->mi", HALF, T2v, L2v, false, Go);
    auto Zf = mk({o, o, v, v});
    auto Zji = sview(Zf.p, {o, o, v, v}, {vv, ovv, v, 1});
    auto Zba = sview(Zf.p, {o, o, v, v}, {ovv, vv, 1, v});
    run("ijae,eb->ijab", ONE, L2v, Gac, true, Zf);
    run("ijae,eb->ijab", MONE, L2v, Gac, true, Zba);
    run("imab,jm->ijab", MONE, L2v, Gki, true, Zji);
    auto M1 = mk({o, o});
    run("ie,ne->in", ONE, l1, t1, false, M1);
    run("in,njab->ijab", ONE, M1, Voovv, true, Zji);
    run("ma,ijmb->ijab", MONE, l1, Wooov, true, Zf);
    run("ijae,be->ijab", MONE, Voovv, Gv, true, Zba);
    run("imab,mj->ijab", MONE, Voovv, Go, true, Zf);
    auto Rv = mk({o, o, v, v});
    run("aime,bjme->ijab", MONE, Lq, Wqb, false, Rv);
    auto Yv = mk({o, v, X});
    run("ie,aeP->iaP", ONE, l1, conj(Bvv), false, Yv);
    run("iaP,jbP->ijab", ONE, Yv, Bov, true, Rv);
    run("iaz,jbz->ijab", ONE, sview(l1.p, {o, v, 1}, {v, 1, 1}), sview(Hkc.p, {o, v, 1}, {v, 1, 1}), true, Rv);
    auto l2p = mk({Po, Pv}), t2p = mk({Po, Pv}), LT = mk({Po, Po}), Znp2 = mk({Po, Pv});
    run("py,qy->pq", ONE, l2p, t2p, false, LT);
    run("pq,qx->px", ONE, LT, mk({Po, Pv}), false, Znp2);
    run("pq,qx->px", ONE, mk({Po, Po}), l2p, true, Znp2);
    auto S1l = mk({o, v});
    run("imag,mg->ia", ONE, mk({o, o, v, v}), t1, true, S1l);
    run("me,aime->ia", ONE, l1, Wqb, true, S1l);
    run("imef,fmP->ieP", ONE, L2v, Bvo, false, Yv);
    run("ieP,aeP->ia", ONE, Yv, conj(Bvv), true, S1l);
    run("ni,na->ia", MONE, Go, Hkc, true, S1l);
    auto LTo = mk({o, o, o, o});
    run("imef,noef->imno", ONE, L2v, TAU, false, LTo);
    run("imno,noma->ia", NQ, LTo, Vooov, true, S1l);
    auto Z1 = mk({o, o, v, v});
    run("fime,gnme->infg", ONE, Lq, Tq, false, Z1);
    auto Q1 = mk({o, o, X});
    run("infg,fgP->inP", ONE, Z1, Bvv, false, Q1);
    run("inP,naP->ia", MONE, Q1, Bov, true, S1l);
    run("infg,ngP->ifP", ONE, Z1, Bov, false, Yv);
    run("ifP,faP->ia", ONE, Yv, Bvv, true, S1l);
    auto Lt = mk({o, o, o, v}), M2 = mk({o, o, o, v});
    run("imef,ne->imnf", ONE, L2v, t1, false, Lt);
    run("imnf,fmP->inP", ONE, Lt, Bvo, false, Q1);
    run("imnf,nmP->ifP", ONE, Lt, Boo, false, Yv);
    run("imnf,omfg->inog", ONE, Lt, T2v, false, M2);
    run("inog,noag->ia", ONE, M2, Voovv, true, S1l);
    run("mnae,mnei->ia", NHALF, L2v, Cfb, true, S1l);
    auto gP = mk({X}), gt = mk({o, v});
    run("efP,ef->P", ONE, Bvv, Gv, false, gP);
    run("iaP,P->ia", MONE, Bov, gP, true, S1l);
    run("ef,ifP->ieP", ONE, Gv, Bov, false, Yv);
    run("ef,ne->nf", ONE, Gv, t1, false, gt);
    run("nf,nifa->ia", ONE, gt, Voovv, true, S1l);
    run("mn,mina->ia", MONE, Go, Wooov, true, S1l);
    // density pieces
    run("me,ie->im", ONE, l1, t1, false, M1);
    run("me,imae->ia", ONE, l1, T2v, true, gt);
    run("im,ma->ia", MONE, Go, t1, true, gt);
    run("ma,mb->ab", ONE, t1, l1, false, Gv);
    // ladder tile build on the dressed factor rows (row stride v X)
    {
      const int a = 1, nb = v - a - 1;
      auto Ba = sview(Bd.p + 2 * (int64_t)a * v * X, {v, X}, {X, 1});
      auto Bb = sview(Bd.p + 2 * (int64_t)(a + 1) * v * X, {nb, v, X}, {(int64_t)v * X, X, 1});
      run("cP,bdP->cbd", ONE, Ba, Bb, false, mk({v, nb, v}));
    }
  }
  // small nvir: the ladder tiles of all rows in one product ((a, c) rows at the factor's row
  // stride), and the hole ladder's tau term on packed pairs
  run("acP,bdP->acbd", ONE, Bvv, Bvv, false, mk({v, v, v, v}));
  run("qx,px->qp", ONE, mk({Po, Pv}), mk({Po, Pv}), true, mk({Po, Po}));
  // perturbative triples: packed tiles of an occupied block (per a, rows b > a) and the
  // contractions of a batch into the packed parts We[i][(a<b)][c] and Wm[i][a][(b<c)]
  {
    const int64_t vv = (int64_t)v * v, ov = (int64_t)o * v, oov = (int64_t)o * o * v,
                  ovv = (int64_t)o * vv, pvv = Pv * v, opv = (int64_t)o * Pv;
    const int i0 = 1, ni = 2, j = 2, k = 2;
    auto Ve = mk({3, Pv, v});
    for (int a = 0; a + 1 < v; ++a) {
      const int nb = v - a - 1;
      const int64_t off = (int64_t)a * v - (int64_t)a * (a + 1) / 2;
      auto Cv = sview(Ve.p + 2 * off * v, {ni, nb, v}, {pvv, (int64_t)v, 1});
      auto Bvo_a = sview(Bvo.p + 2 * ((int64_t)a * nX + (int64_t)i0 * X), {ni, X}, {X, 1});
      auto Bvv_b = sview(Bvv.p + 2 * (int64_t)(a + 1) * nX, {nb, v, X}, {nX, X, 1});
      run("beP,iP->ibe", ONE, Bvv_b, Bvo_a, false, Cv);
      auto Bvv_a = sview(Bvv.p + 2 * (int64_t)a * nX, {v, X}, {X, 1});
      auto Bvo_b = sview(Bvo.p + 2 * ((int64_t)(a + 1) * nX + (int64_t)i0 * X), {nb, ni, X}, {nX, X, 1});
      run("eP,biP->ibe", MONE, Bvv_a, Bvo_b, true, Cv);
    }
    auto T2f = mk({o, o, v, v});
    auto T2pv = mk({o, o, Pv});
    auto We = mk({ni, Pv, v});
    auto Wm = mk({ni, v, Pv});
    run("ixe,ce->ixc", MONE, sview(Ve.p, {ni, Pv, v}, {pvv, (int64_t)v, 1}),
        sview(T2f.p + 2 * ((int64_t)j * o + k) * vv, {v, v}, {(int64_t)v, 1}), false, We);
    run("xe,ice->ixc", MONE, sview(Ve.p + 2 * pvv, {Pv, v}, {(int64_t)v, 1}),
        sview(T2f.p + 2 * ((int64_t)k * o + 0) * vv, {ni, v, v}, {vv, (int64_t)v, 1}), true, We);
    run("xe,ice->ixc", MONE, sview(Ve.p, {Pv, v}, {(int64_t)v, 1}),
        sview(T2f.p + 2 * ((int64_t)0 * o + j) * vv, {ni, v, v}, {ovv, (int64_t)v, 1}), true, We);
    run("ima,my->iay", MONE, conj(sview(Vooov.p + 2 * ((int64_t)0 * o + j) * ov, {ni, o, v}, {oov, (int64_t)v, 1})),
        sview(T2pv.p + 2 * (int64_t)k * opv, {o, Pv}, {Pv, 1}), false, Wm);
    run("ma,imy->iay", MONE, conj(sview(Vooov.p + 2 * ((int64_t)1 * o + 2) * ov, {o, v}, {(int64_t)v, 1})),
        sview(T2pv.p, {ni, o, Pv}, {opv, Pv, 1}), true, Wm);
    run("ima,my->iay", MONE, conj(sview(Vooov.p + 2 * ((int64_t)k * o + 0) * ov, {ni, o, v}, {ov, (int64_t)v, 1})),
        sview(T2pv.p + 2 * (int64_t)j * opv, {o, Pv}, {Pv, 1}), true, Wm);
    // the two sums over m fused over K = (t, m): t selects the amplitude row j1 or k1 > j1
    const int j1 = 0, k1 = 2;
    run("iatm,tmy->iay", MONE, mk({ni, v, 2, o}),
        sview(T2pv.p + 2 * (int64_t)j1 * opv, {2, o, Pv}, {(int64_t)(k1 - j1) * opv, Pv, 1}), false, Wm);
    run("iatm,tmy->iay", MONE, mk({ni, v, 2, o}),
        sview(T2pv.p + 2 * (int64_t)1 * opv, {2, o, Pv}, {opv, Pv, 1}), true, Wm);
  }
  // DF factors: transform and metric GEMMs, the Newton-Schulz product
  {
    const int m = 6, ns = 4, Xq = 5;
    auto C = mk({m, ns}), J = mk({Xq, m, m}), T1 = mk({Xq, ns, m}), M = mk({Xq, ns, ns});
    run("mp,Qmn->Qpn", ONE, conj(C), J, false, T1);
    run("Qpn,nq->Qpq", ONE, T1, C, false, M);
    run("PQ,Qx->Px", CPX, mk({Xq, Xq}), view(M.p, {Xq, (int64_t)ns * ns}), false, mk({Xq, (int64_t)ns * ns}));
    run("ab,bc->ac", ONE, mk({Xq, Xq}), mk({Xq, Xq}), false, mk({Xq, Xq}));
  }
  // generic: conjugation, complex alpha, batch labels, empty sum
  run("zmk,zkn->zmn", CPX, conj(mk({3, 4, 5})), mk({3, 5, 6}), false, mk({3, 4, 6}));
  run("mk,kn->nm", CPX, mk({7, 2}), conj(mk({2, 9})), true, mk({9, 7}));
  run("mk,kn->mn", ONE, mk({3, 0}), mk({0, 4}), false, mk({3, 4}));
  printf("%d cases, %d failures, %ld launches\n", cases, fails, g_launches);
  for (auto* b : pool) delete b;
  return fails ? 1 : 0;
}
