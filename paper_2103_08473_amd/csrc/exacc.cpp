// exacc C ABI: one handle per CCSD solve resident on the device.
//
// Per iteration (Appendix A, eq. CC_general), all on the handle's stream:
//   tau and permuted amplitude copies -> one-body intermediates H/G ->
//   H^{ak}_{ci} (ring intermediate) -> ring contraction -> C^{kb}_{ij} ->
//   A^{kl}_{ij} and hole ladder -> particle ladder from density-fitting tiles ->
//   singles residual -> residual assembly fused with the denominator step ->
//   DIIS Gram row -> (host: small bordered solve) -> extrapolation -> energy.
// The diagonal Fock terms (eps_a + eps_b - eps_i - eps_j) t of the residual are
// added in the assembly kernel rather than through H and G; the sum is the same.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/exacc.h"
#include "common.h"
#include "einsum.h"

namespace exacc {

static thread_local std::string g_last_error;

void raise(int status, const std::string& msg) { throw Error{status, msg}; }

void hip_check(hipError_t e, const char* what, const char* file, int line) {
  if (e == hipSuccess) return;
  char buf[512];
  snprintf(buf, sizeof buf, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();  // a failed allocation leaves the device usable
    raise(EXACC_ERR_NOMEM, buf);
  }
  raise(EXACC_ERR_DEVICE, buf);
}

typedef std::complex<double> zc;

static inline int64_t npair(int64_t m) { return m * (m - 1) / 2; }

// ------------------------------------------------------------------ memory plan
struct Plan {
  int o, v, X, n;
  int64_t Po, Pv, L, vv, oovv;
  int64_t chunk_pairs;  // ladder W rows
  bool ladder_grouped = false;  // all virtual rows of the ladder in one product (small nvir)
  int nslots;
  int64_t vovv_chunk;   // b values per vovv build step (create only)
  // complex-element counts
  struct Item {
    const char* name;
    int64_t elems;
    bool transient;
  };
  std::vector<Item> items;
  size_t bytes_persistent = 0, bytes_peak = 0;
  // the defect-corrected phase also covers the ring (its reference arrays are planned in)
  bool ring_dc = false;
  size_t bytes_peak_no_ring_dc = 0;
};

static Plan make_plan(int o, int v, int X, const exacc_ccsd_opts& op) {
  Plan p;
  p.o = o;
  p.v = v;
  p.X = X;
  p.n = o + v;
  p.Po = npair(o);
  p.Pv = npair(v);
  p.L = (int64_t)o * v + p.Po * p.Pv;
  p.vv = (int64_t)v * v;
  p.oovv = (int64_t)o * o * p.vv;
  p.nslots = std::max(1, op.diis_size);
  const int64_t rowbytes = std::max<int64_t>(1, p.Pv) * 16;
  int64_t cp = op.ladder_chunk_pairs;
  if (cp <= 0) cp = std::max<int64_t>(v, (int64_t)(2ll << 30) / rowbytes);
  cp = std::min<int64_t>(std::max<int64_t>(cp, std::max(1, v - 1)), std::max<int64_t>(1, p.Pv));
  p.chunk_pairs = cp;
  p.ladder_grouped = v >= 2 && v <= op.ladder_group_nvir && cp == p.Pv;
  const int64_t vovv_row = (int64_t)o * v * v;  // per b
  p.vovv_chunk = std::max<int64_t>(1, std::min<int64_t>(v, (int64_t)(2ll << 30) / (16 * vovv_row)));
  const int64_t n = p.n, oo = (int64_t)o * o;
  const bool mixed = op.precision != EXACC_FP64;
  // bytes of each buffer class (16 bytes per complex element, +256 alignment slack)
  auto B16 = [](int64_t e) { return (size_t)std::max<int64_t>(e, 1) * 16 + 256; };
  const size_t common = B16(n * n * X)                          // Bt
                        + B16(oo * oo) + B16(oo * o * v)         // Voooo, Vooov
                        + B16(p.Po * p.Pv)                       // Voovv_p
                        + B16(p.L) + B16(2 * p.nslots * p.L)     // x, DIIS
                        + 5 * B16(p.oovv)                        // TAU, Tq, Xp/R, H4, Z
                        + 2 * B16(p.Po * p.Pv)                   // taup, Znp
                        + B16(2 * p.vv + 3 * oo + 3 * (int64_t)o * v + X + oo * X +
                              2 * (int64_t)v * o * X + p.Po * v * o + oo * v * o + oo * oo +
                              p.Po * p.Po)                       // small intermediates
                        + B16(p.ladder_grouped ? p.vv * p.vv : (int64_t)v * std::max(1, v - 1) * v)  // Ta
                        + B16(p.chunk_pairs * std::max<int64_t>(1, p.Pv))  // W
                        + (256u << 20) + (2u << 20);             // split-K, reductions
  const size_t big64 = B16(p.oovv) + B16((int64_t)v * o * p.Pv);  // Voovv, Vvovv_p (FP64)
  const size_t bvs = op.precision == EXACC_MIXED_BF16X3
                        ? B16(p.vv * bf16x3_split_k(X) / 2)       // split B_vv rows, 8 B per k
                        : 0;
  const size_t big32 = (B16(p.oovv) + B16((int64_t)v * o * p.Pv) + B16(n * n * X) + B16(oo * oo) +
                        B16(oo * o * v) + B16(p.Po * p.Pv)) / 2 + bvs;  // FP32 copies
  const size_t vovv_tmp = B16(p.vovv_chunk * vovv_row) + B16(p.vovv_chunk * o * p.Pv);
  const size_t create_peak = B16(n * n * X) * 2 + B16(p.oovv) + big32 + vovv_tmp;  // staging
  // defect-corrected ladder after the switch: tau_ref and Zref, and the low-precision
  // ladder operand (the split B_vv rows, or the FP32 factors) kept until it ends
  const size_t dc = (mixed && op.ladder_defect_correction)
                        ? 2 * B16(p.Po * p.Pv) +
                              (op.precision == EXACC_MIXED_BF16X3 ? bvs : B16(n * n * X) / 2)
                        : 0;
  // ring part of the defect correction: the reference amplitudes, the FP64 reference ring
  // product, FP32 copies of the reference intermediate H and of the correction dH, the kept
  // FP32 <kl||cd>, the DF t1 intermediates of the amplitude difference; and for the vovv.tau
  // product of C^{kb}_{ij} the kept FP32 vovv class and the FP64 reference product
  const size_t ring_dc = dc ? B16(p.L) + B16(p.oovv) + B16(p.oovv) + B16(p.oovv) / 2 +
                                  B16(oo * X + (int64_t)v * o * X + (int64_t)o * v) +
                                  B16((int64_t)v * o * p.Pv) / 2 + B16(p.Po * v * o) +
                                  (op.precision == EXACC_MIXED_BF16X3 ? B16(n * n * X) / 2 : 0)
                            : 0;
  const size_t phase64 = common + big64 + vovv_tmp + dc;
  const size_t phase32 = common + big32;
  p.bytes_persistent = mixed ? phase32 : common + big64;
  p.bytes_peak = std::max(create_peak, mixed ? std::max(phase32, phase64) : phase64);
  p.bytes_peak_no_ring_dc = p.bytes_peak;
  if (ring_dc) {
    const size_t with = std::max(p.bytes_peak, phase64 + ring_dc);
    if (op.hbm_budget_bytes == 0 || with <= op.hbm_budget_bytes) {
      p.ring_dc = true;
      p.bytes_peak = with;
    }
  }
  return p;
}

// ------------------------------------------------------------------ handle
struct Timer {
  bool on = false;
  std::vector<std::string> names;
  std::vector<double> ms;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  int id(const char* nm) {
    for (size_t i = 0; i < names.size(); ++i)
      if (names[i] == nm) return (int)i;
    names.push_back(nm);
    ms.push_back(0.0);
    return (int)names.size() - 1;
  }
  hipEvent_t ev() {
    if (used == pool.size()) {
      hipEvent_t e;
      HIPCHECK(hipEventCreate(&e));
      pool.push_back(e);
    }
    return pool[used++];
  }
};

struct Handle {
  Plan P;
  exacc_ccsd_opts op;
  hipStream_t s = nullptr;
  bool own_stream = false;
  std::vector<void*> allocs;
  std::vector<AllocRange> ranges;  // allocs with sizes, for the planner's extent check
  double* eps = nullptr;
  // Voovv and Vvovv_p exist in FP64 only while FP64 contractions are in use
  double *Bt = nullptr, *Voooo, *Vooov, *Voovv = nullptr, *Voovv_p, *Vvovv_p = nullptr;
  // Xp is reused for the ring output R once the ring intermediate is built;
  // Z holds the doubles residual pieces that carry no permutation operator
  double *x, *diis, *TAU, *taup, *Tq, *Xp, *H4, *Z, *Znp;
  double *Hac, *Gac, *Hki, *Gki, *Hkc, *y, *U, *Vt, *M1, *Y, *S1, *Cp, *Cf, *Af, *Ap;
  double *Ta, *W, *t1w;
  // FP32 copies of B and the stored integral classes (mixed precision only)
  float *Voovv_p32 = nullptr;  // FP32 <kl||cd> packed over k<l, c<d (low-precision hole ladder)
  float *Bt32 = nullptr, *Voooo32 = nullptr, *Vooov32 = nullptr, *Voovv32 = nullptr,
        *Vvovv_p32 = nullptr;
  // BF16x3 mode: the virtual-virtual factor rows B[(a,c)][P] split once into
  // bf16 hi/lo planes (layout of gemm_bf16x3_split), read by every ladder tile build
  unsigned short* Bvs = nullptr;
  bool phase32 = false;       // current iteration runs its contractions in FP32
  bool last32 = false;        // the last completed iteration ran in FP32
  int fp64_iters = 0;         // FP64 iterations since the last switch
  double best32 = -1.0;       // lowest ||Delta|| of the low-precision phase so far
  int since_best32 = 0;       // low-precision iterations since that lowest value
  // defect-corrected particle ladder after the switch (opts.ladder_defect_correction):
  // dc = 1: the next FP64 iteration stores tau_ref and Zref = L(tau_ref); dc = 2: the ladder
  // is Zref + L_low(tau - tau_ref); 0: off
  int dc = 0;
  bool last_dc = false;       // the last completed iteration used the corrected ladder
  double best_dc = -1.0;
  int since_best_dc = 0;
  double *tau_ref = nullptr, *Zref = nullptr;
  // ring part (plan.ring_dc): x_ref = amplitudes of the reference iteration, Rref = its
  // FP64 ring product H Tq, Href32 = FP32 H, D32 = FP32 correction dH; Ud, Vtd, t1d: the DF
  // t1 intermediates and t1 of the amplitude difference
  double *x_ref = nullptr, *Rref = nullptr, *Ud = nullptr, *Vtd = nullptr, *t1d = nullptr;
  double* Cref = nullptr;  // reference vovv.tau product of C^{kb}_{ij}, [(i<j)][b][k]
  float *Href32 = nullptr, *D32 = nullptr;
  // Lambda equations (App. D): buffers allocated on first use.  prepared: the
  // similarity-transformed Hamiltonian pieces (H4 = W_ovvo as [b][j][m][e], Cf = W_ovoo,
  // Ap = W_oooo packed, Gac/Gki/Hkc = F_vv/-F_oo/F_ov, Wooov, the dressed factor Bd) were
  // built from the current amplitudes and no other call has reused those buffers since.
  struct Lam {
    bool prepared = false;
    double *lam = nullptr;   // [l1 (o v), l2 (i<j, a<b)], L complex
    double *l1w, *Lq, *Z1, *Bd, *Wooov, *O3a, *O3b, *LTp, *Q1, *gP, *gt, *s1, *gam;
  } lam;
  int diis_owner = 0;         // 0: the amplitude DIIS history, 1: the Lambda one
  double* red = nullptr;      // reduction partials
  double* redout = nullptr;   // reduced values (device)
  double* host = nullptr;     // pinned readback
  int* rowmap_o = nullptr;    // k*o+l for pairs k<l
  // DIIS state
  std::vector<int> order;     // slot ids, oldest first
  std::vector<std::vector<zc>> G;
  double first_norm = -1.0;
  zc energy = 0.0;
  int iters = 0;
  Timer tm;

  // executable graphs of the residual computation (opts.graph_residual), one per iteration
  // kind: 0 FP64, 1 low precision, 2 FP64 with the defect-corrected products
  hipGraphExec_t gexec[3] = {nullptr, nullptr, nullptr};

  double* slot_x(int k) { return diis + (int64_t)2 * k * 2 * P.L; }
  double* slot_e(int k) { return diis + ((int64_t)2 * k + 1) * 2 * P.L; }

  ~Handle() {
    for (auto& g : gexec)
      if (g) (void)hipGraphExecDestroy(g);
    for (void* p : allocs) (void)hipFree(p);
    if (host) (void)hipHostFree(host);
    for (auto e : tm.pool) (void)hipEventDestroy(e);
    if (own_stream && s) (void)hipStreamDestroy(s);
  }
  void* ws = nullptr;  // split-K scratch
  size_t ws_bytes = 0;
  void use() {
    set_alloc_registry(ranges.data(), (int)ranges.size());
    set_gett_workspace(ws, ws_bytes);
  }
  template <typename T>
  void dfree(T*& p) {
    if (!p) return;
    for (size_t i = 0; i < allocs.size(); ++i)
      if (allocs[i] == (void*)p) {
        allocs.erase(allocs.begin() + i);
        break;
      }
    for (size_t i = 0; i < ranges.size(); ++i)
      if (ranges[i].base == (const void*)p) {
        ranges.erase(ranges.begin() + i);
        break;
      }
    HIPCHECK(hipFree(p));
    p = nullptr;
    use();
  }
  double* dalloc(int64_t complex_elems) {
    void* p = nullptr;
    const size_t b = (size_t)std::max<int64_t>(complex_elems, 1) * 16;
    HIPCHECK(hipMalloc(&p, b));
    allocs.push_back(p);
    ranges.push_back({p, b});
    set_alloc_registry(ranges.data(), (int)ranges.size());
    return (double*)p;
  }
};

// Calls after create that allocate on top of the handle (the Lambda buffers, the triples
// temporaries) stay within opts.hbm_budget_bytes together with what the handle holds.
static void check_budget(const Handle& h, size_t extra, const char* what) {
  if (!h.op.hbm_budget_bytes) return;
  size_t held = 0;
  for (const AllocRange& r : h.ranges) held += r.bytes;
  if (held + extra > h.op.hbm_budget_bytes)
    raise(EXACC_ERR_NOMEM, std::string(what) + " would exceed hbm_budget_bytes");
}

struct Scope {  // event-bracketed stage (only with opts.timing)
  Handle& h;
  int id;
  hipEvent_t a{}, b{};
  Scope(Handle& hh, const char* nm) : h(hh), id(-1) {
    if (!h.tm.on) return;
    id = h.tm.id(nm);
    a = h.tm.ev();
    b = h.tm.ev();
    HIPCHECK(hipEventRecord(a, h.s));
  }
  ~Scope() {
    if (id < 0) return;
    (void)hipEventRecord(b, h.s);
    h.tm.pending.push_back({id, {a, b}});
  }
};

static void timer_collect(Handle& h) {
  if (!h.tm.on) return;
  for (auto& pe : h.tm.pending) {
    float ms = 0;
    HIPCHECK(hipEventSynchronize(pe.second.second));
    HIPCHECK(hipEventElapsedTime(&ms, pe.second.first, pe.second.second));
    h.tm.ms[pe.first] += ms;
  }
  h.tm.pending.clear();
  h.tm.used = 0;
}

static const cplx ONE{1, 0}, MONE{-1, 0}, HALF{0.5, 0};

// ------------------------------------------------------------------ views
// Typed pointers for one precision.  R = double: the FP64 buffers.  R = float:
// FP32 integral copies; the work arrays alias the FP64 buffers (half their size).
template <typename R>
struct Work {
  R *Bt, *Voooo, *Vooov, *Voovv, *Vvovv_p;
  R *TAU, *taup, *Tq, *Xp, *H4, *R_, *Z, *Znp;
  R *Hac, *Gac, *Hki, *Gki, *Hkc, *y, *U, *Vt, *M1, *Y, *S1, *Cp, *Cf, *Af, *Ap, *Ta, *W;
  R* t1;  // t1 in R, as a contraction operand
};
template <typename R>
static Work<R> work(Handle& h);
template <>
Work<double> work<double>(Handle& h) {
  return Work<double>{h.Bt, h.Voooo, h.Vooov, h.Voovv, h.Vvovv_p, h.TAU, h.taup,
                      h.Tq, h.Xp, h.H4, h.Xp, h.Z, h.Znp, h.Hac, h.Gac, h.Hki, h.Gki,
                      h.Hkc, h.y, h.U, h.Vt, h.M1, h.Y, h.S1, h.Cp, h.Cf, h.Af, h.Ap, h.Ta, h.W,
                      h.t1w};
}
template <>
Work<float> work<float>(Handle& h) {
  auto f = [](double* p) { return reinterpret_cast<float*>(p); };
  return Work<float>{h.Bt32, h.Voooo32, h.Vooov32, h.Voovv32, h.Vvovv_p32,
                     f(h.TAU), f(h.taup), f(h.Tq), f(h.Xp), f(h.H4), f(h.Xp), f(h.Z),
                     f(h.Znp), f(h.Hac), f(h.Gac), f(h.Hki), f(h.Gki), f(h.Hkc),
                     f(h.y), f(h.U), f(h.Vt), f(h.M1), f(h.Y), f(h.S1), f(h.Cp),
                     f(h.Cf), f(h.Af), f(h.Ap), f(h.Ta), f(h.W), f(h.t1w)};
}

template <typename R>
struct Views {
  TV<R> Bvv, Bov, Bvo, Boo;
};
template <typename R>
static Views<R> bviews(Handle& h, R* Bt) {
  const int o = h.P.o, v = h.P.v, X = h.P.X, n = h.P.n;
  Views<R> w;
  const int64_t nX = (int64_t)n * X;
  w.Boo = sview(Bt, {o, o, X}, {nX, X, 1});
  w.Bov = sview(Bt + 2 * (int64_t)o * X, {o, v, X}, {nX, X, 1});
  w.Bvo = sview(Bt + 2 * (int64_t)o * nX, {v, o, X}, {nX, X, 1});
  w.Bvv = sview(Bt + 2 * ((int64_t)o * nX + (int64_t)o * X), {v, v, X}, {nX, X, 1});
  return w;
}

// Zero and copy inside the iteration run as kernels (a captured iteration graph then holds
// kernel nodes only).
template <typename R>
static void dzero(Handle& h, R* dst, int64_t celems) {
  k_zero_bytes(dst, celems * 2 * (int64_t)sizeof(R), h.s);
}

template <typename R>
static void dcopy(Handle& h, R* dst, const R* src, int64_t celems) {
  k_copy_bytes(dst, src, celems * 2 * (int64_t)sizeof(R), h.s);
}


// ------------------------------------------------------------------ integrals
// <kl||ij> = (ki|lj) - (kj|li) and <kl||ic> = (ki|lc) - (kc|li) (FP64, small)
static void build_oooo_ooov(Handle& h) {
  const int o = h.P.o, v = h.P.v;
  const hipStream_t s = h.s;
  Views<double> b = bviews(h, h.Bt);
  auto Voooo = view(h.Voooo, {o, o, o, o});
  contract(s, "kiP,ljP->klij", ONE, b.Boo, b.Boo, false, Voooo);
  contract(s, "kjP,liP->klij", MONE, b.Boo, b.Boo, true, Voooo);
  auto Vooov = view(h.Vooov, {o, o, o, v});
  contract(s, "kiP,lcP->klic", ONE, b.Boo, b.Bov, false, Vooov);
  contract(s, "kcP,liP->klic", MONE, b.Bov, b.Boo, true, Vooov);
}

// <kl||cd> = (kc|ld) - (kd|lc), full [k][l][c][d] FP64
static void build_oovv(Handle& h, double* dst) {
  const int o = h.P.o, v = h.P.v;
  Views<double> b = bviews(h, h.Bt);
  auto V = view(dst, {o, o, v, v});
  contract(h.s, "kcP,ldP->klcd", ONE, b.Bov, b.Bov, false, V);
  contract(h.s, "kdP,lcP->klcd", MONE, b.Bov, b.Bov, true, V);
}

// <bk||cd> = (bc|kd) - (bd|kc) packed over c<d, rows (b, k), built in chunks of b
// from the FP64 factors; T = float rounds each packed chunk into the FP32 copy.
template <typename T>
static void build_vovv_packed(Handle& h, T* dst) {
  const int o = h.P.o, v = h.P.v;
  if (h.P.Pv == 0) return;
  Views<double> b = bviews(h, h.Bt);
  const int64_t nX = (int64_t)h.P.n * h.P.X;
  const int64_t tmp_e = h.P.vovv_chunk * o * h.P.vv, stage_e = h.P.vovv_chunk * o * h.P.Pv;
  double* tmp = h.dalloc(tmp_e);
  double* stage = sizeof(T) == sizeof(double) ? nullptr : h.dalloc(stage_e);
  for (int b0 = 0; b0 < v; b0 += (int)h.P.vovv_chunk) {
    const int nb = (int)std::min<int64_t>(h.P.vovv_chunk, v - b0);
    auto Bc = sview(b.Bvv.p + 2 * (int64_t)b0 * nX, {nb, v, h.P.X}, {nX, h.P.X, 1});
    auto t = view(tmp, {nb, o, v, v});
    contract(h.s, "bcP,kdP->bkcd", ONE, Bc, b.Bov, false, t);
    contract(h.s, "bdP,kcP->bkcd", MONE, Bc, b.Bov, true, t);
    const int64_t rows = (int64_t)nb * o, off = (int64_t)b0 * o * h.P.Pv;
    if (stage) {
      k_pack_last2<double>(stage, tmp, nullptr, rows, v, h.P.vv, h.s);
      k_cast(stage, reinterpret_cast<float*>(dst) + 2 * off, 2 * rows * h.P.Pv, h.s);
    } else {
      k_pack_last2<double>(reinterpret_cast<double*>(dst) + 2 * off, tmp, nullptr, rows, v, h.P.vv, h.s);
    }
  }
  HIPCHECK(hipStreamSynchronize(h.s));
  h.dfree(tmp);
  h.dfree(stage);
}

// FP64 classes for FP64 contractions (mixed modes: at the switch; the FP32 copies go)
static void ensure_fp64_classes(Handle& h, bool keep_low_ladder = false) {
  if (h.Voovv && h.Vvovv_p) return;
  Scope sc(h, "switch_to_fp64");
  if (!keep_low_ladder || !h.Bvs) h.dfree(h.Bvs);
  // the FP32 factors stay for the corrected ring's t1 terms (and, in the FP32 mode, the ladder)
  if (!keep_low_ladder || (h.Bvs && !h.P.ring_dc)) h.dfree(h.Bt32);
  h.dfree(h.Voooo32);
  h.dfree(h.Vooov32);
  h.dfree(h.Voovv_p32);
  if (!keep_low_ladder || !h.P.ring_dc) h.dfree(h.Voovv32);
  if (!keep_low_ladder || !h.P.ring_dc) h.dfree(h.Vvovv_p32);
  h.Voovv = h.dalloc(h.P.oovv);
  build_oovv(h, h.Voovv);
  h.Vvovv_p = h.dalloc((int64_t)h.P.v * h.P.o * h.P.Pv);
  build_vovv_packed<double>(h, h.Vvovv_p);
}

// ------------------------------------------------------------------ residual pieces
// Fills S1 (singles, without the diagonal Fock part) and the doubles pieces
// Znp (packed) and Z (full) with no permutation left to apply, and R which
// still needs P_ij P_ab (applied in the assembly), for the
// amplitudes in h.x.
// Particle-ladder product Znp[p][(a<b)] += sum_{c<d} Lp[p][(c<d)] (F_ac.F_bd - F_ad.F_bc), the
// integrals formed tile by tile from factor rows F[a][c][P] (row a at F + a * row_stride,
// [c][P] contiguous) and never stored whole: for each a, Ta[c][b][d] = sum_P F_ac F_bd over
// b > a, antisymmetrised into W[(a,b)][(c<d)], then one GEMM per chunk of W rows.
// bf: BF16x3 products; the pre-split rows h.Bvs (when present) are the factor B_vv itself
// and may stand in for F only when use_bvs is set.
// herm: the factors are Hermitian (F_ac = conj F_ca, true of B_vv), so W as a matrix over
// pairs is Hermitian, <ab||cd> = conj <cd||ab>, and only its blocks on and above the
// diagonal are built (ladder_apply_herm); the Lambda equations' T1-dressed factors are not
// Hermitian and take the full build.
template <typename R>
static void ladder_apply_herm(Handle& h, const Work<R>& w, const R* F, int64_t row_stride,
                              const TV<R>& Lp, R* Znp, bool bf, bool use_bvs);
// Small nvir (plan.ladder_grouped): all virtual rows in three launches instead of two per
// row, the per-row products being too small to fill the chip.  T[a][c][b][d] = sum_P F_ac F_bd
// over all a, b, c, d in one product (v^4 naux complex multiply-adds against the Hermitian
// build's v^4 naux / 4, cheap at this size), W[(a<b)][(c<d)] = T[a][c][b][d] - T[a][d][b][c]
// in one pass, then Znp += Lp W^T.  Needs no Hermitian factors.
template <typename R>
static void ladder_apply_grouped(Handle& h, const Work<R>& w, const R* F, int64_t row_stride,
                                 const TV<R>& Lp, R* Znp, bool bf, bool use_bvs) {
  const int v = h.P.v, X = h.P.X;
  const int64_t Po = h.P.Po, Pv = h.P.Pv, vv = h.P.vv;
  const hipStream_t s = h.s;
  {
    Scope sc(h, "ladder_build");
    if (bf && use_bvs && h.Bvs) {  // pre-split rows (a, c), all v^2 of them contiguous
      gemm_bf16x3_split(h.Bvs, h.Bvs, (int)vv, (int)vv, X, reinterpret_cast<float*>(w.Ta), vv, s);
    } else {
      auto Fv = sview(const_cast<R*>(F), {v, v, X}, {row_stride, X, 1});
      contract(s, "acP,bdP->acbd", ONE, Fv, Fv, false, view(w.Ta, {v, v, v, v}),
               bf ? GETT_LADDER_BUILD_BF16X3 : GETT_LADDER_BUILD);
    }
  }
  {
    Scope sc(h, "ladder_antisym");
    k_ladder_antisym_all<R>(w.Ta, w.W, v, s);
  }
  Scope sc(h, "ladder_contract");
  contract(s, "py,xy->px", ONE, Lp, view(w.W, {Pv, Pv}), true, sview(Znp, {Po, Pv}, {Pv, 1}),
           bf ? GETT_LADDER_CONTRACT_BF16X3 : GETT_LADDER_CONTRACT);
}

template <typename R>
static void ladder_apply(Handle& h, const Work<R>& w, const R* F, int64_t row_stride, const TV<R>& Lp,
                         R* Znp, bool bf, bool use_bvs, bool herm) {
  if (h.P.ladder_grouped && h.P.Po > 0 && h.P.Pv > 0)
    return ladder_apply_grouped<R>(h, w, F, row_stride, Lp, Znp, bf, use_bvs);
  if (herm) return ladder_apply_herm<R>(h, w, F, row_stride, Lp, Znp, bf, use_bvs);
  const int v = h.P.v, X = h.P.X;
  const int64_t Po = h.P.Po, Pv = h.P.Pv;
  const hipStream_t s = h.s;
  const int lad_build = bf ? GETT_LADDER_BUILD_BF16X3 : GETT_LADDER_BUILD;
  const int lad_contract = bf ? GETT_LADDER_CONTRACT_BF16X3 : GETT_LADDER_CONTRACT;
  if (Po == 0 || Pv == 0) return;
  int64_t rows = 0, start = 0;
  auto flush = [&]() {
    if (rows == 0) return;
    Scope sc(h, "ladder_contract");
    auto Wv = view(w.W, {rows, Pv});
    auto Zc = sview(Znp + 2 * start, {Po, rows}, {Pv, 1});
    contract(s, "py,xy->px", ONE, Lp, Wv, true, Zc, lad_contract);
    start += rows;
    rows = 0;
  };
  for (int a = 0; a + 1 < v; ++a) {
    const int nb = v - a - 1;
    if (rows + nb > h.P.chunk_pairs) flush();
    {
      Scope sc(h, "ladder_build");
      if (bf && use_bvs && h.Bvs) {  // Ta[c][b][d] = sum_P B[(a,c)][P] B[(b,d)][P], b > a, pre-split rows
        const int64_t rs = 4 * (int64_t)bf16x3_split_k(X);
        gemm_bf16x3_split(h.Bvs + (int64_t)a * v * rs, h.Bvs + (int64_t)(a + 1) * v * rs, v, nb * v, X,
                          reinterpret_cast<float*>(w.Ta), (int64_t)nb * v, s);
      } else {
        auto Ba = sview(const_cast<R*>(F) + 2 * (int64_t)a * row_stride, {v, X}, {X, 1});
        auto Bb = sview(const_cast<R*>(F) + 2 * (int64_t)(a + 1) * row_stride, {nb, v, X}, {row_stride, X, 1});
        contract(s, "cP,bdP->cbd", ONE, Ba, Bb, false, view(w.Ta, {v, nb, v}), lad_build);
      }
    }
    {
      Scope sc(h, "ladder_antisym");
      k_ladder_antisym<R>(w.Ta, w.W + 2 * rows * Pv, nb, v, Pv, s);
    }
    rows += nb;
  }
  flush();
}

// Chunks [a0, a1) of virtual rows for the Hermitian ladder: W holds rows x Pw (Pw =
// pairs of the w = v - a0 virtuals c, d >= a0) and, with the transposed tail, (Pw - rows)
// x rows more; a chunk takes rows while that fits in cap elements (at least one row; the
// W buffer holds one row of the first chunk in either layout).
struct LadderChunk {
  int a0, a1;
  int64_t rows;
};
static std::vector<LadderChunk> ladder_chunks(int v, int64_t cap, bool tail) {
  std::vector<LadderChunk> out;
  for (int a0 = 0; a0 + 1 < v;) {
    const int64_t Pw = npair(v - a0);
    int a1 = a0;
    int64_t rows = 0;
    while (a1 + 1 < v) {
      const int64_t r2 = rows + (v - a1 - 1);
      if (rows > 0 && r2 * Pw + (tail ? (Pw - r2) * r2 : 0) > cap) break;
      rows = r2;
      ++a1;
    }
    out.push_back({a0, a1, rows});
    a0 = a1;
  }
  return out;
}

// Packed index of the first pair (a, a + 1) over v virtuals.
static inline int64_t pair_offset(int a, int v) { return (int64_t)a * v - (int64_t)a * (a + 1) / 2; }

// The pairs (c<d) with c >= a0 are the tail [pair_offset(a0), P_v) of the packed pair
// range, and the rows (a, b > a), a in [a0, a1), of a chunk are its first `rows` pairs.
// Per chunk: for each a, Ta[c][b][d] = sum_P F_ac F_bd over c, d >= a0 and b > a
// (w^2 (v - a - 1) naux complex multiply-adds instead of v^2 (v - a - 1) naux),
// antisymmetrised into W[(a,b)][(c<d), c >= a0]; then
//   forward:  Znp[:, (ab) in chunk] += Lp[:, tail] W^T           (all c >= a0)
//   backward: Znp[:, (cd), c >= a1] += Lp[:, chunk] conj(W[:, c >= a1])
// The backward product gives each later row the part of its sum over (c<d) in this chunk,
// W[(cd)][(ab)] = conj W[(ab)][(cd)]; so every Znp column receives the sum over all pairs.
// The backward product reads W through its transpose (K contiguous) for the BF16x3 GEMM,
// directly (K strided) otherwise.
template <typename R>
static void ladder_apply_herm(Handle& h, const Work<R>& w, const R* F, int64_t row_stride,
                              const TV<R>& Lp, R* Znp, bool bf, bool use_bvs) {
  const int v = h.P.v, X = h.P.X;
  const int64_t Po = h.P.Po, Pv = h.P.Pv;
  const hipStream_t s = h.s;
  if (Po == 0 || Pv == 0) return;
  const int lad_build = bf ? GETT_LADDER_BUILD_BF16X3 : GETT_LADDER_BUILD;
  const int lad_contract = bf ? GETT_LADDER_CONTRACT_BF16X3 : GETT_LADDER_CONTRACT;
  const bool tail_t = bf;
  // W buffer capacity in complex elements of R (the FP32 types alias the FP64 buffer)
  const int64_t cap = h.P.chunk_pairs * Pv * (int64_t)(sizeof(double) / sizeof(R));
  const int64_t ldl = Lp.str[0];
  for (const LadderChunk& ch : ladder_chunks(v, cap, tail_t)) {
    const int a0 = ch.a0, wv = v - a0;
    const int64_t Pw = npair(wv), rows = ch.rows, off = pair_offset(a0, v);
    int64_t xoff = 0;
    for (int a = a0; a < ch.a1; ++a) {
      const int nb = v - a - 1;
      {
        Scope sc(h, "ladder_build");
        if (bf && use_bvs && h.Bvs) {  // pre-split rows B[(a, c)] and B[(b, d)], c, d >= a0
          const int64_t rs = 4 * (int64_t)bf16x3_split_k(X);
          gemm_bf16x3_split(h.Bvs + ((int64_t)a * v + a0) * rs, h.Bvs + ((int64_t)(a + 1) * v + a0) * rs,
                            wv, nb * wv, X, reinterpret_cast<float*>(w.Ta), (int64_t)nb * wv, s, wv, v);
        } else {
          auto Ba = sview(const_cast<R*>(F) + 2 * ((int64_t)a * row_stride + (int64_t)a0 * X), {wv, X}, {X, 1});
          auto Bb = sview(const_cast<R*>(F) + 2 * ((int64_t)(a + 1) * row_stride + (int64_t)a0 * X),
                          {nb, wv, X}, {row_stride, X, 1});
          contract(s, "cP,bdP->cbd", ONE, Ba, Bb, false, view(w.Ta, {wv, nb, wv}), lad_build);
        }
      }
      {
        Scope sc(h, "ladder_antisym");
        k_ladder_antisym<R>(w.Ta, w.W + 2 * xoff * Pw, nb, wv, Pw, s);
      }
      xoff += nb;
    }
    Scope sc(h, "ladder_contract");
    auto Lt = sview(Lp.p + 2 * off, {Po, Pw}, {ldl, 1});
    contract(s, "py,xy->px", ONE, Lt, view(w.W, {rows, Pw}), true,
             sview(Znp + 2 * off, {Po, rows}, {Pv, 1}), lad_contract);
    const int64_t nt = Pw - rows;
    if (nt > 0) {
      auto Lc = sview(Lp.p + 2 * off, {Po, rows}, {ldl, 1});
      auto Zt = sview(Znp + 2 * (off + rows), {Po, nt}, {Pv, 1});
      if (tail_t) {
        R* Wt = w.W + 2 * rows * Pw;
        k_transpose_tail<R>(w.W, rows, Pw, rows, nt, Wt, rows, s);
        contract(s, "px,yx->py", ONE, Lc, conj(view(Wt, {nt, rows})), true, Zt, lad_contract);
      } else {
        contract(s, "px,xy->py", ONE, Lc, conj(sview(w.W + 2 * rows, {rows, nt}, {Pw, 1})), true, Zt,
                 lad_contract);
      }
    }
  }
}

// The ring term of the FP64 iterations after a mixed-precision switch (when its reference
// arrays fit): with H = H^{ak}_{ci}, Tq the permuted T2 and the reference point of the
// first FP64 iteration (x_ref, Rref = H_ref Tq_ref, Href32),
//   H Tq = Rref + H_ref dTq + dH Tq,   dH = H1(dt1) + dXp <kl||cd>,
// exactly, where d = current - reference, H1 the t1-linear DF terms of H and Xp the
// ring operand (t2 / 2 + t1 t1): the differences are formed in FP64 from the amplitudes,
// the three o^3 v^3 products run in the low precision of the mode (their rounding is
// relative to the small differences), and so do the two o^2 v^2 naux products of H1(dt1),
// on the FP32 factors kept through the corrected phase (its o^3 v^2 ooov term stays FP64).
// Scratch: Z and H4 as FP32 halves (dT2 then Tq; dTq, dXp), Xp for the FP64 part of dH
// before it takes R, the FP64 DF buffers Ud and Vtd for their FP32 counterparts.
static void ring_defect_corrected(Handle& h, const Work<double>& w, const Views<double>& b, bool ccd) {
  const int o = h.P.o, v = h.P.v, X = h.P.X;
  const hipStream_t s = h.s;
  const int64_t ov = (int64_t)o * v, oovv = h.P.oovv;
  const int rk = h.op.precision == EXACC_MIXED_BF16X3 ? GETT_RING_BF16X3 : GETT_RING;
  float* Za = reinterpret_cast<float*>(w.Z);
  float* Zb = Za + 2 * oovv;
  float* Ha = reinterpret_cast<float*>(w.H4);
  float* Hb = Ha + 2 * oovv;
  {
    Scope sc(h, "ring_dc");
    k_sub(h.x, h.x_ref, h.t1d, 2 * ov, s);
    k_unpack_diff(h.x + 2 * ov, h.x_ref + 2 * ov, Za, o, v, s);
    k_ring_operands<float>(Za, h.x, Ha, Hb, o, v, s, h.x_ref);  // dTq, dXp
    k_cast(w.Tq, Za, 2 * oovv, s);                               // Tq in FP32
  }
  if (!ccd && h.Bt32) {
    // H1(dt1) on the FP32 factors: the two o^2 v^2 naux products in the mode's low
    // precision (their rounding is relative to dt1), the o^3 v^2 ooov term in FP64
    Scope sc(h, "ring_dc");
    Views<float> b32 = bviews(h, h.Bt32);
    float* Vtd32 = reinterpret_cast<float*>(h.Vtd);  // v o X complex, half of the FP64 buffer
    float* t1d32 = Vtd32 + 2 * (int64_t)v * o * X;   // o v complex, in the other half
    float* Ud32 = reinterpret_cast<float*>(h.Ud);
    k_cast(h.t1d, t1d32, 2 * ov, s);
    auto t1d = view(t1d32, {o, v});
    auto Ud = view(Ud32, {o, o, X});
    auto Vtd = view(Vtd32, {v, o, X});
    contract(s, "kdP,id->kiP", ONE, b32.Bov, t1d, false, Ud);
    contract(s, "acP,ic->aiP", ONE, b32.Bvv, t1d, false, Vtd);
    contract(s, "klic,la->aikc", MONE, view(w.Vooov, {o, o, o, v}), view(h.t1d, {o, v}), false,
             view(w.Xp, {v, o, o, v}));
    k_cast(w.Xp, h.D32, 2 * oovv, s);
    auto D = view(h.D32, {v, o, o, v});
    contract(s, "acP,kiP->aikc", ONE, b32.Bvv, Ud, true, D, rk);
    contract(s, "aiP,kcP->aikc", MONE, Vtd, b32.Bov, true, D, rk);
  } else if (!ccd) {
    Scope sc(h, "ring_dc");
    auto t1d = view(h.t1d, {o, v});
    auto Ud = view(h.Ud, {o, o, X});
    auto Vtd = view(h.Vtd, {v, o, X});
    auto Hd = view(w.Xp, {v, o, o, v});
    contract(s, "kdP,id->kiP", ONE, b.Bov, t1d, false, Ud);
    contract(s, "acP,ic->aiP", ONE, b.Bvv, t1d, false, Vtd);
    contract(s, "acP,kiP->aikc", ONE, b.Bvv, Ud, false, Hd);
    contract(s, "aiP,kcP->aikc", MONE, Vtd, b.Bov, true, Hd);
    contract(s, "klic,la->aikc", MONE, view(w.Vooov, {o, o, o, v}), t1d, true, Hd);
    k_cast(w.Xp, h.D32, 2 * oovv, s);
  } else {
    dzero(h, h.D32, oovv);
  }
  {
    Scope sc(h, "ring_build");
    const int64_t o_vv = (int64_t)o * v * v;
    auto V32 = sview(h.Voovv32, {o, o, v, v}, {o_vv, (int64_t)v, ov, 1});
    contract(s, "aild,klcd->aikc", ONE, view(Hb, {v, o, o, v}), V32, true, view(h.D32, {v, o, o, v}), rk);
  }
  {
    Scope sc(h, "ring");
    auto Rl = view(Zb, {o, o, v, v});
    contract(s, "aikc,bjkc->ijab", ONE, view(h.Href32, {v, o, o, v}), view(Ha, {v, o, o, v}), false, Rl, rk);
    contract(s, "aikc,bjkc->ijab", ONE, view(h.D32, {v, o, o, v}), view(Za, {v, o, o, v}), true, Rl, rk);
    dzero(h, w.R_, oovv);
    k_add2(w.R_, h.Rref, Zb, 2 * oovv, s);
    if (!ccd)
      contract(s, "aiP,bjP->ijab", ONE, view(w.Vt, {v, o, X}), b.Bvo, true, view(w.R_, {o, o, v, v}));
  }
}

// The particle ladder of the FP64 iterations after a mixed-precision switch.  dc = 1: the
// full FP64 product at the current amplitudes, kept as Zref = L(tau_ref) with tau_ref.
// dc = 2: L(tau) = L(tau_ref) + L(tau - tau_ref), the second product in the mode's low
// precision (FP32, or BF16x3 on the kept split rows) on the FP32 rounding of the FP64
// difference tau - tau_ref; its rounding error is relative to |tau - tau_ref|, which is
// about the step norm at the switch and does not grow as the iteration converges.  The
// FP32 difference and product live in the H4 work array, free once the ring is done.
static void ladder_defect_corrected(Handle& h, const Work<double>& w, const TV<double>& taup) {
  const int64_t np = h.P.Po * h.P.Pv, nX = (int64_t)h.P.n * h.P.X;
  if (np == 0) return;
  if (h.dc == 1) {
    Views<double> b = bviews(h, h.Bt);
    dzero(h, h.Zref, np);
    ladder_apply<double>(h, w, b.Bvv.p, nX, taup, h.Zref, false, true, true);
    Scope sc(h, "ladder_dc");
    k_add2(w.Znp, h.Zref, nullptr, 2 * np, h.s);
    dcopy(h, h.tau_ref, w.taup, np);
    return;
  }
  Work<float> w32 = work<float>(h);
  float* dtau = reinterpret_cast<float*>(h.H4);
  float* Zd = dtau + 2 * np;
  {
    Scope sc(h, "ladder_dc");
    k_diff_cast(w.taup, h.tau_ref, dtau, 2 * np, h.s);
    dzero(h, Zd, np);
  }
  const bool bf = h.op.precision == EXACC_MIXED_BF16X3 && h.Bvs;
  const float* F = h.Bt32 ? bviews(h, h.Bt32).Bvv.p : nullptr;
  if (!bf && !F) raise(EXACC_ERR_DEVICE, "defect-corrected ladder without its low-precision factors");
  ladder_apply<float>(h, w32, F, nX, view(dtau, {h.P.Po, h.P.Pv}), Zd, bf, true, true);
  Scope sc(h, "ladder_dc");
  k_add2(w.Znp, h.Zref, Zd, 2 * np, h.s);
}

template <typename R>
static void compute_residual(Handle& h) {
  Work<R> w = work<R>(h);
  const int o = h.P.o, v = h.P.v, X = h.P.X;
  const int64_t Po = h.P.Po, Pv = h.P.Pv;
  const hipStream_t s = h.s;
  // BF16x3 products for the ladder and ring in the low-precision phase of the BF16x3 mode
  const bool bf = sizeof(R) == sizeof(float) && h.op.precision == EXACC_MIXED_BF16X3;
  const int ring_kind = bf ? GETT_RING_BF16X3 : GETT_RING;
  // the density-fitted o^2 v^2 naux terms of the ring intermediate and the vovv . tau
  // product of C^{kb}_{ij} (K contiguous in both operands) also take BF16x3 products there
  const int df_kind = bf ? GETT_RING_BF16X3 : GETT_GENERIC;
  // CCD: t1 is zero, so every contraction with a t1 (or U, Vt, y) factor is skipped
  const bool ccd = h.op.doubles_only != 0;
  Views<R> b = bviews(h, w.Bt);
  const double* t1p = h.x;
  const double* t2p = h.x + 2 * (int64_t)o * v;
  auto t1 = view(w.t1, {o, v});
  // T2[i][k][a][b] read through the permuted copy Tq[b][i][k][a]
  const int64_t ov = (int64_t)o * v, oov = (int64_t)o * o * v;
  auto T2 = sview(w.Tq, {o, o, v, v}, {ov, v, 1, oov});
  auto TAU = view(w.TAU, {o, o, v, v});
  auto taup = view(w.taup, {Po, Pv});
  // <kl||cd>: FP64 stored [k][l][c][d]; the FP32 copy is stored [k][c][l][d] so that the
  // ring build's K = (l, d) is contiguous (BF16x3-eligible); other uses read it strided
  const int64_t o_vv = (int64_t)o * v * v;
  auto Voovv = sizeof(R) == sizeof(double)
                   ? view(w.Voovv, {o, o, v, v})
                   : sview(w.Voovv, {o, o, v, v}, {o_vv, (int64_t)v, (int64_t)o * v, 1});
  auto Vooov = view(w.Vooov, {o, o, o, v});
  {
    Scope sc(h, "prep");
    if (sizeof(R) == sizeof(double))
      dcopy(h, (double*)w.t1, h.x, (int64_t)o * v);
    else
      k_cast(h.x, (float*)w.t1, 2 * (int64_t)o * v, s);
    // full T2 goes to Z as scratch: Z is first written after Tq and Xp exist
    k_unpack_tau<R>(t1p, t2p, w.Z, w.TAU, w.taup, o, v, s);
    k_ring_operands<R>(w.Z, t1p, w.Tq, w.Xp, o, v, s);
  }
  auto U = view(w.U, {o, o, X});
  auto Vt = view(w.Vt, {v, o, X});
  auto Hac = view(w.Hac, {v, v}), Gac = view(w.Gac, {v, v});
  auto Hki = view(w.Hki, {o, o}), Gki = view(w.Gki, {o, o});
  auto Hkc = view(w.Hkc, {o, v});
  {
    Scope sc(h, "onebody");
    contract(s, "klcd,klda->ac", HALF, Voovv, TAU, false, Hac);
    contract(s, "klcd,licd->ki", HALF, Voovv, TAU, false, Hki);
    dcopy(h, w.Gac, w.Hac, (int64_t)v * v);
    dcopy(h, w.Gki, w.Hki, (int64_t)o * o);
  }
  if (!ccd) {
    Scope sc(h, "onebody");
    contract(s, "klcd,ld->kc", ONE, Voovv, t1, false, Hkc);
    // DF t1 intermediates: y^P = sum_kd B^P_kd t_k^d, U^P_ki = sum_d B^P_kd t_i^d,
    // Vt^P_ai = sum_c B^P_ac t_i^c
    auto y = view(w.y, {X});
    contract(s, "kdP,kd->P", ONE, b.Bov, t1, false, y);
    contract(s, "kdP,id->kiP", ONE, b.Bov, t1, false, U);
    contract(s, "acP,ic->aiP", ONE, b.Bvv, t1, false, Vt);
    // sum_kd <ak||cd> t_k^d = sum_kd (ac|kd) t_k^d - sum_kd (ad|kc) t_k^d
    //                       = sum_P B^P_ac y^P - sum_kP Vt^P_ak B^P_kc
    contract(s, "acP,P->ac", ONE, b.Bvv, y, true, Gac);
    contract(s, "akP,kcP->ac", MONE, Vt, b.Bov, true, Gac);
    contract(s, "klic,lc->ki", MONE, Vooov, t1, true, Gki);
  }
  // singles residual S1 (CCSD's, also CC2's)
  auto singles = [&]() {
    Scope sc(h, "singles");
    auto S1 = view(w.S1, {o, v});
    contract(s, "ac,ic->ia", ONE, Hac, t1, false, S1);
    contract(s, "ki,ka->ia", ONE, Hki, t1, true, S1);
    contract(s, "kc,ikac->ia", ONE, Hkc, T2, true, S1);
    auto M1 = view(w.M1, {o, o});
    contract(s, "kc,ic->ki", ONE, Hkc, t1, false, M1);
    contract(s, "ki,ka->ia", ONE, M1, t1, true, S1);
    auto Y = view(w.Y, {o, v, X});
    contract(s, "ikcd,kdP->icP", ONE, TAU, b.Bov, false, Y);
    contract(s, "icP,acP->ia", ONE, Y, b.Bvv, true, S1);
    contract(s, "klic,klca->ia", HALF, Vooov, TAU, true, S1);
    // - sum_kc <ak||ci> t_k^c = - sum_kP Vt^P_ak B^P_ki + sum_P B^P_ai y^P
    contract(s, "akP,kiP->ia", MONE, Vt, b.Boo, true, S1);
    contract(s, "aiP,P->ia", ONE, b.Bvo, view(w.y, {X}), true, S1);
  };
  if (h.op.cc2) {
    // CC2 doubles: <ab||ij> of the T1-transformed Hamiltonian, from the dressed factor
    // B~^P_ai = B^P_ai + sum_c B^P_ac t_i^c - sum_k t_k^a (B^P_ki + sum_d B^P_kd t_i^d);
    // the assembly adds (e_a + e_b - e_i - e_j) t_ij^ab and nothing else
    singles();
    Scope sc(h, "cc2_doubles");
    auto Q = view(w.Y, {v, o, X});  // the singles' Y is free again
    contract(s, "kiP,ka->aiP", ONE, U, t1, false, Q);
    contract(s, "kiP,ka->aiP", ONE, b.Boo, t1, true, Q);
    k_dress_vo<R>(w.Vt, w.Bt, w.Y, o, v, h.P.n, X, s);
    auto Z = view(w.Z, {o, o, v, v});
    auto Zji = sview(w.Z, {o, o, v, v}, {(int64_t)v * v, (int64_t)o * v * v, v, 1});
    contract(s, "aiP,bjP->ijab", ONE, Vt, Vt, false, Z);
    contract(s, "aiP,bjP->ijab", MONE, Vt, Vt, true, Zji);
    return;
  }
  auto H4 = view(w.H4, {v, o, o, v});
  bool ring_done = false;
  if constexpr (sizeof(R) == sizeof(double)) {
    if (h.dc == 2 && h.P.ring_dc) {
      ring_defect_corrected(h, w, b, ccd);
      ring_done = true;
    }
  }
  if (!ring_done) {
  {
    Scope sc(h, "ring_build");
    // <ak||ci> = (ac|ki) - (ai|kc), formed from the factors each iteration
    contract(s, "acP,kiP->aikc", ONE, b.Bvv, b.Boo, false, H4, df_kind);
    contract(s, "aiP,kcP->aikc", MONE, b.Bvo, b.Bov, true, H4, df_kind);
    if (!ccd) {
      contract(s, "acP,kiP->aikc", ONE, b.Bvv, U, true, H4, df_kind);
      contract(s, "aiP,kcP->aikc", MONE, Vt, b.Bov, true, H4, df_kind);
      contract(s, "klic,la->aikc", MONE, Vooov, t1, true, H4);
    }
    contract(s, "aild,klcd->aikc", ONE, view(w.Xp, {v, o, o, v}), Voovv, true, H4, ring_kind);
  }
  auto Rv = view(w.R_, {o, o, v, v});
  {
    Scope sc(h, "ring");
    contract(s, "aikc,bjkc->ijab", ONE, H4, view(w.Tq, {v, o, o, v}), false, Rv, ring_kind);
    if constexpr (sizeof(R) == sizeof(double)) {
      if (h.dc == 1 && h.P.ring_dc) {  // reference point of the corrected ring
        dcopy(h, h.Rref, w.R_, h.P.oovv);
        k_cast(w.H4, h.Href32, 2 * h.P.oovv, s);
        dcopy(h, h.x_ref, h.x, h.P.L);
      }
    }
    if (!ccd) contract(s, "aiP,bjP->ijab", ONE, Vt, b.Bvo, true, Rv, df_kind);
  }
  }
  // Z and its views with i<->j or a<->b swapped: a term X launched into Z and,
  // negated, into a swapped view accumulates P^-_ij X (or P^-_ab X) directly
  const int64_t vv = (int64_t)v * v, ovv = (int64_t)o * v * v;
  auto Z = view(w.Z, {o, o, v, v});
  auto Zji = sview(w.Z, {o, o, v, v}, {vv, ovv, v, 1});
  auto Zba = sview(w.Z, {o, o, v, v}, {ovv, vv, 1, v});
  {
    Scope sc(h, "fock_terms");
    contract(s, "kj,ikab->ijab", ONE, Gki, T2, false, Z);
    contract(s, "kj,ikab->ijab", MONE, Gki, T2, true, Zji);
    contract(s, "ac,ijcb->ijab", ONE, Gac, T2, true, Z);
    contract(s, "ac,ijcb->ijab", MONE, Gac, T2, true, Zba);
  }
  if (!ccd) {  // C^{kb}_{ij} enters only through P_ab sum_k C t_k^a
    Scope sc(h, "cterm");
    auto Cp = view(w.Cp, {Po, v, o});
    bool cdone = false;
    if constexpr (sizeof(R) == sizeof(double)) {
      if (h.P.ring_dc && h.dc == 2) {  // Cp = Cp(tau_ref) - vovv_low . (tau - tau_ref)_low
        const int64_t np = Po * Pv, nc = Po * v * o;
        float* dtau = reinterpret_cast<float*>(w.H4);
        float* C32 = dtau + 2 * h.P.oovv;
        k_diff_cast(w.taup, h.tau_ref, dtau, 2 * np, s);
        const int ck = h.op.precision == EXACC_MIXED_BF16X3 ? GETT_RING_BF16X3 : GETT_GENERIC;
        contract(s, "bkx,px->pbk", MONE, view(h.Vvovv_p32, {v, o, Pv}), view(dtau, {Po, Pv}), false,
                 view(C32, {Po, v, o}), ck);
        dzero(h, w.Cp, nc);
        k_add2(w.Cp, h.Cref, C32, 2 * nc, s);
        cdone = true;
      }
    }
    if (!cdone) contract(s, "bkx,px->pbk", MONE, view(w.Vvovv_p, {v, o, Pv}), taup, false, Cp, df_kind);
    if constexpr (sizeof(R) == sizeof(double)) {
      if (h.P.ring_dc && h.dc == 1) dcopy(h, h.Cref, w.Cp, Po * v * o);
    }
    k_expand_c<R>(w.Vooov, w.Cp, w.Cf, o, v, s);
    auto Cf = view(w.Cf, {o, o, v, o});
    // P^-_ij sum_c <bk||ci> t_j^c with <bk||ci> = (bc|ki) - (bi|kc):
    //   sum_c (bc|ki) t_j^c = sum_P Vt^P_bj B^P_ki,  sum_c (bi|kc) t_j^c = sum_P B^P_bi U^P_kj
    const int64_t vo = (int64_t)v * o, oo = (int64_t)o * o, oovo = oo * v * o;
    auto Cfji = sview(w.Cf, {o, o, v, o}, {vo, o * vo, o, 1});
    contract(s, "bjP,kiP->ijbk", ONE, Vt, b.Boo, true, Cf);
    contract(s, "biP,kjP->ijbk", MONE, b.Bvo, U, true, Cf);
    contract(s, "bjP,kiP->ijbk", MONE, Vt, b.Boo, true, Cfji);
    contract(s, "biP,kjP->ijbk", ONE, b.Bvo, U, true, Cfji);
    (void)oovo;
    contract(s, "ijak,kb->ijab", ONE, Cf, t1, true, Z);
    contract(s, "ijak,kb->ijab", MONE, Cf, t1, true, Zba);
  }
  auto Znp = view(w.Znp, {Po, Pv});
  {
    Scope sc(h, "hole_ladder");
    auto Af = view(w.Af, {o, o, o, o});
    dcopy(h, w.Af, w.Voooo, (int64_t)o * o * o * o);
    if (!ccd) {
      contract(s, "klic,jc->klij", ONE, Vooov, t1, true, Af);
      contract(s, "kljc,ic->klij", MONE, Vooov, t1, true, Af);
    }
    if constexpr (sizeof(R) == sizeof(double)) {
      // 1/2 sum_cd <kl||cd> tau_ij^cd = sum_{c<d} <kl||cd> tau_ij^cd, formed on the packed
      // pairs (k<l), (i<j), (c<d) that A enters the hole ladder with: P_o^2 P_v complex
      // multiply-adds instead of o^4 v^2 / 2
      if (Po > 0) {
        k_pack_last2<R>(w.Ap, w.Af, h.rowmap_o, Po, o, (int64_t)o * o, s);
        contract(s, "qx,px->qp", ONE, view(h.Voovv_p, {Po, Pv}), taup, true, view(w.Ap, {Po, Po}));
      }
    } else if (h.Voovv_p32) {  // the same on the FP32 copy of the packed class
      if (Po > 0) {
        k_pack_last2<R>(w.Ap, w.Af, h.rowmap_o, Po, o, (int64_t)o * o, s);
        contract(s, "qx,px->qp", ONE, view(h.Voovv_p32, {Po, Pv}), taup, true, view(w.Ap, {Po, Po}));
      }
    } else {
      contract(s, "klcd,ijcd->klij", HALF, Voovv, TAU, true, Af);
      if (Po > 0) k_pack_last2<R>(w.Ap, w.Af, h.rowmap_o, Po, o, (int64_t)o * o, s);
    }
    contract(s, "qp,qx->px", ONE, view(w.Ap, {Po, Po}), taup, false, Znp);
  }
  // particle ladder: Znp[ij][ab] += sum_{c<d} tau[ij][cd] <ab||cd>, <ab||cd> = (ac|bd) - (ad|bc)
  // (BF16x3 products in the low-precision phase of the BF16x3 mode)
  bool ladder_done = false;
  if constexpr (sizeof(R) == sizeof(double)) {
    if (h.dc != 0) {
      ladder_defect_corrected(h, w, taup);
      ladder_done = true;
    }
  }
  if (!ladder_done) ladder_apply<R>(h, w, b.Bvv.p, (int64_t)h.P.n * X, taup, w.Znp, bf, true, true);
  if (ccd)
    dzero(h, w.S1, (int64_t)o * v);
  else
    singles();
}

// ------------------------------------------------------------------ small host linear algebra
// Eigenvalues of a Hermitian m x m matrix via cyclic Jacobi on its real 2m x 2m embedding.
static std::vector<double> herm_eigvals(const std::vector<std::vector<zc>>& Gm) {
  const int m = (int)Gm.size(), N = 2 * m;
  std::vector<double> a(N * N);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      const double re = Gm[i][j].real(), im = Gm[i][j].imag();
      a[i * N + j] = re;
      a[(i + m) * N + (j + m)] = re;
      a[i * N + (j + m)] = -im;
      a[(i + m) * N + j] = im;
    }
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0, tot = 0;
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) {
        tot += a[i * N + j] * a[i * N + j];
        if (i != j) off += a[i * N + j] * a[i * N + j];
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < N; ++p)
      for (int q = p + 1; q < N; ++q) {
        const double apq = a[p * N + q];
        if (apq == 0.0) continue;
        const double theta = (a[q * N + q] - a[p * N + p]) / (2 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1));
        const double c = 1 / std::sqrt(t * t + 1), sn = t * c;
        for (int k = 0; k < N; ++k) {
          const double akp = a[k * N + p], akq = a[k * N + q];
          a[k * N + p] = c * akp - sn * akq;
          a[k * N + q] = sn * akp + c * akq;
        }
        for (int k = 0; k < N; ++k) {
          const double apk = a[p * N + k], aqk = a[q * N + k];
          a[p * N + k] = c * apk - sn * aqk;
          a[q * N + k] = sn * apk + c * aqk;
        }
      }
  }
  std::vector<double> w(N);
  for (int i = 0; i < N; ++i) w[i] = a[i * N + i];
  std::sort(w.begin(), w.end());
  std::vector<double> out(m);
  for (int i = 0; i < m; ++i) out[i] = w[2 * i];  // each eigenvalue appears twice
  return out;
}

// Solve the (m+1) bordered DIIS system [[G, 1], [1^T, 0]] [c; lam] = [0; 1].
static std::vector<zc> diis_solve(const std::vector<std::vector<zc>>& Gm) {
  const int m = (int)Gm.size(), N = m + 1;
  std::vector<zc> A(N * N, 0.0), r(N, 0.0);
  for (int i = 0; i < m; ++i) {
    for (int j = 0; j < m; ++j) A[i * N + j] = Gm[i][j];
    A[i * N + m] = 1.0;
    A[m * N + i] = 1.0;
  }
  r[m] = 1.0;
  for (int c = 0; c < N; ++c) {
    int piv = c;
    for (int i = c + 1; i < N; ++i)
      if (std::abs(A[i * N + c]) > std::abs(A[piv * N + c])) piv = i;
    if (piv != c) {
      for (int j = 0; j < N; ++j) std::swap(A[c * N + j], A[piv * N + j]);
      std::swap(r[c], r[piv]);
    }
    const zc d = A[c * N + c];
    for (int i = c + 1; i < N; ++i) {
      const zc f = A[i * N + c] / d;
      if (f == 0.0) continue;
      for (int j = c; j < N; ++j) A[i * N + j] -= f * A[c * N + j];
      r[i] -= f * r[c];
    }
  }
  for (int i = N - 1; i >= 0; --i) {
    zc acc = r[i];
    for (int j = i + 1; j < N; ++j) acc -= A[i * N + j] * r[j];
    r[i] = acc / A[i * N + i];
  }
  r.resize(m);
  return r;
}

// ------------------------------------------------------------------ assembly
// Sum the residual pieces (precision R) with the FP64 driver and diagonal Fock
// part; either take the Jacobi step into (xt, e) with |step|^2 partials, or
// write the full residual into (s1, s2).
template <typename R>
static int assemble(Handle& h, double* xt, double* e, double* s1, double* s2, double shift) {
  Work<R> w = work<R>(h);
  const int o = h.P.o, v = h.P.v;
  const int64_t ov = (int64_t)o * v, np = h.P.Po * h.P.Pv;
  k_assemble_t1<R>(w.S1, h.x, h.eps, o, v, shift, h.op.doubles_only != 0, xt, e, s1,
                   s1 ? nullptr : h.red, h.s);
  int nb = 0;
  if (np > 0) {
    nb = assemble_t2_blocks(np);
    const bool cc2 = h.op.cc2 != 0;
    k_assemble_t2<R>(cc2 ? nullptr : w.Znp, w.Z, cc2 ? nullptr : w.R_, cc2 ? nullptr : h.Voovv_p,
                     h.x + 2 * ov, h.eps, o, v, shift,
                     xt ? xt + 2 * ov : nullptr, e ? e + 2 * ov : nullptr, s2,
                     s2 ? nullptr : h.red + 1, nb, h.s);
  }
  return nb;
}

static void compute_residual_phase(Handle& h) {
  if (h.phase32)
    compute_residual<float>(h);
  else
    compute_residual<double>(h);
}

// Release the graph of one iteration kind (its buffers are about to go, or it will not run
// again).
static void drop_graph(Handle& h, int kind) {
  if (!h.gexec[kind]) return;
  HIPCHECK(hipStreamSynchronize(h.s));
  HIPCHECK(hipGraphExecDestroy(h.gexec[kind]));
  h.gexec[kind] = nullptr;
}

// The residual computation of one iteration.  With opts.graph_residual the first iteration
// of each kind records its kernels into a graph (stream capture: every launch, the
// planner's included, is recorded, not run) and every iteration of that kind then replays
// it with one launch: the same kernels with the same arguments in the same order, so the
// results are bitwise those of the direct launches, without the host's per-kernel launch
// and planning cost.  The captured kernels read and write only the handle's fixed buffers
// (amplitudes, work arrays, stored classes); a kind's graph is released before any of its
// buffers is (the switch, the end of the corrected phase).  The reference iteration of the
// corrected phase runs once and is not captured; timed runs (opts.timing) are not captured.
static void residual_step(Handle& h) {
  const int kind = h.phase32 ? 1 : h.dc == 0 ? 0 : h.dc == 2 ? 2 : -1;
  if (!h.op.graph_residual || h.tm.on || kind < 0) {
    compute_residual_phase(h);
    return;
  }
  if (!h.gexec[kind]) {
    hipGraph_t g = nullptr;
    HIPCHECK(hipStreamBeginCapture(h.s, hipStreamCaptureModeThreadLocal));
    try {
      compute_residual_phase(h);
    } catch (...) {
      hipGraph_t partial = nullptr;
      (void)hipStreamEndCapture(h.s, &partial);
      if (partial) (void)hipGraphDestroy(partial);
      (void)hipGetLastError();
      throw;
    }
    HIPCHECK(hipStreamEndCapture(h.s, &g));
    const hipError_t e = hipGraphInstantiate(&h.gexec[kind], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      h.gexec[kind] = nullptr;
      HIPCHECK(e);
    }
  }
  HIPCHECK(hipGraphLaunch(h.gexec[kind], h.s));
}

// ------------------------------------------------------------------ one iteration
static zc device_energy(Handle& h) {
  Scope sc(h, "energy");
  const int o = h.P.o, v = h.P.v;
  const int64_t np = h.P.Po * h.P.Pv;
  if (np == 0) return 0.0;  // f_ia = 0: no singles term
  const int nb = energy_blocks(np);
  k_energy(h.Voovv_p, h.x + 2 * (int64_t)o * v, h.x, o, v, h.red, nb, h.s);
  k_reduce_sum(h.red, nb, 2, h.redout, h.s);
  HIPCHECK(hipMemcpyAsync(h.host, h.redout, 16, hipMemcpyDeviceToHost, h.s));
  HIPCHECK(hipStreamSynchronize(h.s));
  return zc(h.host[0], h.host[1]);
}

// The assembly wrote (x + e, e) into DIIS slot `slot` and the squared step norm into
// redout[0]: add the Gram row of e against the stored error vectors, drop the oldest
// pairs while the subspace is ill-conditioned, solve for the coefficients and write the
// extrapolated vector to target.  Returns ||e||.
static double diis_commit(Handle& h, int slot, double* target) {
  const int64_t L = h.P.L;
  const int cap = h.P.nslots;
  const double* e = h.slot_e(slot);
  // Gram row of the new error vector against every stored one (and itself)
  std::vector<int> ids = h.order;
  ids.push_back(slot);
  const int m = (int)ids.size();
  if (h.op.diis_size > 0) {
    Scope sc(h, "diis");
    std::vector<const double*> es;
    for (int k : ids) es.push_back(h.slot_e(k));
    const int nb = dot_many_blocks(L);
    k_dot_many(es.data(), m, e, L, h.red + 8192, nb, h.s);
    k_reduce_sum(h.red + 8192, nb, 2 * m, h.redout + 8, h.s);
  }
  HIPCHECK(hipMemcpyAsync(h.host, h.redout, (8 + 2 * m) * sizeof(double), hipMemcpyDeviceToHost, h.s));
  HIPCHECK(hipStreamSynchronize(h.s));
  const double rnorm = std::sqrt(h.host[0]);
  h.order.push_back(slot);
  if ((int)h.G.size() < cap) h.G.assign(cap, std::vector<zc>(cap, 0.0));
  if (h.op.diis_size > 0)
    for (int k = 0; k < m; ++k) {
      const zc g(h.host[8 + 2 * k], h.host[8 + 2 * k + 1]);  // <e_k, e_new>
      h.G[ids[k]][slot] = g;
      h.G[slot][ids[k]] = std::conj(g);
    }
  // coefficients: drop the oldest while the subspace is ill-conditioned
  std::vector<zc> c;
  while (h.op.diis_size > 0 && h.order.size() >= 2) {
    const int mm = (int)h.order.size();
    std::vector<std::vector<zc>> Gm(mm, std::vector<zc>(mm));
    for (int i = 0; i < mm; ++i)
      for (int j = 0; j < mm; ++j) Gm[i][j] = h.G[h.order[i]][h.order[j]];
    const std::vector<double> w = herm_eigvals(Gm);
    if (!(w[0] > 0.0) || w[mm - 1] / w[0] > 1e14) {
      h.order.erase(h.order.begin());
      continue;
    }
    c = diis_solve(Gm);
    break;
  }
  if (c.empty()) c.assign(h.order.size(), 1.0);
  {
    Scope sc(h, "diis");
    std::vector<const double*> xs;
    std::vector<cplx> cc;
    for (size_t k = 0; k < h.order.size(); ++k) {
      xs.push_back(h.slot_x(h.order[k]));
      cc.push_back(cplx{c[k].real(), c[k].imag()});
    }
    k_lincomb(target, xs.data(), cc.data(), (int)xs.size(), L, h.s);
  }
  return rnorm;
}

// Pick the DIIS slot for the next pair (drop the oldest pair when full).
static int diis_slot(Handle& h) {
  const int cap = h.P.nslots;
  if ((int)h.order.size() == cap) h.order.erase(h.order.begin());
  int slot = 0;
  for (; slot < cap; ++slot)
    if (std::find(h.order.begin(), h.order.end(), slot) == h.order.end()) break;
  return slot;
}

// Leave the defect-corrected phase: full FP64 iterations from here on; the reference
// product and the low-precision ladder operands are released.
static void end_defect_correction(Handle& h) {
  HIPCHECK(hipStreamSynchronize(h.s));
  drop_graph(h, 2);
  h.dc = 0;
  h.fp64_iters = 0;
  h.dfree(h.tau_ref);
  h.dfree(h.Zref);
  h.dfree(h.Bvs);
  h.dfree(h.Bt32);
  h.dfree(h.x_ref);
  h.dfree(h.Rref);
  h.dfree(h.Href32);
  h.dfree(h.D32);
  h.dfree(h.Ud);
  h.dfree(h.Vtd);
  h.dfree(h.t1d);
  h.dfree(h.Cref);
  h.dfree(h.Voovv32);
  h.dfree(h.Vvovv_p32);
}

static double one_iteration(Handle& h) {
  const bool was32 = h.phase32;
  const int dc_now = h.dc;
  residual_step(h);
  const int slot = diis_slot(h);
  double* xt = h.slot_x(slot);
  double* e = h.slot_e(slot);
  {
    Scope sc(h, "assemble");
    const int nb = was32 ? assemble<float>(h, xt, e, nullptr, nullptr, h.op.level_shift)
                         : assemble<double>(h, xt, e, nullptr, nullptr, h.op.level_shift);
    k_reduce_sum(h.red, nb + 1, 1, h.redout, h.s);
  }
  const double rnorm = diis_commit(h, slot, h.x);
  h.energy = device_energy(h);
  timer_collect(h);
  h.iters++;
  // precision schedule: low-precision contractions until the step norm falls
  // below the switch threshold or stops improving (no new lowest value for
  // kStall iterations: the rounding floor of the low-precision residual), then
  // FP64 contractions with a fresh DIIS subspace
  // (with the defect-corrected ladder: one FP64 iteration that stores the reference
  // ladder product, corrected iterations until ||Delta|| <= tol or they stall, then full
  // FP64 iterations; the DIIS subspace carries over, the residual being the same to the
  // corrected product's rounding)
  constexpr int kStall = 4;
  h.last32 = was32;
  h.last_dc = dc_now == 2;
  if (!was32 && dc_now != 2) h.fp64_iters++;
  if (was32) {
    if (h.best32 < 0.0 || rnorm < h.best32) {
      h.best32 = rnorm;
      h.since_best32 = 0;
    } else {
      h.since_best32++;
    }
  }
  if (was32 && (rnorm < h.op.mixed_switch_tol || h.since_best32 >= kStall)) {
    const bool dc = h.op.ladder_defect_correction != 0 && !h.op.cc2 && h.P.Po * h.P.Pv > 0;
    drop_graph(h, 1);
    ensure_fp64_classes(h, dc);
    if (dc) {
      h.tau_ref = h.dalloc(h.P.Po * h.P.Pv);
      h.Zref = h.dalloc(h.P.Po * h.P.Pv);
      if (h.P.ring_dc) {
        const int o = h.P.o, v = h.P.v, X = h.P.X;
        h.x_ref = h.dalloc(h.P.L);
        h.Rref = h.dalloc(h.P.oovv);
        h.Href32 = reinterpret_cast<float*>(h.dalloc((h.P.oovv + 1) / 2));
        h.D32 = reinterpret_cast<float*>(h.dalloc((h.P.oovv + 1) / 2));
        h.Ud = h.dalloc((int64_t)o * o * X);
        h.Vtd = h.dalloc((int64_t)v * o * X);
        h.t1d = h.dalloc((int64_t)o * v);
        h.Cref = h.dalloc(h.P.Po * v * o);
      }
      h.dc = 1;
    }
    HIPCHECK(hipStreamSynchronize(h.s));
    timer_collect(h);
    h.phase32 = false;
    h.fp64_iters = 0;
    h.order.clear();
  } else if (dc_now == 1) {
    h.dc = 2;
    h.best_dc = -1.0;
    h.since_best_dc = 0;
  } else if (dc_now == 2) {
    if (h.best_dc < 0.0 || rnorm < h.best_dc) {
      h.best_dc = rnorm;
      h.since_best_dc = 0;
    } else {
      h.since_best_dc++;
    }
    if (rnorm <= h.op.tol || h.since_best_dc >= kStall) end_defect_correction(h);
  }
  return rnorm;
}

static void reset_diis(Handle& h) {
  h.order.clear();
  h.G.clear();
  h.first_norm = -1.0;
}

// ------------------------------------------------------------------ perturbative triples
// E(+T) and E((T)) of App. C at the current amplitudes (FP64).  The excitation
// elements <ab||ie> = (ai|be) - (ae|bi) are built from the DF factors for the occupied i
// of the resident blocks, packed over a<b ([i][(a<b)][e]).  Then for each occupied pair
// j<k and a batch of i<j (the paper's unique triples, batched over i)
//   W[i][a][b][c] = sum_e (<ab||ie> t_jk^ec + <ab||je> t_ki^ec + <ab||ke> t_ij^ec)
//                 + sum_m (<am||ij> t_km^bc + <am||jk> t_im^bc + <am||ki> t_jm^bc)
// (<am||xy> = -conj(<xy||ma>) from the stored ooov class).  The sum over e is
// antisymmetric in (a, b) and the sum over m in (b, c), so the two parts are formed
// packed, We[i][(a<b)][c] and Wm[i][a][(b<c)]: half the o^3 v^4 and o^4 v^3 work of the
// full W, in six GETTs.  The energy kernel forms the cyclic sums W~, Z~, Y~ from the two
// packed parts and the three energy terms of each triple, reduced in a fixed order.  The
// host sums the triples in order: E = (1/6) sum_{i<j<k} sum_{abc} (the (1/36) sum over
// all ijk, abc).
static void triples_impl(Handle& h, double* e4_out, double* e5_out, double* ey_out) {
  if (h.phase32)
    raise(EXACC_ERR_INVALID_ARG,
          "triples need FP64 integrals: the handle is still in its low-precision phase");
  const int o = h.P.o, v = h.P.v, X = h.P.X;
  *e4_out = 0.0;
  *e5_out = 0.0;
  *ey_out = 0.0;
  if (o < 3 || v < 3) return;
  if (h.op.triples_occ_block < 0) raise(EXACC_ERR_INVALID_ARG, "triples_occ_block < 0");
  const hipStream_t s = h.s;
  const int64_t vv = (int64_t)v * v, ooo = (int64_t)o * o * o, Pv = h.P.Pv, pvv = Pv * v;
  const int nblk = triples_blocks(v);
  size_t free_b = 0, total_b = 0;
  HIPCHECK(hipMemGetInfo(&free_b, &total_b));
  const size_t small = (size_t)(2 * ooo + 2 * (int64_t)(o - 2) * nblk + 4) * 16 + (256u << 20);
  const size_t trow = (size_t)pvv * 16;   // packed tile of one occupied i
  const size_t wrow = 2 * trow;           // We and Wm of one triple
  // occupied block size n_red: all of nocc when its tiles fit beside one W row, else the
  // largest with three blocks of tiles resident (or the requested size)
  int red = o;
  if (small + (size_t)o * trow + wrow > free_b) {
    if (small + 3 * trow + wrow > free_b)
      raise(EXACC_ERR_NOMEM, "triples: three <ab||ie> tile rows and one W row do not fit in free device memory");
    red = (int)std::min<int64_t>(o, (int64_t)((free_b - small - wrow) / (3 * trow)));
  }
  if (h.op.triples_occ_block > 0) red = std::min(red, h.op.triples_occ_block);
  const int nb_occ = (o + red - 1) / red;
  const int slots = nb_occ == 1 ? 1 : 3;
  const size_t tiles = (size_t)slots * red * trow;
  if (small + tiles + wrow > free_b)
    raise(EXACC_ERR_NOMEM, "triples: the <ab||ie> tiles of three occupied blocks do not fit; lower triples_occ_block");
  // W rows (one per triple of a batch): what fits beside the tiles, at most n_red
  const int64_t cap = std::max<int64_t>(
      1, std::min<int64_t>(std::min(red, o - 2), (int64_t)((free_b - small - tiles) / 2 / wrow)));
  h.use();
  check_budget(h, tiles + (size_t)cap * wrow + (size_t)(4 * cap * nblk + 4 * ooo) * 8 +
                     (size_t)cap * v * 2 * o * 16,
               "triples temporaries");
  double *Ve = nullptr, *We = nullptr, *Wm = nullptr, *part = nullptr, *tri = nullptr, *Acat = nullptr;
  struct Free {  // released on every exit, a failed allocation included
    Handle& h;
    double** p[6];
    ~Free() {
      for (auto q : p) try {
          h.dfree(*q);
        } catch (...) {
        }
    }
  } fr{h, {&Ve, &We, &Wm, &part, &tri, &Acat}};
  Ve = h.dalloc((int64_t)slots * red * pvv);
  We = h.dalloc(cap * pvv);
  Wm = h.dalloc(cap * pvv);
  part = h.dalloc(2 * cap * nblk);  // 4 doubles per block
  tri = h.dalloc(2 * ooo);          // (e4, e5, ey, -) at [i][j][k]
  Acat = h.dalloc(cap * v * 2 * o);
  // full t2 [i][j][a][b] into H4 and t2 packed over the virtual pair [k][m][(b<c)] into
  // TAU (FP64 work arrays rebuilt every iteration)
  k_unpack_full(h.x, h.x + 2 * (int64_t)o * v, nullptr, h.H4, o, v, s);
  double* T2 = h.H4;
  double* T2pv = h.TAU;
  k_pack_last2<double>(T2pv, T2, nullptr, (int64_t)o * o, v, vv, s);
  Views<double> b = bviews(h, h.Bt);
  const int64_t nX = (int64_t)h.P.n * X;
  // tiles <ab||ie> = (ai|be) - (ae|bi), a<b, of occupied block q into slot sl,
  // [i][(a<b)][e]: per a, the rows b > a; e contiguous, so the W GETTs read both operands
  // along K
  int held[3] = {-1, -1, -1};
  auto build = [&](int q, int sl) {
    if (held[sl] == q) return;
    const int i0 = q * red, ni = std::min(red, o - i0);
    double* tq = Ve + 2 * (int64_t)sl * red * pvv;
    for (int a = 0; a + 1 < v; ++a) {
      const int nb = v - a - 1;
      const int64_t off = (int64_t)a * v - (int64_t)a * (a + 1) / 2;  // first pair (a, a+1)
      auto Cv = sview(tq + 2 * off * v, {ni, nb, v}, {pvv, (int64_t)v, 1});
      auto Bvo_a = sview(b.Bvo.p + 2 * ((int64_t)a * nX + (int64_t)i0 * X), {ni, X}, {X, 1});
      auto Bvv_b = sview(b.Bvv.p + 2 * (int64_t)(a + 1) * nX, {nb, v, X}, {nX, X, 1});
      contract(s, "beP,iP->ibe", ONE, Bvv_b, Bvo_a, false, Cv);
      auto Bvv_a = sview(b.Bvv.p + 2 * (int64_t)a * nX, {v, X}, {X, 1});
      auto Bvo_b = sview(b.Bvo.p + 2 * ((int64_t)(a + 1) * nX + (int64_t)i0 * X), {nb, ni, X}, {nX, X, 1});
      contract(s, "eP,biP->ibe", MONE, Bvv_a, Bvo_b, true, Cv);
    }
    held[sl] = q;
  };
  int slot_of[3] = {0, 0, 0};  // slot holding the tiles of the current K, J, I blocks
  auto tile = [&](int i, int which) {
    return Ve + 2 * ((int64_t)slot_of[which] * red + (i - (i / red) * red)) * pvv;
  };
  const int64_t ovv = (int64_t)o * vv, oov = (int64_t)o * o * v, ov = (int64_t)o * v, opv = (int64_t)o * Pv;
  // t_jk^{ce} as [c][e] (e contiguous); t_jk^{ec} = -t_jk^{ce}
  auto Tpair = [&](int j, int k) { return sview(T2 + 2 * ((int64_t)j * o + k) * vv, {v, v}, {(int64_t)v, 1}); };
  // three nested loops over occupied blocks, unique block triples bi <= bj <= bk
  for (int bk = 0; bk < nb_occ; ++bk)
    for (int bj = 0; bj <= bk; ++bj)
      for (int bi = 0; bi <= bj; ++bi) {
        if (slots == 1) {
          build(0, 0);
        } else {
          build(bk, 0);
          slot_of[0] = 0;
          if (bj == bk) {
            slot_of[1] = 0;
          } else {
            build(bj, 1);
            slot_of[1] = 1;
          }
          if (bi == bk) {
            slot_of[2] = 0;
          } else if (bi == bj) {
            slot_of[2] = slot_of[1];
          } else {
            build(bi, 2);
            slot_of[2] = 2;
          }
        }
        const int k_lo = std::max(bk * red, 2), k_hi = std::min(o, (bk + 1) * red);
        for (int k = k_lo; k < k_hi; ++k) {
          const int j_hi = std::min(k, std::min(o, (bj + 1) * red));
          for (int j = std::max(bj * red, 1); j < j_hi; ++j) {
            const int i_hi = std::min(j, std::min(o, (bi + 1) * red));
            for (int i0 = bi * red; i0 < i_hi; i0 += (int)cap) {
              const int ni = (int)std::min<int64_t>(cap, i_hi - i0);
              auto Wev = view(We, {ni, Pv, v});
              auto Wmv = view(Wm, {ni, v, Pv});
              auto Vt3 = [&](double* p) { return sview(p, {Pv, v}, {(int64_t)v, 1}); };
              // sum_e <ab||ie> t_jk^ec = -sum_e <ab||ie> t_jk^ce, i over the batch
              contract(s, "ixe,ce->ixc", MONE, sview(tile(i0, 2), {ni, Pv, v}, {pvv, (int64_t)v, 1}),
                       Tpair(j, k), false, Wev);
              // sum_e <ab||je> t_ki^ec, t_ki^ce = T2[k][i][c][e]
              contract(s, "xe,ice->ixc", MONE, Vt3(tile(j, 1)),
                       sview(T2 + 2 * ((int64_t)k * o + i0) * vv, {ni, v, v}, {vv, (int64_t)v, 1}), true, Wev);
              // sum_e <ab||ke> t_ij^ec, t_ij^ce = T2[i][j][c][e]
              contract(s, "xe,ice->ixc", MONE, Vt3(tile(k, 0)),
                       sview(T2 + 2 * ((int64_t)i0 * o + j) * vv, {ni, v, v}, {ovv, (int64_t)v, 1}), true, Wev);
              // sum_m <am||ki> t_jm^bc + sum_m <am||ij> t_km^bc (b<c) as one product over
              // K = (t, m), 2 nocc: the two excitation elements gathered into Acat[i][a][t][m],
              // t_jm and t_km read as T2pv[j + t (k - j)]
              k_triples_acat(h.Vooov, i0, ni, j, k, o, v, Acat, s);
              contract(s, "iatm,tmy->iay", MONE, view(Acat, {ni, v, 2, o}),
                       sview(T2pv + 2 * (int64_t)j * opv, {2, o, Pv}, {(int64_t)(k - j) * opv, Pv, 1}),
                       false, Wmv);
              // sum_m <am||jk> t_im^bc
              contract(s, "ma,imy->iay", MONE,
                       conj(sview(h.Vooov + 2 * ((int64_t)j * o + k) * ov, {o, v}, {(int64_t)v, 1})),
                       sview(T2pv + 2 * (int64_t)i0 * opv, {ni, o, Pv}, {opv, Pv, 1}), true, Wmv);
              k_triples_energy(We, Wm, h.Voovv, T2, h.x, h.eps, i0, ni, j, k, o, v, part, nblk, tri, s);
            }
          }
        }
      }
  std::vector<double> host(4 * ooo);
  HIPCHECK(hipMemcpyAsync(host.data(), tri, host.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHECK(hipStreamSynchronize(s));
  double e4 = 0, e5 = 0, ey = 0;
  for (int i = 0; i < o; ++i)
    for (int j = i + 1; j < o; ++j)
      for (int k = j + 1; k < o; ++k) {
        const int64_t q = ((int64_t)i * o + j) * o + k;
        e4 += host[4 * q];
        e5 += host[4 * q + 1];
        ey += host[4 * q + 2];
      }
  *e4_out = e4 / 6.0;
  *e5_out = (e4 + e5) / 6.0;
  *ey_out = (e4 + ey) / 6.0;
}

// ------------------------------------------------------------------ create
// ------------------------------------------------------------------ Lambda equations
// App. D: the left-hand (Lambda) equations at converged amplitudes, FP64.  The
// intermediates are the one- and two-body elements of e^-T H e^T, built once per
// amplitude set (lambda_prepare); each Lambda iteration then forms R1, R2 from them,
// with the expensive pieces taken through the DF factors instead of stored whole:
//   * the particle ladder 1/2 sum_ef l_ij^ef W_efab, with W_efab = sum_P (Bd_ae Bd_bf -
//     Bd_af Bd_be) + 1/2 sum_mn t_mn^ef <mn||ab> and the T1-dressed factor
//     Bd[a][e][P] = B^P_ea - sum_m t_m^e B^P_ma: the amplitude ladder's tile builder run
//     on Bd, plus two packed o^4 v^2 GEMMs;
//   * 1/2 sum_mef l_im^ef W_efam (the vvvo element) term by term: <ef||am> through
//     (ea|fm), the W_vvvv part as t1 times the ladder product above, and the t2 part
//     through the ring-shaped Z1[i][n][f][g] = sum_me l_im^ef t_nm^eg;
//   * the vovv element through its definition <ej||ab> - sum_n t_n^e <nj||ab>.
// The diagonal Fock part of R is left to the assembly (D times lambda), as for the
// amplitudes, so F_vv and F_oo here exclude it.
static void lambda_invalidate(Handle& h) { h.lam.prepared = false; }

static void lambda_alloc(Handle& h) {
  if (h.lam.lam) return;
  const int64_t o = h.P.o, v = h.P.v, X = h.P.X;
  const int64_t need = h.P.L + 3 * o * v + 2 * h.P.oovv + v * v * X + 3 * o * o * o * v +
                       h.P.Po * h.P.Po + o * o * X + X + (o + v) * (o + v);
  size_t fr = 0, tot = 0;
  HIPCHECK(hipMemGetInfo(&fr, &tot));
  if ((size_t)need * 16 + (256u << 20) > fr) raise(EXACC_ERR_NOMEM, "Lambda buffers do not fit");
  check_budget(h, (size_t)need * 16, "Lambda buffers");
  // into a local set first: the handle records them only once every allocation succeeded;
  // on a failed allocation the ones already made are released before the error propagates
  Handle::Lam L;
  struct Undo {
    Handle& h;
    Handle::Lam& L;
    bool armed = true;
    ~Undo() {
      if (!armed) return;
      for (double** q : {&L.l1w, &L.s1, &L.gt, &L.Lq, &L.Z1, &L.Bd, &L.Wooov, &L.O3a, &L.O3b, &L.LTp,
                         &L.Q1, &L.gP, &L.gam, &L.lam})
        try {
          h.dfree(*q);
        } catch (...) {
        }
    }
  } undo{h, L};
  L.l1w = h.dalloc(o * v);
  L.s1 = h.dalloc(o * v);
  L.gt = h.dalloc(o * v);
  L.Lq = h.dalloc(h.P.oovv);
  L.Z1 = h.dalloc(h.P.oovv);
  L.Bd = h.dalloc(v * v * X);
  L.Wooov = h.dalloc(o * o * o * v);
  L.O3a = h.dalloc(o * o * o * v);
  L.O3b = h.dalloc(o * o * o * v);
  L.LTp = h.dalloc(h.P.Po * h.P.Po);
  L.Q1 = h.dalloc(o * o * X);
  L.gP = h.dalloc(X);
  L.gam = h.dalloc((o + v) * (o + v));
  L.lam = h.dalloc(h.P.L);
  dzero(h, L.lam, h.P.L);
  undo.armed = false;
  h.lam = L;
}

static void lambda_check(Handle& h) {
  if (h.phase32)
    raise(EXACC_ERR_INVALID_ARG, "Lambda equations need the FP64 integrals: iterate into the FP64 phase first");
  if (h.op.doubles_only || h.op.cc2)
    raise(EXACC_ERR_INVALID_ARG, "Lambda equations are those of CCSD; not for CCD or CC2 handles");
  h.use();
  lambda_alloc(h);
}

static void lambda_prepare(Handle& h) {
  if (h.lam.prepared) return;
  Work<double> w = work<double>(h);
  const int o = h.P.o, v = h.P.v, X = h.P.X, n = h.P.n;
  const int64_t Po = h.P.Po, ov = (int64_t)o * v, oov = (int64_t)o * o * v;
  const hipStream_t s = h.s;
  Views<double> b = bviews(h, w.Bt);
  Handle::Lam& L = h.lam;
  const double* t1p = h.x;
  const double* t2p = h.x + 2 * ov;
  Scope sc(h, "lambda_prepare");
  dcopy(h, h.t1w, h.x, ov);
  auto t1 = view(h.t1w, {o, v});
  k_unpack_tau<double>(t1p, t2p, w.Z, w.TAU, w.taup, o, v, s);
  k_ring_operands<double>(w.Z, t1p, w.Tq, w.Xp, o, v, s);
  auto T2 = sview(w.Tq, {o, o, v, v}, {ov, v, 1, oov});
  auto TAU = view(w.TAU, {o, o, v, v});
  auto Voovv = view(w.Voovv, {o, o, v, v});
  auto Vooov = view(w.Vooov, {o, o, o, v});
  // one-body: Gac = F_vv, Gki = -F_oo (both without the diagonal Fock part), Hkc = F_ov
  auto Hac = view(w.Hac, {v, v}), Gac = view(w.Gac, {v, v});
  auto Hki = view(w.Hki, {o, o}), Gki = view(w.Gki, {o, o});
  auto Hkc = view(w.Hkc, {o, v});
  contract(s, "klcd,klda->ac", HALF, Voovv, TAU, false, Hac);
  contract(s, "klcd,licd->ki", HALF, Voovv, TAU, false, Hki);
  dcopy(h, w.Gac, w.Hac, (int64_t)v * v);
  dcopy(h, w.Gki, w.Hki, (int64_t)o * o);
  contract(s, "klcd,ld->kc", ONE, Voovv, t1, false, Hkc);
  auto y = view(w.y, {X});
  auto U = view(w.U, {o, o, X});
  auto Vt = view(w.Vt, {v, o, X});
  contract(s, "kdP,kd->P", ONE, b.Bov, t1, false, y);
  contract(s, "kdP,id->kiP", ONE, b.Bov, t1, false, U);
  contract(s, "acP,ic->aiP", ONE, b.Bvv, t1, false, Vt);
  contract(s, "acP,P->ac", ONE, b.Bvv, y, true, Gac);
  contract(s, "akP,kcP->ac", MONE, Vt, b.Bov, true, Gac);
  contract(s, "klic,lc->ki", MONE, Vooov, t1, true, Gki);
  // W_oooo [m][n][i][j] in Af, packed over both pairs into Ap[(mn)][(ij)]
  auto Af = view(w.Af, {o, o, o, o});
  dcopy(h, w.Af, w.Voooo, (int64_t)o * o * o * o);
  contract(s, "klic,jc->klij", ONE, Vooov, t1, true, Af);
  contract(s, "kljc,ic->klij", MONE, Vooov, t1, true, Af);
  contract(s, "klcd,ijcd->klij", HALF, Voovv, TAU, true, Af);
  if (Po > 0) k_pack_last2<double>(w.Ap, w.Af, h.rowmap_o, Po, o, (int64_t)o * o, s);
  // W_ooov [m][n][i][e] = <mn||ie> + sum_f t_i^f <mn||fe>
  auto Wooov = view(L.Wooov, {o, o, o, v});
  dcopy(h, L.Wooov, w.Vooov, (int64_t)o * o * o * v);
  contract(s, "if,mnfe->mnie", ONE, t1, Voovv, true, Wooov);
  // W_ovvo as Wq[b][j][m][e] = W_ovvo[j][e][b][m] = -H'[e][m][j][b], H'[a][i][k][c] the ring
  // intermediate of the amplitude equations with the full t2 in place of t2/2
  auto Wq = sview(w.H4, {v, o, o, v}, {1, v, ov, oov});
  contract(s, "acP,kiP->aikc", MONE, b.Bvv, b.Boo, false, Wq);
  contract(s, "aiP,kcP->aikc", ONE, b.Bvo, b.Bov, true, Wq);
  contract(s, "acP,kiP->aikc", MONE, b.Bvv, U, true, Wq);
  contract(s, "aiP,kcP->aikc", ONE, Vt, b.Bov, true, Wq);
  contract(s, "klic,la->aikc", ONE, Vooov, t1, true, Wq);
  contract(s, "aild,klcd->aikc", MONE, view(w.Xp, {v, o, o, v}), Voovv, true, Wq);
  contract(s, "aild,klcd->aikc", cplx{-0.5, 0}, view(w.Tq, {v, o, o, v}), Voovv, true, Wq);
  // W_ovoo as Cf[i][j][b][m] = W_ovoo[m][b][i][j]
  const int64_t vo = (int64_t)v * o;
  auto Cp = view(w.Cp, {Po, v, o});
  auto taup = view(w.taup, {Po, h.P.Pv});
  if (Po > 0) contract(s, "bkx,px->pbk", MONE, view(w.Vvovv_p, {v, o, h.P.Pv}), taup, false, Cp);
  k_expand_c<double>(w.Vooov, w.Cp, w.Cf, o, v, s);
  auto Cf = view(w.Cf, {o, o, v, o});
  auto Cfji = sview(w.Cf, {o, o, v, o}, {vo, o * vo, o, 1});
  contract(s, "me,ijbe->ijbm", MONE, Hkc, T2, true, Cf);
  contract(s, "nb,mnij->ijbm", MONE, t1, Af, true, Cf);
  contract(s, "mnie,jnbe->ijbm", ONE, Vooov, T2, true, Cf);
  contract(s, "mnie,jnbe->ijbm", MONE, Vooov, T2, true, Cfji);
  contract(s, "miP,bjP->ijbm", ONE, U, b.Bvo, true, Cf);
  contract(s, "mjP,biP->ijbm", MONE, b.Boo, Vt, true, Cf);
  contract(s, "miP,bjP->ijbm", MONE, U, b.Bvo, true, Cfji);
  contract(s, "mjP,biP->ijbm", ONE, b.Boo, Vt, true, Cfji);
  auto Wt = view(L.O3a, {o, o, o, v});
  contract(s, "ie,mnef->mnif", ONE, t1, Voovv, false, Wt);
  contract(s, "mnif,njbf->ijbm", MONE, Wt, T2, true, Cf);
  contract(s, "mnif,njbf->ijbm", ONE, Wt, T2, true, Cfji);
  // dressed factor Bd[a][e][P] = B^P_ea - sum_m t_m^e B^P_ma (B^P_qp = conj(B^P_pq))
  k_conj_rows(L.Bd, b.Bvv.p, v, (int64_t)n * X, (int64_t)v * X, s);
  contract(s, "amP,me->aeP", MONE, conj(b.Bvo), t1, true, view(L.Bd, {v, v, X}));
  L.prepared = true;
}

// R1 into S1 and the pieces of R2 into Z (no permutation), R (P_ij P_ab at assembly)
// and Znp (packed), at the Lambda amplitudes in h.lam.lam.
static void lambda_compute(Handle& h) {
  lambda_prepare(h);
  Work<double> w = work<double>(h);
  const int o = h.P.o, v = h.P.v, X = h.P.X;
  const int64_t Po = h.P.Po, Pv = h.P.Pv, ov = (int64_t)o * v, oov = (int64_t)o * o * v;
  const int64_t vv = (int64_t)v * v, ovv = (int64_t)o * v * v;
  const hipStream_t s = h.s;
  Views<double> b = bviews(h, w.Bt);
  Handle::Lam& L = h.lam;
  Scope sc(h, "lambda_residual");
  const double* l2p = L.lam + 2 * ov;
  dcopy(h, L.l1w, L.lam, ov);
  k_unpack_full(nullptr, l2p, nullptr, w.Z, o, v, s);
  k_ring_operands<double>(w.Z, h.x, L.Lq, w.Xp, o, v, s);  // Lq[b][i][k][a] = l_ik^ab
  auto l1 = view(L.l1w, {o, v});
  auto t1 = view(h.t1w, {o, v});
  auto L2 = sview(L.Lq, {o, o, v, v}, {ov, v, 1, oov});
  auto T2 = sview(w.Tq, {o, o, v, v}, {ov, v, 1, oov});
  auto Voovv = view(w.Voovv, {o, o, v, v});
  auto Vooov = view(w.Vooov, {o, o, o, v});
  auto Gac = view(w.Gac, {v, v}), Gki = view(w.Gki, {o, o}), Hkc = view(w.Hkc, {o, v});
  auto Wooov = view(L.Wooov, {o, o, o, v});
  auto Wq = view(w.H4, {v, o, o, v});
  // G^e_a and G^i_m of App. D: Gv[a][e] = -1/2 sum t_mn^ef l_mn^af, Go[m][i] = 1/2 sum t_mn^ef l_in^ef
  auto Gv = view(w.Hac, {v, v}), Go = view(w.Hki, {o, o});
  contract(s, "mnef,mnaf->ae", cplx{-0.5, 0}, T2, L2, false, Gv);
  contract(s, "mnef,inef->mi", HALF, T2, L2, false, Go);

  // ---- R2, pieces without a permutation operator (Z and its swapped views)
  auto Z = view(w.Z, {o, o, v, v});
  auto Zji = sview(w.Z, {o, o, v, v}, {vv, ovv, v, 1});
  auto Zba = sview(w.Z, {o, o, v, v}, {ovv, vv, 1, v});
  dcopy(h, w.Z, w.Voovv, h.P.oovv);  // <ij||ab>
  contract(s, "ijae,eb->ijab", ONE, L2, Gac, true, Z);
  contract(s, "ijae,eb->ijab", MONE, L2, Gac, true, Zba);
  contract(s, "imab,jm->ijab", ONE, L2, Gki, true, Z);
  contract(s, "imab,jm->ijab", MONE, L2, Gki, true, Zji);
  auto M1 = view(w.M1, {o, o});
  contract(s, "ie,ne->in", ONE, l1, t1, false, M1);
  contract(s, "in,njab->ijab", MONE, M1, Voovv, true, Z);
  contract(s, "in,njab->ijab", ONE, M1, Voovv, true, Zji);
  contract(s, "ma,ijmb->ijab", MONE, l1, Wooov, true, Z);
  contract(s, "ma,ijmb->ijab", ONE, l1, Wooov, true, Zba);
  contract(s, "ijae,be->ijab", ONE, Voovv, Gv, true, Z);
  contract(s, "ijae,be->ijab", MONE, Voovv, Gv, true, Zba);
  contract(s, "imab,mj->ijab", MONE, Voovv, Go, true, Z);
  contract(s, "imab,mj->ijab", ONE, Voovv, Go, true, Zji);
  // ---- R2, pieces under P_ij P_ab (R)
  auto Rv = view(w.R_, {o, o, v, v});
  contract(s, "aime,bjme->ijab", MONE, view(L.Lq, {v, o, o, v}), Wq, false, Rv, GETT_RING);
  auto Yv = view(w.Y, {o, v, X});
  contract(s, "ie,aeP->iaP", ONE, l1, conj(b.Bvv), false, Yv);
  contract(s, "iaP,jbP->ijab", ONE, Yv, b.Bov, true, Rv);
  contract(s, "iaz,jbz->ijab", ONE, sview(L.l1w, {o, v, 1}, {v, 1, 1}), sview(w.Hkc, {o, v, 1}, {v, 1, 1}),
           true, Rv);
  // ---- R2, packed pieces (Znp): first the W_vvvv ladder alone, which R1 also needs
  auto Znp = view(w.Znp, {Po, Pv});
  auto l2v = view(const_cast<double*>(l2p), {Po, Pv});
  if (Po > 0 && Pv > 0) {
    auto LT = view(L.LTp, {Po, Po});
    contract(s, "py,qy->pq", ONE, l2v, view(h.x + 2 * ov, {Po, Pv}), false, LT);
    contract(s, "pq,qx->px", ONE, LT, view(h.Voovv_p, {Po, Pv}), false, Znp);
    ladder_apply<double>(h, w, L.Bd, (int64_t)v * X, l2v, w.Znp, false, false, false);
  }
  // ---- R1
  auto S1 = view(w.S1, {o, v});
  dcopy(h, w.S1, w.Hkc, ov);
  if (Po > 0 && Pv > 0) {  // sum_mg t_m^g (1/2 sum_ef l_im^ef W_efag)
    k_unpack_full(nullptr, w.Znp, nullptr, L.Z1, o, v, s);
    contract(s, "imag,mg->ia", ONE, view(L.Z1, {o, o, v, v}), t1, true, S1);
    contract(s, "pq,qx->px", ONE, view(w.Ap, {Po, Po}), l2v, true, Znp);  // 1/2 l_mn^ab W_ijmn
  }
  contract(s, "ie,ea->ia", ONE, l1, Gac, true, S1);
  contract(s, "ma,im->ia", ONE, l1, Gki, true, S1);
  contract(s, "me,aime->ia", ONE, l1, Wq, true, S1);
  // 1/2 sum l_im^ef <ef||am> = sum_mef l_im^ef (ea|fm)
  contract(s, "imef,fmP->ieP", ONE, L2, b.Bvo, false, Yv);
  contract(s, "ieP,aeP->ia", ONE, Yv, conj(b.Bvv), true, S1);
  contract(s, "ni,na->ia", MONE, Go, Hkc, true, S1);
  // 1/4 sum_{mno} (sum_ef l_im^ef tau_no^ef) <no||am>
  auto LTo = view(w.Af, {o, o, o, o});
  contract(s, "imef,noef->imno", ONE, L2, view(w.TAU, {o, o, v, v}), false, LTo);
  contract(s, "imno,noma->ia", cplx{-0.25, 0}, LTo, Vooov, true, S1);
  // - sum_{nfg} Z1[i][n][f][g] <nf||ag>, Z1 = sum_me l_im^ef t_nm^eg
  auto Z1 = view(L.Z1, {o, o, v, v});
  contract(s, "fime,gnme->infg", ONE, view(L.Lq, {v, o, o, v}), view(w.Tq, {v, o, o, v}), false, Z1,
           GETT_RING);
  auto Q1 = view(L.Q1, {o, o, X});
  contract(s, "infg,fgP->inP", ONE, Z1, b.Bvv, false, Q1);
  contract(s, "inP,naP->ia", MONE, Q1, b.Bov, true, S1);
  contract(s, "infg,ngP->ifP", ONE, Z1, b.Bov, false, Yv);
  contract(s, "ifP,faP->ia", ONE, Yv, b.Bvv, true, S1);
  // - sum Lt[i][m][n][f] (<nf||am> - sum_og t_om^fg <no||ag>), Lt = sum_e l_im^ef t_n^e
  auto Lt = view(L.O3a, {o, o, o, v});
  contract(s, "imef,ne->imnf", ONE, L2, t1, false, Lt);
  contract(s, "imnf,fmP->inP", ONE, Lt, b.Bvo, false, Q1);
  contract(s, "inP,naP->ia", MONE, Q1, b.Bov, true, S1);
  contract(s, "imnf,nmP->ifP", ONE, Lt, b.Boo, false, Yv);
  contract(s, "ifP,faP->ia", ONE, Yv, b.Bvv, true, S1);
  auto M2 = view(L.O3b, {o, o, o, v});
  contract(s, "imnf,omfg->inog", ONE, Lt, T2, false, M2);
  contract(s, "inog,noag->ia", ONE, M2, Voovv, true, S1);
  // - 1/2 sum l_mn^ae W_iemn (W_ovoo in Cf[m][n][e][i])
  contract(s, "mnae,mnei->ia", cplx{-0.5, 0}, L2, view(w.Cf, {o, o, v, o}), true, S1);
  // - sum_ef G_ef W_eifa, W_eifa = <ei||fa> - sum_n t_n^e <ni||fa>
  auto gP = view(L.gP, {X});
  contract(s, "efP,ef->P", ONE, b.Bvv, Gv, false, gP);
  contract(s, "iaP,P->ia", MONE, b.Bov, gP, true, S1);
  contract(s, "ef,ifP->ieP", ONE, Gv, b.Bov, false, Yv);
  contract(s, "ieP,aeP->ia", ONE, Yv, conj(b.Bvv), true, S1);
  auto gt = view(L.gt, {o, v});
  contract(s, "ef,ne->nf", ONE, Gv, t1, false, gt);
  contract(s, "nf,nifa->ia", ONE, gt, Voovv, true, S1);
  contract(s, "mn,mina->ia", MONE, Go, Wooov, true, S1);
}

// Assembly of R + D lambda: the Jacobi step into (xt, e), or the full residual into (s1, s2).
static int lambda_assemble(Handle& h, double* xt, double* e, double* s1, double* s2) {
  Work<double> w = work<double>(h);
  const int o = h.P.o, v = h.P.v;
  const int64_t ov = (int64_t)o * v, np = h.P.Po * h.P.Pv;
  k_assemble_t1<double>(w.S1, h.lam.lam, h.eps, o, v, 0.0, 0, xt, e, s1, s1 ? nullptr : h.red, h.s);
  int nb = 0;
  if (np > 0) {
    nb = assemble_t2_blocks(np);
    k_assemble_t2<double>(w.Znp, w.Z, w.R_, nullptr, h.lam.lam + 2 * ov, h.eps, o, v, 0.0,
                          xt ? xt + 2 * ov : nullptr, e ? e + 2 * ov : nullptr, s2,
                          s2 ? nullptr : h.red + 1, nb, h.s);
  }
  return nb;
}

static double lambda_iteration(Handle& h) {
  if (h.diis_owner != 1) {
    reset_diis(h);
    h.diis_owner = 1;
  }
  lambda_compute(h);
  const int slot = diis_slot(h);
  {
    Scope sc(h, "assemble");
    const int nb = lambda_assemble(h, h.slot_x(slot), h.slot_e(slot), nullptr, nullptr);
    k_reduce_sum(h.red, nb + 1, 1, h.redout, h.s);
  }
  const double r = diis_commit(h, slot, h.lam.lam);
  timer_collect(h);
  return r;
}

// The one-body density of App. E at the current t and lambda into gamma_dev [n][n].
static void lambda_density(Handle& h, double* gamma_dev) {
  lambda_prepare(h);
  Work<double> w = work<double>(h);
  const int o = h.P.o, v = h.P.v;
  const int64_t ov = (int64_t)o * v, oov = (int64_t)o * o * v;
  const hipStream_t s = h.s;
  Handle::Lam& L = h.lam;
  dcopy(h, L.l1w, L.lam, ov);
  k_unpack_full(nullptr, L.lam + 2 * ov, nullptr, w.Z, o, v, s);
  k_ring_operands<double>(w.Z, h.x, L.Lq, w.Xp, o, v, s);
  auto l1 = view(L.l1w, {o, v});
  auto t1 = view(h.t1w, {o, v});
  auto L2 = sview(L.Lq, {o, o, v, v}, {ov, v, 1, oov});
  auto T2 = sview(w.Tq, {o, o, v, v}, {ov, v, 1, oov});
  auto Gv = view(w.Hac, {v, v}), Go = view(w.Hki, {o, o});
  contract(s, "mnef,mnaf->ae", cplx{-0.5, 0}, T2, L2, false, Gv);
  contract(s, "mnef,inef->mi", HALF, T2, L2, false, Go);
  auto M = view(w.M1, {o, o});
  contract(s, "me,ie->im", ONE, l1, t1, false, M);
  auto Dvo = view(L.gt, {o, v});
  dcopy(h, L.gt, h.t1w, ov);
  contract(s, "me,imae->ia", ONE, l1, T2, true, Dvo);
  contract(s, "im,ma->ia", MONE, M, t1, true, Dvo);
  contract(s, "im,ma->ia", MONE, Go, t1, true, Dvo);
  contract(s, "ie,ea->ia", ONE, t1, Gv, true, Dvo);
  auto N = view(L.Z1, {v, v});
  contract(s, "ma,mb->ab", ONE, t1, l1, false, N);
  k_lambda_density(w.Hki, w.M1, L.l1w, L.gt, w.Hac, L.Z1, o, v, gamma_dev, s);
}

static void validate_host_inputs(int o, int v, const double* eps) {
  double emax = -1e300, emin = 1e300;
  for (int i = 0; i < o + v; ++i)
    if (!std::isfinite(eps[i])) raise(EXACC_ERR_INVALID_ARG, "non-finite spinor energy");
  for (int i = 0; i < o; ++i) emax = std::max(emax, eps[i]);
  for (int a = 0; a < v; ++a) emin = std::min(emin, eps[o + a]);
  if (!(emin - emax > 1e-8)) raise(EXACC_ERR_INVALID_ARG, "no gap between occupied and virtual energies");
}

static Handle* create_impl(int o, int v, int X, const double* eps, const double* B,
                           const exacc_ccsd_opts& op) {
  if (o < 1 || v < 1 || X < 1) raise(EXACC_ERR_INVALID_ARG, "nocc, nvir and naux must be >= 1");
  if (!eps || !B) raise(EXACC_ERR_INVALID_ARG, "null input pointer");
  if ((int64_t)o * o > 65535) raise(EXACC_ERR_INVALID_ARG, "nocc too large (nocc^2 > 65535)");
  if (op.precision != EXACC_FP64 && op.precision != EXACC_MIXED_FP32 &&
      op.precision != EXACC_MIXED_BF16X3)
    raise(EXACC_ERR_UNSUPPORTED, "unknown precision mode");
  if (op.diis_size < 0 || op.diis_size > 16) raise(EXACC_ERR_INVALID_ARG, "diis_size must be 0..16");
  if (op.doubles_only != 0 && op.doubles_only != 1) raise(EXACC_ERR_INVALID_ARG, "doubles_only must be 0 or 1");
  if (op.cc2 != 0 && op.cc2 != 1) raise(EXACC_ERR_INVALID_ARG, "cc2 must be 0 or 1");
  if (op.cc2 && op.doubles_only) raise(EXACC_ERR_INVALID_ARG, "cc2 and doubles_only are exclusive");
  if (!(op.tol >= 0) || !std::isfinite(op.level_shift))
    raise(EXACC_ERR_INVALID_ARG, "bad tol or level_shift");
  exacc_ccsd_opts opx = op;
  Plan P = make_plan(o, v, X, opx);
  if (opx.precision != EXACC_FP64 && opx.ladder_defect_correction) {
    // the defect correction's reference arrays only where they fit in the device memory
    // (4 GiB kept free): first without the ring part, then without any
    size_t fr = 0, tot = 0;
    HIPCHECK(hipMemGetInfo(&fr, &tot));
    const size_t keep = (size_t)4 << 30;
    if (P.ring_dc && P.bytes_peak + keep > tot) {
      P.ring_dc = false;
      P.bytes_peak = P.bytes_peak_no_ring_dc;
    }
    if (P.bytes_peak + keep > tot) {
      opx.ladder_defect_correction = 0;
      P = make_plan(o, v, X, opx);
    }
  }
  if (op.hbm_budget_bytes && P.bytes_peak > op.hbm_budget_bytes)
    raise(EXACC_ERR_NOMEM, "memory plan exceeds hbm_budget_bytes");
  Handle* h = new Handle();
  try {
    h->P = P;
    h->op = opx;
    h->tm.on = op.timing != 0;
    if (op.stream) {
      h->s = (hipStream_t)op.stream;
    } else {
      HIPCHECK(hipStreamCreateWithFlags(&h->s, hipStreamNonBlocking));
      h->own_stream = true;
    }
    const int n = o + v;
    const int64_t nnX = (int64_t)n * n * X;
    HIPCHECK(hipHostMalloc((void**)&h->host, 4096 * sizeof(double), hipHostMallocDefault));
    // eps: validate on the host
    std::vector<double> eh(n);
    if (op.inputs_on_device)
      HIPCHECK(hipMemcpy(eh.data(), eps, n * sizeof(double), hipMemcpyDeviceToHost));
    else
      std::memcpy(eh.data(), eps, n * sizeof(double));
    validate_host_inputs(o, v, eh.data());
    h->eps = (double*)h->dalloc((n + 1) / 2);
    HIPCHECK(hipMemcpyAsync(h->eps, eh.data(), n * sizeof(double), hipMemcpyHostToDevice, h->s));
    h->red = h->dalloc(65536);
    h->ws_bytes = (size_t)256 << 20;
    h->ws = h->dalloc((int64_t)(h->ws_bytes / 16));
    h->redout = h->dalloc(64);
    // B: stage raw, check Hermiticity and finiteness on the device, transpose to [p][q][P]
    const double* Braw = B;
    double* Bstage = nullptr;
    if (!op.inputs_on_device) {
      HIPCHECK(hipMalloc((void**)&Bstage, nnX * 16));
      HIPCHECK(hipMemcpyAsync(Bstage, B, nnX * 16, hipMemcpyHostToDevice, h->s));
      Braw = Bstage;
    }
    struct Free {
      double* p;
      ~Free() {
        if (p) (void)hipFree(p);
      }
    } fb{Bstage};
    k_check_B(Braw, X, n, h->redout, h->red, h->s);
    HIPCHECK(hipMemcpyAsync(h->host, h->redout, 3 * sizeof(double), hipMemcpyDeviceToHost, h->s));
    HIPCHECK(hipStreamSynchronize(h->s));
    if (h->host[2] != 0.0) raise(EXACC_ERR_INVALID_ARG, "non-finite entries in B");
    if (h->host[0] > 1e-12 * std::max(h->host[1], 1e-300))
      raise(EXACC_ERR_INVALID_ARG, "B[P] is not Hermitian");
    h->Bt = h->dalloc(nnX);
    k_transpose_B(Braw, h->Bt, X, (int64_t)n * n, h->s);
    HIPCHECK(hipStreamSynchronize(h->s));
    if (Bstage) {
      HIPCHECK(hipFree(Bstage));
      fb.p = nullptr;
    }
    const int64_t oo = (int64_t)o * o;
    {
      std::vector<int> rm;
      for (int k = 0; k < o; ++k)
        for (int l = k + 1; l < o; ++l) rm.push_back(k * o + l);
      void* p = nullptr;
      HIPCHECK(hipMalloc(&p, std::max<size_t>(1, rm.size()) * sizeof(int)));
      h->allocs.push_back(p);
      h->rowmap_o = (int*)p;
      if (!rm.empty())
        HIPCHECK(hipMemcpyAsync(h->rowmap_o, rm.data(), rm.size() * sizeof(int), hipMemcpyHostToDevice,
                                h->s));
    }
    // ---- stored integral classes, before the work arrays (lower create-time peak)
    {
      Scope sc(*h, "integrals");
      h->use();
      h->Voooo = h->dalloc(oo * oo);
      h->Vooov = h->dalloc(oo * o * v);
      build_oooo_ooov(*h);
      h->Voovv_p = h->dalloc(P.Po * P.Pv);
      h->Voovv = h->dalloc(P.oovv);
      build_oovv(*h, h->Voovv);
      if (P.Po > 0) k_pack_last2<double>(h->Voovv_p, h->Voovv, h->rowmap_o, P.Po, v, P.vv, h->s);
      if (op.precision == EXACC_FP64) {
        h->Vvovv_p = h->dalloc((int64_t)v * o * P.Pv);
        build_vovv_packed<double>(*h, h->Vvovv_p);
      } else {
        // low-precision phase: FP32 copies only; the FP64 classes are rebuilt at the switch
        auto mk32 = [&](const double* src64, int64_t celems) {
          float* p = reinterpret_cast<float*>(h->dalloc((celems + 1) / 2));
          k_cast(src64, p, 2 * celems, h->s);
          return p;
        };
        h->Bt32 = mk32(h->Bt, nnX);
        if (op.precision == EXACC_MIXED_BF16X3 && v > 1) {
          // rows (a, c) of the vv block: a at stride n*X, c at stride X
          h->Bvs = reinterpret_cast<unsigned short*>(h->dalloc(P.vv * bf16x3_split_k(X) / 2));
          split_rows_bf16x3(h->Bt32 + 2 * ((int64_t)o * n + o) * X, P.vv, v, (int64_t)n * X, X, X,
                            h->Bvs, h->s);
        }
        h->Voooo32 = mk32(h->Voooo, oo * oo);
        h->Vooov32 = mk32(h->Vooov, oo * o * v);
        h->Voovv_p32 = mk32(h->Voovv_p, P.Po * P.Pv);
        {
          // [k][c][l][d] layout for the FP32 copy (contiguous (l, d) for the ring build)
          Views<double> b = bviews(*h, h->Bt);
          auto Vperm = sview(h->Voovv, {o, o, v, v}, {(int64_t)o * v * v, (int64_t)v, (int64_t)o * v, 1});
          contract(h->s, "kcP,ldP->klcd", ONE, b.Bov, b.Bov, false, Vperm);
          contract(h->s, "kdP,lcP->klcd", MONE, b.Bov, b.Bov, true, Vperm);
          h->Voovv32 = mk32(h->Voovv, P.oovv);
        }
        HIPCHECK(hipStreamSynchronize(h->s));
        h->dfree(h->Voovv);
        h->Vvovv_p32 = reinterpret_cast<float*>(h->dalloc(((int64_t)v * o * P.Pv + 1) / 2));
        build_vovv_packed<float>(*h, h->Vvovv_p32);
        h->phase32 = true;
      }
      HIPCHECK(hipStreamSynchronize(h->s));
    }
    // ---- amplitudes, DIIS and work arrays
    h->x = h->dalloc(P.L);
    h->diis = h->dalloc(2 * P.nslots * P.L);
    h->TAU = h->dalloc(P.oovv);
    h->taup = h->dalloc(P.Po * P.Pv);
    h->Tq = h->dalloc(P.oovv);
    h->Xp = h->dalloc(P.oovv);
    h->H4 = h->dalloc(P.oovv);
    h->Z = h->dalloc(P.oovv);
    h->Znp = h->dalloc(P.Po * P.Pv);
    h->Hac = h->dalloc(P.vv);
    h->Gac = h->dalloc(P.vv);
    h->Hki = h->dalloc(oo);
    h->Gki = h->dalloc(oo);
    h->M1 = h->dalloc(oo);
    h->Hkc = h->dalloc((int64_t)o * v);
    h->S1 = h->dalloc((int64_t)o * v);
    h->t1w = h->dalloc((int64_t)o * v);
    h->y = h->dalloc(X);
    h->U = h->dalloc(oo * X);
    h->Vt = h->dalloc((int64_t)v * o * X);
    h->Y = h->dalloc((int64_t)o * v * X);
    h->Cp = h->dalloc(P.Po * v * o);
    h->Cf = h->dalloc(oo * v * o);
    h->Af = h->dalloc(oo * oo);
    h->Ap = h->dalloc(P.Po * P.Po);
    h->Ta = h->dalloc(h->P.ladder_grouped ? h->P.vv * h->P.vv : (int64_t)v * std::max(1, v - 1) * v);
    h->W = h->dalloc(P.chunk_pairs * std::max<int64_t>(1, P.Pv));
    h->use();
    HIPCHECK(hipMemsetAsync(h->x, 0, P.L * 16, h->s));
    HIPCHECK(hipStreamSynchronize(h->s));
    timer_collect(*h);
    return h;
  } catch (...) {
    if (h->s) (void)hipStreamSynchronize(h->s);
    set_alloc_registry(nullptr, 0);
    set_gett_workspace(nullptr, 0);
    delete h;
    throw;
  }
}

}  // namespace exacc

// ====================================================================== C ABI
using namespace exacc;

template <typename F>
static int guarded(F&& f) {
  try {
    g_last_error.clear();
    return f();
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.status;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return EXACC_ERR_NOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return EXACC_ERR_DEVICE;
  }
}

extern "C" {

void exacc_ccsd_default_opts(exacc_ccsd_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->precision = EXACC_FP64;
  o->diis_size = 8;
  o->max_iter = 30;
  o->tol = 1e-9;
  o->level_shift = 0.0;
  o->fp64_final_iters = 3;
  o->doubles_only = 0;
  o->cc2 = 0;
  o->mixed_switch_tol = 1e-5;
  o->ladder_defect_correction = 1;
  o->graph_residual = 0;
  o->ladder_group_nvir = 64;
}

size_t exacc_ccsd_memory_estimate(int nocc, int nvir, int naux, const exacc_ccsd_opts* opts) {
  if (nocc < 1 || nvir < 1 || naux < 1) return 0;
  exacc_ccsd_opts d;
  exacc_ccsd_default_opts(&d);
  return make_plan(nocc, nvir, naux, opts ? *opts : d).bytes_peak;
}

int exacc_ccsd_create(exacc_ccsd_t* out, int nocc, int nvir, int naux, const double* eps,
                      const double* B, const exacc_ccsd_opts* opts) {
  if (out) *out = nullptr;
  return guarded([&] {
    if (!out) raise(EXACC_ERR_INVALID_ARG, "null handle pointer");
    exacc_ccsd_opts d;
    exacc_ccsd_default_opts(&d);
    Handle* h = create_impl(nocc, nvir, naux, eps, B, opts ? *opts : d);
    *out = reinterpret_cast<exacc_ccsd_t>(h);
    return EXACC_OK;
  });
}

int exacc_ccsd_iterate(exacc_ccsd_t hh, int max_steps, int* steps_done, double* residual,
                       int* converged) {
  if (steps_done) *steps_done = 0;
  if (converged) *converged = 0;
  return guarded([&] {
    if (!hh) raise(EXACC_ERR_INVALID_ARG, "null handle");
    Handle& h = *reinterpret_cast<Handle*>(hh);
    h.use();
    lambda_invalidate(h);
    if (h.diis_owner != 0) {
      reset_diis(h);
      h.diis_owner = 0;
    }
    for (int k = 0; k < max_steps; ++k) {
      const double r = one_iteration(h);
      if (steps_done) *steps_done = k + 1;
      if (residual) *residual = r;
      if (h.first_norm < 0) h.first_norm = r;
      if (!std::isfinite(r) || !std::isfinite(h.energy.real()) || !std::isfinite(h.energy.imag()) ||
          r > 1e6 * std::max(h.first_norm, 1e-300))
        return (int)EXACC_ERR_DIVERGED;
      const int need = h.op.precision == EXACC_FP64 ? 0 : h.op.fp64_final_iters;
      if (r <= h.op.tol && !h.last32 && !h.last_dc && h.fp64_iters >= need) {
        if (converged) *converged = 1;
        return (int)EXACC_OK;
      }
    }
    return (int)EXACC_NOT_CONVERGED;
  });
}

int exacc_ccsd_energy(exacc_ccsd_t hh, double* e_re, double* e_im) {
  return guarded([&] {
    if (!hh) raise(EXACC_ERR_INVALID_ARG, "null handle");
    Handle& h = *reinterpret_cast<Handle*>(hh);
    h.use();
    const zc e = device_energy(h);
    timer_collect(h);
    if (e_re) *e_re = e.real();
    if (e_im) *e_im = e.imag();
    return (int)EXACC_OK;
  });
}

int exacc_ccsd_get_amplitudes(exacc_ccsd_t hh, double* t1, double* t2, int on_device) {
  return guarded([&] {
    if (!hh) raise(EXACC_ERR_INVALID_ARG, "null handle");
    Handle& h = *reinterpret_cast<Handle*>(hh);
    h.use();
    lambda_invalidate(h);
    const int o = h.P.o, v = h.P.v;
    const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (t1) HIPCHECK(hipMemcpyAsync(t1, h.x, (size_t)o * v * 16, k, h.s));
    if (t2) {
      k_unpack_full(h.x, h.x + 2 * (int64_t)o * v, nullptr, h.Tq, o, v, h.s);
      HIPCHECK(hipMemcpyAsync(t2, h.Tq, (size_t)h.P.oovv * 16, k, h.s));
    }
    HIPCHECK(hipStreamSynchronize(h.s));
    return (int)EXACC_OK;
  });
}

int exacc_ccsd_set_amplitudes(exacc_ccsd_t hh, const double* t1, const double* t2, int on_device) {
  return guarded([&] {
    if (!hh) raise(EXACC_ERR_INVALID_ARG, "null handle");
    Handle& h = *reinterpret_cast<Handle*>(hh);
    h.use();
    lambda_invalidate(h);
    const int o = h.P.o, v = h.P.v;
    const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (t1)
      HIPCHECK(hipMemcpyAsync(h.x, t1, (size_t)o * v * 16, k, h.s));
    else
      HIPCHECK(hipMemsetAsync(h.x, 0, (size_t)o * v * 16, h.s));
    if (t2) {
      HIPCHECK(hipMemcpyAsync(h.Tq, t2, (size_t)h.P.oovv * 16, k, h.s));
      k_pack_amplitudes(nullptr, h.Tq, h.x + 2 * (int64_t)o * v, o, v, h.s);
    } else if (h.P.Po * h.P.Pv > 0) {
      HIPCHECK(hipMemsetAsync(h.x + 2 * (int64_t)o * v, 0, (size_t)h.P.Po * h.P.Pv * 16, h.s));
    }
    HIPCHECK(hipStreamSynchronize(h.s));
    reset_diis(h);
    if (h.dc == 2) h.dc = 1;  // the corrected ladder takes a new reference point
    return (int)EXACC_OK;
  });
}

int exacc_ccsd_residual(exacc_ccsd_t hh, double* s1, double* s2, int on_device) {
  return guarded([&] {
    if (!hh) raise(EXACC_ERR_INVALID_ARG, "null handle");
    Handle& h = *reinterpret_cast<Handle*>(hh);
    h.use();
    lambda_invalidate(h);
    const int o = h.P.o, v = h.P.v;
    compute_residual_phase(h);
    const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    // full residual into Tq (FP64 buffer; its contents are rebuilt each iteration) and S1
    // into the t1w buffer, both unused by the assembly
    HIPCHECK(hipMemsetAsync(h.Tq, 0, (size_t)h.P.oovv * 16, h.s));
    if (h.phase32)
      assemble<float>(h, nullptr, nullptr, h.t1w, h.Tq, 0.0);
    else
      assemble<double>(h, nullptr, nullptr, h.t1w, h.Tq, 0.0);
    if (s1) HIPCHECK(hipMemcpyAsync(s1, h.t1w, (size_t)o * v * 16, k, h.s));
    if (s2) HIPCHECK(hipMemcpyAsync(s2, h.Tq, (size_t)h.P.oovv * 16, k, h.s));
    HIPCHECK(hipStreamSynchronize(h.s));
    timer_collect(h);
    return (int)EXACC_OK;
  });
}

int exacc_ccsd_triples(exacc_ccsd_t hh, double* e_plus_t, double* e_paren_t, double* e_minus_t) {
  return guarded([&] {
    if (!hh) raise(EXACC_ERR_INVALID_ARG, "null handle");
    Handle& h = *reinterpret_cast<Handle*>(hh);
    h.use();
    lambda_invalidate(h);
    double e4 = 0, e5 = 0, ey = 0;
    triples_impl(h, &e4, &e5, &ey);
    if (e_plus_t) *e_plus_t = e4;
    if (e_paren_t) *e_paren_t = e5;
    if (e_minus_t) *e_minus_t = ey;
    return (int)EXACC_OK;
  });
}

int exacc_ccsd_lambda_iterate(exacc_ccsd_t hh, int max_steps, int* steps_done, double* residual,
                              int* converged) {
  if (steps_done) *steps_done = 0;
  if (converged) *converged = 0;
  return guarded([&] {
    if (!hh) raise(EXACC_ERR_INVALID_ARG, "null handle");
    Handle& h = *reinterpret_cast<Handle*>(hh);
    lambda_check(h);
    double first = -1.0;
    for (int k = 0; k < max_steps; ++k) {
      const double r = lambda_iteration(h);
      if (steps_done) *steps_done = k + 1;
      if (residual) *residual = r;
      if (first < 0) first = r;
      if (!std::isfinite(r) || r > 1e6 * std::max(first, 1e-300)) return (int)EXACC_ERR_DIVERGED;
      if (r <= h.op.tol) {
        if (converged) *converged = 1;
        return (int)EXACC_OK;
      }
    }
    return (int)EXACC_NOT_CONVERGED;
  });
}

int exacc_ccsd_lambda_residual(exacc_ccsd_t hh, double* r1, double* r2, int on_device) {
  return guarded([&] {
    if (!hh) raise(EXACC_ERR_INVALID_ARG, "null handle");
    Handle& h = *reinterpret_cast<Handle*>(hh);
    lambda_check(h);
    const int o = h.P.o, v = h.P.v;
    lambda_compute(h);
    // full residual into Z1 and R1 into the s1 buffer, both unused by the assembly
    dzero(h, h.lam.Z1, h.P.oovv);
    lambda_assemble(h, nullptr, nullptr, h.lam.s1, h.lam.Z1);
    const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (r1) HIPCHECK(hipMemcpyAsync(r1, h.lam.s1, (size_t)o * v * 16, k, h.s));
    if (r2) HIPCHECK(hipMemcpyAsync(r2, h.lam.Z1, (size_t)h.P.oovv * 16, k, h.s));
    HIPCHECK(hipStreamSynchronize(h.s));
    timer_collect(h);
    return (int)EXACC_OK;
  });
}

int exacc_ccsd_get_lambda(exacc_ccsd_t hh, double* l1, double* l2, int on_device) {
  return guarded([&] {
    if (!hh) raise(EXACC_ERR_INVALID_ARG, "null handle");
    Handle& h = *reinterpret_cast<Handle*>(hh);
    lambda_check(h);
    const int o = h.P.o, v = h.P.v;
    const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (l1) HIPCHECK(hipMemcpyAsync(l1, h.lam.lam, (size_t)o * v * 16, k, h.s));
    if (l2) {
      k_unpack_full(nullptr, h.lam.lam + 2 * (int64_t)o * v, nullptr, h.lam.Z1, o, v, h.s);
      HIPCHECK(hipMemcpyAsync(l2, h.lam.Z1, (size_t)h.P.oovv * 16, k, h.s));
    }
    HIPCHECK(hipStreamSynchronize(h.s));
    return (int)EXACC_OK;
  });
}

int exacc_ccsd_set_lambda(exacc_ccsd_t hh, const double* l1, const double* l2, int on_device) {
  return guarded([&] {
    if (!hh) raise(EXACC_ERR_INVALID_ARG, "null handle");
    Handle& h = *reinterpret_cast<Handle*>(hh);
    lambda_check(h);
    const int o = h.P.o, v = h.P.v;
    const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (l1)
      HIPCHECK(hipMemcpyAsync(h.lam.lam, l1, (size_t)o * v * 16, k, h.s));
    else
      dzero(h, h.lam.lam, (int64_t)o * v);
    if (l2) {
      HIPCHECK(hipMemcpyAsync(h.lam.Z1, l2, (size_t)h.P.oovv * 16, k, h.s));
      k_pack_amplitudes(nullptr, h.lam.Z1, h.lam.lam + 2 * (int64_t)o * v, o, v, h.s);
    } else {
      dzero(h, h.lam.lam + 2 * (int64_t)o * v, h.P.Po * h.P.Pv);
    }
    HIPCHECK(hipStreamSynchronize(h.s));
    if (h.diis_owner == 1) reset_diis(h);
    return (int)EXACC_OK;
  });
}

int exacc_ccsd_density(exacc_ccsd_t hh, double* gamma, int on_device) {
  return guarded([&] {
    if (!hh) raise(EXACC_ERR_INVALID_ARG, "null handle");
    if (!gamma) raise(EXACC_ERR_INVALID_ARG, "null output");
    Handle& h = *reinterpret_cast<Handle*>(hh);
    lambda_check(h);
    const int64_t n = h.P.n;
    double* g = on_device ? gamma : h.lam.gam;
    lambda_density(h, g);
    if (!on_device) HIPCHECK(hipMemcpyAsync(gamma, g, (size_t)n * n * 16, hipMemcpyDeviceToHost, h.s));
    HIPCHECK(hipStreamSynchronize(h.s));
    timer_collect(h);
    return (int)EXACC_OK;
  });
}

int exacc_df_factors(int nao, int nspinor, int naux, const double* C, const double* J, const double* V,
                     double* B, int ptrs_on_device, void* stream, int* ns_iterations) {
  return guarded([&] {
    if (nao < 1 || nspinor < 1 || naux < 1 || nspinor > nao)
      raise(EXACC_ERR_INVALID_ARG, "DF factors: need 1 <= nspinor <= nao and naux >= 1");
    if (!C || !J || !V || !B) raise(EXACC_ERR_INVALID_ARG, "DF factors: null pointer");
    if ((int64_t)naux * nao * nao > 0x7fffffffLL || (int64_t)naux * nspinor * nspinor > 0x7fffffffLL ||
        (int64_t)naux * naux > 0x7fffffffLL)
      raise(EXACC_ERR_INVALID_ARG, "DF factors: extent beyond 2^31");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    bool own = false;
    if (!s) {
      HIPCHECK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      own = true;
    }
    struct StreamGuard {
      hipStream_t s;
      bool own;
      ~StreamGuard() {
        if (own) (void)hipStreamDestroy(s);
      }
    } sg{s, own};
    const int it = df_factors_impl(nao, nspinor, naux, C, J, V, B, ptrs_on_device != 0, s);
    if (ns_iterations) *ns_iterations = it;
    return (int)EXACC_OK;
  });
}

int exacc_df_factors_noalloc(int nao, int nspinor, int naux, const double* C, const double* J,
                             const double* V, double* B, void* stream, int* ns_iterations) {
  return guarded([&] {
    if (nao < 1 || nspinor < 1 || naux < 1 || nspinor > nao)
      raise(EXACC_ERR_INVALID_ARG, "DF factors: need 1 <= nspinor <= nao and naux >= 1");
    if (!C || !J || !V || !B) raise(EXACC_ERR_INVALID_ARG, "DF factors: null pointer");
    if ((int64_t)naux * nao * nao > 0x7fffffffLL || (int64_t)naux * nspinor * nspinor > 0x7fffffffLL ||
        (int64_t)naux * naux > 0x7fffffffLL)
      raise(EXACC_ERR_INVALID_ARG, "DF factors: extent beyond 2^31");
    const int it = df_factors_noalloc_impl(nao, nspinor, naux, C, J, V, B,
                                           reinterpret_cast<hipStream_t>(stream));
    if (ns_iterations) *ns_iterations = it;
    return (int)EXACC_OK;
  });
}

int exacc_ccsd_stage_times(exacc_ccsd_t hh, const char** names, double* ms, int* count, int reset) {
  return guarded([&] {
    if (!hh || !count) raise(EXACC_ERR_INVALID_ARG, "null argument");
    Handle& h = *reinterpret_cast<Handle*>(hh);
    const int cap = *count;
    const int nn = (int)h.tm.names.size();
    for (int i = 0; i < nn && i < cap; ++i) {
      if (names) names[i] = h.tm.names[i].c_str();
      if (ms) ms[i] = h.tm.ms[i];
    }
    *count = nn;
    if (reset)
      for (auto& x : h.tm.ms) x = 0.0;
    return (int)EXACC_OK;
  });
}

int exacc_ccsd_phase(exacc_ccsd_t hh, int* fp32, int* fp64_iters) {
  return guarded([&] {
    if (!hh) raise(EXACC_ERR_INVALID_ARG, "null handle");
    Handle& h = *reinterpret_cast<Handle*>(hh);
    if (fp32) *fp32 = h.phase32 ? 1 : (h.dc == 2 ? 2 : 0);
    if (fp64_iters) *fp64_iters = h.fp64_iters;
    return (int)EXACC_OK;
  });
}

double exacc_ladder_flops(int nocc, int nvir, int naux) {
  const double Po = 0.5 * nocc * (nocc - 1.0), Pv = 0.5 * nvir * (nvir - 1.0);
  // sum_{m=1}^{nvir} m^2 (m - 1) = (nvir (nvir + 1) / 2)^2 - nvir (nvir + 1) (2 nvir + 1) / 6
  const double v = nvir, s3 = 0.25 * v * v * (v + 1) * (v + 1), s2 = v * (v + 1) * (2 * v + 1) / 6.0;
  return 8.0 * (naux * (s3 - s2) + Po * Pv * Pv);
}

int exacc_ccsd_destroy(exacc_ccsd_t hh) {
  if (!hh) return EXACC_OK;
  return guarded([&] {
    Handle* h = reinterpret_cast<Handle*>(hh);
    if (h->s) (void)hipStreamSynchronize(h->s);
    set_alloc_registry(nullptr, 0);
    set_gett_workspace(nullptr, 0);
    delete h;
    return (int)EXACC_OK;
  });
}

const char* exacc_status_string(int st) {
  switch (st) {
    case EXACC_OK: return "ok";
    case EXACC_NOT_CONVERGED: return "not converged";
    case EXACC_ERR_INVALID_ARG: return "invalid argument";
    case EXACC_ERR_NOMEM: return "out of device memory or over budget";
    case EXACC_ERR_DEVICE: return "device error";
    case EXACC_ERR_DIVERGED: return "diverged";
    case EXACC_ERR_UNSUPPORTED: return "unsupported option";
    default: return "unknown status";
  }
}

const char* exacc_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
