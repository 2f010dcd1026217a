// Host driver of the NNCP hot path and its C ABI (include/nncp.h).
//
// One outer iteration (Algorithm 1) is, for n = 1..N:
//   node op   -- the tree node whose lowest mode is n: the root partial MTTKRP
//                of n's half (n = 1 or n = s+1) or a leading multi-TTV from the
//                parent node (Section IV-A; node {a..b} splits into {a} | {a+1..b});
//   leaf op   -- a trailing multi-TTV to M^(n), unless the node is the leaf;
//   update    -- HALS or MU on the rows of the factor (Section II-B);
//   finalize  -- Gram, column norms lambda, the next mode's S, and after mode N
//                the fit (Section IV-B, appendix algorithm).
// The whole iteration is captured once into a HIP graph and replayed.
//
// During the iteration the factor buffers hold the unnormalised result of each
// mode's last update, and lam[n] holds its column norms; every consumer scales
// by 1/lam (Khatri-Rao operands, multi-TTV vectors, normalised Grams), so the
// arithmetic equals that of the normalised algorithm. nncp_plan_finish writes
// the normalised factors back.
#include <algorithm>
#include <cmath>
#include <atomic>
#include <chrono>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "nncp_internal.hpp"

using namespace nncpk;

namespace {

#define HIPCHK(x)                                 \
  do {                                            \
    hipError_t e_ = (x);                          \
    if (e_ != hipSuccess) {                       \
      nncpk::note_device_error((int)e_, __LINE__); \
      return NNCP_EDEVICE;                        \
    }                                             \
  } while (0)

constexpr int kFitCap = 1024;

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

inline Sink sink_of(hipStream_t st) {
  Sink s;
  s.st = st;
  return s;
}

// A node {a..b} of the dimension tree (modes 0-based, inclusive) and how it is
// computed: a root branch from the tensor, or from its parent by contracting
// the parent's last modes (it is the parent's left child) or its first modes
// (the right child).
enum TreeKind : int { T_PM_LEFT = 0, T_PM_RIGHT = 1, T_TRAIL = 2, T_LEAD = 3 };
struct TNode {
  int a = 0, b = 0;
  int parent = -1;
  int kind = T_PM_LEFT;
  int64_t rows = 0;     // product of I_a..I_b
  int has_buf = 0;      // a temporary in the workspace (every node except the leaves below a root)
  size_t off = 0;       // its offset
};

struct Layout {
  size_t off_zeros, off_alpha, off_iter, off_counters, off_lam, off_lammodel, off_lamin, off_G, off_S, off_fit,
      off_finpart, off_pmpart, off_hpack, off_sctab, off_nspart, off_M, total;
  int ncounters;
  int node_f64;  // tree temporaries are FP64 for FP32 tensors, FP32 for 16-bit tensors
  // the tree: nodes, and per mode the nodes computed just before its update
  // (top-down; the last one is the leaf {n}, whose MTTKRP goes to M unless the
  // leaf is a root branch itself)
  int ntn;
  TNode tn[2 * kMaxModes];
  int nsched[kMaxModes];
  int sched[kMaxModes][kMaxModes];
  PmLaunch pmL[2];
  // without the dimension tree (ablation): per mode, the side and split of the
  // partial MTTKRP that computes it from X, and two temporaries
  int dside[kMaxModes], dsplit[kMaxModes];
  PmLaunch dpm[kMaxModes];
  size_t off_dtA, off_dtB;
  int ns_blocks;
};

struct Problem {
  int N = 0, R = 0, dtype = 0, s = 0, update = 0, wg_kib = 0, no_tree = 0, sweeps = 1;
  double inner_tol = 0.0;
  uint64_t peel = 0;  // internal splits: bit a*8+b peels the last mode of node {a..b}
  int64_t dims[kMaxModes] = {};
  int64_t IL = 0, IR = 0, I = 0;
};

int validate(const Problem& p) {
  if (p.N < 2 || p.N > kMaxModes) return NNCP_EINVAL;
  if (p.R < 1 || p.R > kMaxRank) return NNCP_EINVAL;
  if (p.dtype != NNCP_F32 && p.dtype != NNCP_BF16 && p.dtype != NNCP_F16) return NNCP_EINVAL;
  if (p.update != NNCP_HALS && p.update != NNCP_MU) return NNCP_EINVAL;
  if (p.s < 1 || p.s > p.N - 1) return NNCP_EINVAL;
  for (int k = 0; k < p.N; ++k)
    if (p.dims[k] < 1 || p.dims[k] > (int64_t)INT32_MAX) return NNCP_EINVAL;
  // every matricisation used by the kernels indexes its reduction with 32 bits
  if (p.IL > (int64_t)UINT32_MAX || p.IR > (int64_t)UINT32_MAX) return NNCP_EINVAL;
  return NNCP_OK;
}

int fill_problem(Problem& p, int N, const int64_t* dims, int R, int dtype, int update, int split) {
  if (!dims || N < 2 || N > kMaxModes) return NNCP_EINVAL;
  p.N = N;
  p.R = R;
  p.dtype = dtype;
  p.update = update;
  long double prodL = 1, total = 1;
  for (int k = 0; k < N; ++k) {
    p.dims[k] = dims[k];
    if (dims[k] < 1) return NNCP_EINVAL;
    total *= (long double)dims[k];
  }
  if (total > 9.0e18L) return NNCP_EINVAL;
  if (split <= 0) {
    // root split minimising I_L + I_R (smallest tree temporaries)
    long double best = -1;
    int bs = 1;
    for (int s = 1; s < N; ++s) {
      long double L = 1, Rr = 1;
      for (int k = 0; k < s; ++k) L *= dims[k];
      for (int k = s; k < N; ++k) Rr *= dims[k];
      if (best < 0 || L + Rr < best) {
        best = L + Rr;
        bs = s;
      }
    }
    p.s = bs;
  } else {
    p.s = split;
  }
  if (p.s < 1 || p.s > N - 1) return NNCP_EINVAL;
  for (int k = 0; k < p.s; ++k) prodL *= dims[k];
  p.IL = (int64_t)prodL;
  p.IR = (int64_t)(total / prodL);
  p.I = (int64_t)total;
  return validate(p);
}

int64_t prod_range(const Problem& p, int a, int b) {
  int64_t r = 1;
  for (int k = a; k <= b; ++k) r *= p.dims[k];
  return r;
}


// Split point c of the internal node {a..b}: children {a..c} and {c+1..b}. The
// paper allows any binary tree over contiguous mode ranges (Section IV-A); its
// N = 5 example peels the first mode ({3,4,5} -> {3} | {4,5}), the default
// here; bit a*8+b of `peel` peels the last mode instead ({a..b-1} | {b}).
inline int tree_split(const Problem& p, int a, int b) { return ((p.peel >> (a * 8 + b)) & 1ull) ? b - 1 : a; }

int add_tnode(const Problem& p, Layout& L, int a, int b, int parent) {
  const int i = L.ntn++;
  TNode& t = L.tn[i];
  t.a = a;
  t.b = b;
  t.parent = parent;
  if (parent < 0) t.kind = a == 0 ? T_PM_LEFT : T_PM_RIGHT;
  else t.kind = a == L.tn[parent].a ? T_TRAIL : T_LEAD;
  t.rows = prod_range(p, a, b);
  t.has_buf = (a < b || parent < 0) ? 1 : 0;
  if (a < b) {
    const int c = tree_split(p, a, b);
    add_tnode(p, L, a, c, i);
    add_tnode(p, L, c + 1, b, i);
  }
  return i;
}

// The two root branches {0..s-1} and {s..N-1}, and each mode's schedule: the
// nodes on the path from its root branch to its leaf whose lowest mode is n,
// top-down. Such a node is computed just before mode n is updated, from its
// parent (computed at that time or earlier): modes below it are then new and
// modes above it old, which is what the direct MTTKRP of each of its leaves
// sees, so the tree gives the direct MTTKRP exactly.
void build_tree(const Problem& p, Layout& L) {
  L.ntn = 0;
  const int root[2] = {add_tnode(p, L, 0, p.s - 1, -1), add_tnode(p, L, p.s, p.N - 1, -1)};
  for (int n = 0; n < p.N; ++n) {
    L.nsched[n] = 0;
    int i = root[n < p.s ? 0 : 1];
    while (true) {
      const TNode& t = L.tn[i];
      if (t.a == n) L.sched[n][L.nsched[n]++] = i;
      if (t.a == t.b) break;
      // the child that holds n
      int next = -1;
      for (int k = 0; k < L.ntn; ++k)
        if (L.tn[k].parent == i && L.tn[k].a <= n && n <= L.tn[k].b) next = k;
      i = next;
    }
  }
}

Layout make_layout(const Problem& p) {
  Layout L{};
  const int N = p.N, R = p.R, RR = R * R;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  L.pmL[0] = pm_plan(0, p.dtype, p.IL, p.IR, (int)p.dims[p.s], R, p.wg_kib);
  L.pmL[1] = pm_plan(1, p.dtype, p.IL, p.IR, (int)p.dims[0], R, p.wg_kib);
  int maxchunks = 1;
  for (int k = 0; k < N; ++k) {
    int rpc;
    maxchunks = std::max(maxchunks, finalize_chunks(p.dims[k], R, &rpc));
  }
  L.ns_blocks = norm_sq_blocks(p.I);
  L.ncounters = std::max(L.pmL[0].ncounters, L.pmL[1].ncounters) + 4;
  L.off_zeros = take(256);
  L.off_alpha = take(sizeof(double));
  L.off_iter = take(sizeof(int));
  L.off_counters = take(sizeof(unsigned) * L.ncounters);
  L.off_lam = take(sizeof(double) * N * R);
  L.off_lammodel = take(sizeof(double) * R);
  L.off_lamin = take(sizeof(double) * R);
  L.off_G = take(sizeof(double) * N * RR);
  L.off_S = take(sizeof(double) * N * RR);
  L.off_fit = take(sizeof(double) * kFitCap);
  L.off_finpart = take(sizeof(double) * (size_t)maxchunks * (RR + 1));
  L.off_pmpart = take(sizeof(double) * std::max(L.pmL[0].partial_doubles, L.pmL[1].partial_doubles));
  L.off_hpack = take(std::max(L.pmL[0].pack_bytes, L.pmL[1].pack_bytes));
  // the scale table of a partial MTTKRP (the largest root launch)
  size_t tab = std::max(pm_sctab_doubles(L.pmL[0]), pm_sctab_doubles(L.pmL[1]));
  L.off_sctab = take(sizeof(double) * tab);
  L.off_nspart = take(sizeof(double) * L.ns_blocks);
  int64_t maxI = 0;
  for (int k = 0; k < N; ++k) maxI = std::max(maxI, p.dims[k]);
  L.off_M = take(sizeof(double) * (size_t)maxI * R);
  L.node_f64 = p.dtype == NNCP_F32 ? 1 : 0;
  build_tree(p, L);
  for (int i = 0; i < L.ntn; ++i)
    if (L.tn[i].has_buf) L.tn[i].off = take((size_t)L.tn[i].rows * R * (L.node_f64 ? 8 : 4));
  L.off_dtA = L.off_dtB = 0;
  if (p.no_tree) {
    // mode n from X directly: left with split n+1 (temporary over modes 1..n, then
    // leading multi-TTVs down to mode n) or right with split n (temporary over
    // modes n..N, then one trailing multi-TTV), whichever temporary is smaller
    int64_t tmax = 1;
    size_t part = 0, pack = 0;
    for (int n = 0; n < N; ++n) {
      const int64_t tl = n <= N - 2 ? prod_range(p, 0, n) : INT64_MAX;
      const int64_t tr = n >= 1 ? prod_range(p, n, N - 1) : INT64_MAX;
      const int side = tl <= tr ? 0 : 1;
      const int s = side == 0 ? n + 1 : n;
      L.dside[n] = side;
      L.dsplit[n] = s;
      const int64_t IL = prod_range(p, 0, s - 1), IR = p.I / IL;
      L.dpm[n] = pm_plan(side, p.dtype, IL, IR, (int)(side == 0 ? p.dims[s] : p.dims[0]), R, p.wg_kib);
      tmax = std::max(tmax, side == 0 ? tl : tr);
      part = std::max(part, L.dpm[n].partial_doubles);
      pack = std::max(pack, L.dpm[n].pack_bytes);
      if (pm_sctab_doubles(L.dpm[n]) > tab) {
        tab = pm_sctab_doubles(L.dpm[n]);
        L.off_sctab = take(sizeof(double) * tab);  // relocated to fit the no-tree launches too
      }
    }
    const size_t tb = (size_t)tmax * R * (L.node_f64 ? 8 : 4);
    L.off_dtA = take(tb);
    L.off_dtB = take(tb);
    if (part > std::max(L.pmL[0].partial_doubles, L.pmL[1].partial_doubles) ||
        pack > std::max(L.pmL[0].pack_bytes, L.pmL[1].pack_bytes)) {
      // relocate the partial and pack regions to fit the no-tree launches too
      L.off_pmpart = take(sizeof(double) * std::max(part, std::max(L.pmL[0].partial_doubles,
                                                                    L.pmL[1].partial_doubles)));
      L.off_hpack = take(std::max(pack, std::max(L.pmL[0].pack_bytes, L.pmL[1].pack_bytes)));
    }
  }
  L.total = o + 256;
  return L;
}

}  // namespace

// ---------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------
struct nncp_plan {
  Problem p;
  Layout L;
  const void* X = nullptr;
  float* H[kMaxModes] = {};
  char* ws = nullptr;
  bool own_ws = false;
  hipStream_t user_stream = nullptr;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool use_graph = true;
  bool phase_timers = false;
  bool record_fit = true;
  double tol = 0.0;
  double phase_ms[6] = {};
  hipEvent_t ev[2] = {nullptr, nullptr};

  template <typename T>
  T* at(size_t off) const { return (T*)(ws + off); }
  unsigned* zeros() const { return at<unsigned>(L.off_zeros); }
  double* alpha() const { return at<double>(L.off_alpha); }
  int* iter() const { return at<int>(L.off_iter); }
  unsigned* counters() const { return at<unsigned>(L.off_counters); }
  double* lam() const { return at<double>(L.off_lam); }
  double* lam_model() const { return at<double>(L.off_lammodel); }
  double* lam_in() const { return at<double>(L.off_lamin); }
  double* G() const { return at<double>(L.off_G); }
  double* S() const { return at<double>(L.off_S); }
  double* fit() const { return at<double>(L.off_fit); }
  double* finpart() const { return at<double>(L.off_finpart); }
  double* pmpart() const { return at<double>(L.off_pmpart); }
  // 16-bit tensors: 64 column scales, then the packed hi/lo first factor
  float* hscale() const { return at<float>(L.off_hpack); }
  unsigned short* hpack() const { return at<unsigned short>(L.off_hpack + 256); }
  double* sctab() const { return at<double>(L.off_sctab); }
  void* dtA() const { return (void*)(ws + L.off_dtA); }
  void* dtB() const { return (void*)(ws + L.off_dtB); }
  double* nspart() const { return at<double>(L.off_nspart); }
  double* Mbuf() const { return at<double>(L.off_M); }
  void* tbuf(int i) const { return (void*)(ws + L.tn[i].off); }
};

namespace {

KrpDesc krp_for(const nncp_plan* P, int a, int b, bool scaled) {
  KrpDesc k{};
  k.nm = b - a + 1;
  for (int j = 0; j < k.nm; ++j) {
    k.f[j] = P->H[a + j];
    k.dim[j] = (int)P->p.dims[a + j];
    k.mode[j] = a + j;
  }
  k.lam = scaled ? P->lam() : nullptr;
  k.lam_ld = P->p.R;
  return k;
}

// Partial MTTKRP of X split after mode s (0-based: rows are modes 0..s-1) on
// `side`, with launch plan lp for the first column chunk, into T.
hipError_t run_pm_at(const nncp_plan* P, int side, int s, const PmLaunch& lp, void* T, int t_f64, const void* X,
                     bool scaled, const Sink& st) {
  const Problem& p = P->p;
  const int I1 = (int)(side == 0 ? p.dims[s] : p.dims[0]);
  const int64_t IL = prod_range(p, 0, s - 1), IR = p.I / IL;
  for (int c0 = 0; c0 < p.R; c0 += kPmMaxCols) {
    PmArgs a{};
    a.X = X;
    a.IL = IL;
    a.IR = IR;
    a.krp = side == 0 ? krp_for(P, s, p.N - 1, scaled) : krp_for(P, 0, s - 1, scaled);
    a.R = std::min(kPmMaxCols, p.R - c0);
    a.col0 = c0;
    a.T = T;
    a.t_f64 = t_f64;
    a.partial = P->pmpart();
    a.hpack = P->hpack();
    a.hscale = P->hscale();
    a.sctab = P->sctab();
    a.zeros = P->zeros();
    a.counters = P->counters();
    const PmLaunch l = (a.R == std::min(kPmMaxCols, p.R)) ? lp : pm_plan(side, p.dtype, IL, IR, I1, a.R, p.wg_kib);
    pm_fill_args(l, a);
    hipError_t e = pm_launch(l, a, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t run_pm(const nncp_plan* P, int side, void* T, int t_f64, const void* X, bool scaled, const Sink& st) {
  return run_pm_at(P, side, P->p.s, P->L.pmL[side], T, t_f64, X, scaled, st);
}

// MTTKRP of mode n without the dimension tree: one partial MTTKRP from X, then
// multi-TTVs down to M^(n). *M / *m_f64 say where it lives.
hipError_t direct_mttkrp(const nncp_plan* P, int n, bool scaled, const Sink& st0, const void** M, int* m_f64) {
  const Problem& p = P->p;
  const int side = P->L.dside[n], s = P->L.dsplit[n];
  const int f64 = P->L.node_f64;
  void* cur = P->dtA();
  void* nxt = P->dtB();
  Sink st = st0;
  st.mode = n;
  st.step = 0;
  hipError_t e = run_pm_at(P, side, s, P->L.dpm[n], cur, f64, P->X, scaled, st);
  if (e != hipSuccess) return e;
  if (side == 0) {
    // temporary over modes 0..n: contract modes 0..n-1 one at a time
    for (int k = 0; k < n; ++k) {
      MttvArgs a{};
      a.T = cur;
      a.t_f64 = f64;
      a.Ia = p.dims[k];
      a.J = prod_range(p, k + 1, n);
      a.R = p.R;
      a.krp = krp_for(P, k, k, scaled);
      a.out = nxt;
      a.out_f64 = f64;
      st.step = k + 1;
      if ((e = mttv_lead_launch(a, st)) != hipSuccess) return e;
      std::swap(cur, nxt);
    }
    *M = cur;
    *m_f64 = f64;
    return hipSuccess;
  }
  // temporary over modes n..N-1: contract modes n+1..N-1 at once
  if (n == p.N - 1) {
    *M = cur;
    *m_f64 = f64;
    return hipSuccess;
  }
  MttvArgs a{};
  a.T = cur;
  a.t_f64 = f64;
  a.Ia = p.dims[n];
  a.J = prod_range(p, n + 1, p.N - 1);
  a.R = p.R;
  a.krp = krp_for(P, n + 1, p.N - 1, scaled);
  a.out = P->Mbuf();
  a.out_f64 = 1;
  *M = P->Mbuf();
  *m_f64 = 1;
  st.step = 1;
  return mttv_trail_launch(a, st);
}

// Computes tree node i (see build_tree): a root partial MTTKRP, or a multi-TTV
// from its parent. A leaf that is not a root branch goes to M (FP64). *M and
// *m_f64 (optional) say where a leaf's MTTKRP lives.
hipError_t tree_op(const nncp_plan* P, int i, bool scaled, const Sink& st, const void** M, int* m_f64) {
  const Problem& p = P->p;
  const TNode& t = P->L.tn[i];
  const int f64 = P->L.node_f64;
  const bool leaf = t.a == t.b;
  if (t.kind == T_PM_LEFT || t.kind == T_PM_RIGHT) {
    if (leaf && M) {
      *M = P->tbuf(i);
      *m_f64 = f64;
    }
    return run_pm(P, t.kind == T_PM_LEFT ? 0 : 1, P->tbuf(i), f64, P->X, scaled, st);
  }
  const TNode& q = P->L.tn[t.parent];
  MttvArgs a{};
  a.T = P->tbuf(t.parent);
  a.t_f64 = f64;
  a.R = p.R;
  if (t.kind == T_TRAIL) {  // keep modes a..b of the parent, contract b+1..q.b
    a.Ia = t.rows;
    a.J = prod_range(p, t.b + 1, q.b);
    a.krp = krp_for(P, t.b + 1, q.b, scaled);
  } else {  // contract modes q.a..a-1 of the parent, keep a..b
    a.Ia = prod_range(p, q.a, t.a - 1);
    a.J = t.rows;
    a.krp = krp_for(P, q.a, t.a - 1, scaled);
  }
  if (leaf) {
    a.out = P->Mbuf();
    a.out_f64 = 1;
    if (M) {
      *M = P->Mbuf();
      *m_f64 = 1;
    }
  } else {
    a.out = P->tbuf(i);
    a.out_f64 = f64;
  }
  return t.kind == T_TRAIL ? mttv_trail_launch(a, st) : mttv_lead_launch(a, st);
}

// The tree ops of mode n (its schedule), numbered as the sink's steps.
hipError_t tree_mode(const nncp_plan* P, int n, bool scaled, const Sink& st0, const void** M, int* m_f64) {
  Sink st = st0;
  st.mode = n;
  for (int k = 0; k < P->L.nsched[n]; ++k) {
    st.step = k;
    hipError_t e = tree_op(P, P->L.sched[n][k], scaled, st, M, m_f64);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

FinalizeArgs fin_args(const nncp_plan* P, int n, const void* M, int m_f64, int set_model, int next_mode,
                      int do_fit) {
  const Problem& p = P->p;
  FinalizeArgs f{};
  f.W = P->H[n];
  f.M = M;
  f.m_f64 = m_f64;
  f.I = p.dims[n];
  f.R = p.R;
  f.N = p.N;
  f.mode = n;
  f.G = P->G();
  f.lam = P->lam();
  f.lam_model = P->lam_model();
  f.S = P->S();
  f.next_mode = next_mode;
  f.set_model = set_model;
  f.do_fit = do_fit;
  f.alpha = P->alpha();
  f.fit_out = P->fit();
  f.iter_counter = P->iter();
  f.fit_capacity = kFitCap;
  f.partial = P->finpart();
  f.nchunks = finalize_chunks(p.dims[n], p.R, &f.rows_per_chunk);
  return f;
}

enum { PH_PM = 0, PH_MTTV = 1, PH_NLS = 2, PH_GRAM = 3, PH_ERR = 4, PH_TOTAL = 5 };

// Enqueue one outer iteration. With timers, events bracket each phase (no graph).
hipError_t enqueue_iteration(nncp_plan* P, const Sink& st0, std::vector<std::pair<int, hipEvent_t>>* marks) {
  const Problem& p = P->p;
  auto mark = [&](int phase) -> hipError_t {
    if (!marks) return hipSuccess;
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    r = hipEventRecord(e, st0.st);
    marks->push_back({phase, e});
    return r;
  };
  hipError_t e;
  for (int n = 0; n < p.N; ++n) {
    const void* M = nullptr;
    int m_f64 = 1;
    Sink st = st0;
    st.mode = n;
    if (p.no_tree) {
      if ((e = mark(PH_PM)) != hipSuccess) return e;
      if ((e = direct_mttkrp(P, n, true, st, &M, &m_f64)) != hipSuccess) return e;
    } else {
      for (int k = 0; k < P->L.nsched[n]; ++k) {
        const int i = P->L.sched[n][k];
        const int kind = P->L.tn[i].kind;
        if ((e = mark(kind == T_PM_LEFT || kind == T_PM_RIGHT ? PH_PM : PH_MTTV)) != hipSuccess) return e;
        st.step = k;
        if ((e = tree_op(P, i, true, st, &M, &m_f64)) != hipSuccess) return e;
      }
    }
    st.step = kStepUpdate;
    if ((e = mark(PH_NLS)) != hipSuccess) return e;
    UpdateArgs u{};
    u.M = M;
    u.m_f64 = m_f64;
    u.W = P->H[n];
    u.I = p.dims[n];
    u.R = p.R;
    u.S = P->S() + (int64_t)n * p.R * p.R;
    u.lam_model = P->lam_model();
    u.lam_self = P->lam() + (int64_t)n * p.R;
    u.update = p.update;
    u.sweeps = p.sweeps;
    u.tol = p.inner_tol;
    if ((e = update_launch(u, st)) != hipSuccess) return e;
    const bool last = (n == p.N - 1);
    if ((e = mark(last ? PH_ERR : PH_GRAM)) != hipSuccess) return e;
    st.step = kStepFinal;
    if ((e = finalize_launch(fin_args(P, n, M, m_f64, 1, (n + 1) % p.N, last ? 1 : 0), st)) != hipSuccess) return e;
  }
  return mark(-1);
}

int destroy_graph(nncp_plan* P) {
  if (P->gexec) hipGraphExecDestroy(P->gexec);
  if (P->graph) hipGraphDestroy(P->graph);
  P->gexec = nullptr;
  P->graph = nullptr;
  return NNCP_OK;
}

// The capture stream and its events are created on first use, so plans that are
// only ever advanced by a batch own none.
int ensure_capture_stream(nncp_plan* P) {
  if (!P->cap_stream && hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking) != hipSuccess)
    return NNCP_EDEVICE;
  for (auto& e : P->ev)
    if (!e && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return NNCP_EDEVICE;
  return NNCP_OK;
}

int build_graph(nncp_plan* P) {
  destroy_graph(P);
  if (ensure_capture_stream(P) != NNCP_OK) return NNCP_EDEVICE;
  HIPCHK(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = enqueue_iteration(P, sink_of(P->cap_stream), nullptr);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(P->cap_stream, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) hipGraphDestroy(g);
    return NNCP_EDEVICE;
  }
  P->graph = g;
  HIPCHK(hipGraphInstantiate(&P->gexec, g, nullptr, nullptr, 0));
  return NNCP_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int nncp_last_device_error(int* hip_error, int* where) {
  const uint64_t v = nncpk::last_device_error();
  if (hip_error) *hip_error = (int)(uint32_t)(v >> 32);
  if (where) *where = (int)(uint32_t)v;
  return v ? NNCP_EDEVICE : NNCP_OK;
}

const char* nncp_strerror(int s) {
  switch (s) {
    case NNCP_OK: return "ok";
    case NNCP_EINVAL: return "invalid argument";
    case NNCP_ENOMEM: return "out of device memory or over budget";
    case NNCP_EDEVICE: return "HIP runtime or kernel launch failure";
    case NNCP_EBUSY: return "job not finished";
    case NNCP_ENOTFOUND: return "unknown job";
    case NNCP_ECANCELED: return "job cancelled or failed";
    default: return "unknown status";
  }
}

int nncp_version(void) { return 100; }

size_t nncp_workspace_bytes(int N, const int64_t* dims, int R, int dtype, const nncp_options* opt) {
  Problem p;
  if (fill_problem(p, N, dims, R, dtype, NNCP_HALS, opt ? opt->split : 0) != NNCP_OK) return 0;
  p.wg_kib = opt ? opt->pm_wg_kib : 0;
  p.no_tree = opt ? (opt->no_tree != 0) : 0;
  p.peel = opt ? opt->tree_peel : 0;
  return make_layout(p).total;
}

int nncp_plan_create(nncp_plan** out, const void* X, int dtype, int N, const int64_t* dims, int R,
                     int update, float* const* H, const double* lambda_in, void* workspace,
                     size_t ws_bytes, const nncp_options* opt, void* stream) {
  if (!out || !X || !H) return NNCP_EINVAL;
  *out = nullptr;
  Problem p;
  int st = fill_problem(p, N, dims, R, dtype, update, opt ? opt->split : 0);
  if (st != NNCP_OK) return st;
  p.wg_kib = opt ? opt->pm_wg_kib : 0;
  p.no_tree = opt ? (opt->no_tree != 0) : 0;
  p.sweeps = (opt && opt->inner_sweeps > 0) ? opt->inner_sweeps : 1;
  if (p.sweeps > NNCP_MAX_SWEEPS) return NNCP_EINVAL;
  p.inner_tol = opt ? opt->inner_tol : 0.0;
  if (!(p.inner_tol >= 0.0) || !std::isfinite(p.inner_tol)) return NNCP_EINVAL;
  p.peel = opt ? opt->tree_peel : 0;
  for (int k = 0; k < N; ++k)
    if (!H[k]) return NNCP_EINVAL;
  nncp_plan* P = new (std::nothrow) nncp_plan();
  if (!P) return NNCP_ENOMEM;
  P->p = p;
  P->L = make_layout(p);
  P->X = X;
  for (int k = 0; k < N; ++k) P->H[k] = H[k];
  P->user_stream = (hipStream_t)stream;
  P->use_graph = !(opt && (opt->no_graph || opt->phase_timers));
  P->phase_timers = opt && opt->phase_timers;
  P->record_fit = !(opt && opt->no_record_fit);
  P->tol = opt ? opt->tol : 0.0;
  if (workspace) {
    if (ws_bytes < P->L.total) {
      delete P;
      return NNCP_EINVAL;
    }
    P->ws = (char*)workspace;
  } else {
    void* w = nullptr;
    if (hipMalloc(&w, P->L.total) != hipSuccess) {
      delete P;
      return NNCP_ENOMEM;
    }
    P->ws = (char*)w;
    P->own_ws = true;
  }
  if (((uintptr_t)P->ws) % 256 != 0) {
    // the layout assumes a 256-byte aligned base
    if (P->own_ws) hipFree(P->ws);
    delete P;
    return NNCP_EINVAL;
  }
  hipStream_t s = P->user_stream;
  auto fail = [&](int code) {
    nncp_plan_destroy(P);
    return code;
  };
  // zero counters, iteration counter, the zero block read by masked loads
  if (fill_u32_launch(P->counters(), P->L.ncounters, 0u, s) != hipSuccess) return fail(NNCP_EDEVICE);
  if (fill_u32_launch(P->zeros(), 64, 0u, s) != hipSuccess) return fail(NNCP_EDEVICE);
  if (fill_u32_launch((unsigned*)P->iter(), 1, 0u, s) != hipSuccess) return fail(NNCP_EDEVICE);
  // lambda_in
  if (lambda_in) {
    if (hipMemcpyAsync(P->lam_in(), lambda_in, sizeof(double) * R, hipMemcpyHostToDevice, s) != hipSuccess)
      return fail(NNCP_EDEVICE);
  } else if (fill_f64_launch(P->lam_in(), R, 1.0, s) != hipSuccess) {
    return fail(NNCP_EDEVICE);
  }
  // alpha = ||X||^2
  if (norm_sq_launch(X, dtype, p.I, P->alpha(), P->nspart(), P->counters() + P->L.ncounters - 2,
                     P->L.ns_blocks, s) != hipSuccess)
    return fail(NNCP_EDEVICE);
  // starting Grams / norms per mode, then model weights and S^(1)
  for (int k = 0; k < N; ++k)
    if (finalize_launch(fin_args(P, k, nullptr, 0, 0, -1, 0), s) != hipSuccess) return fail(NNCP_EDEVICE);
  if (init_model_launch(P->lam_in(), P->lam(), P->lam_model(), P->G(), P->S(), N, R, s) != hipSuccess)
    return fail(NNCP_EDEVICE);
  if (hipStreamSynchronize(s) != hipSuccess) return fail(NNCP_EDEVICE);
  *out = P;
  return NNCP_OK;
}

int nncp_plan_time_node(nncp_plan* P, int mode, int reps, double* ms_avg) {
  if (!P || !ms_avg || reps < 1 || mode < 0 || mode >= P->p.N) return NNCP_EINVAL;
  hipStream_t s = P->user_stream;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return NNCP_EDEVICE;
  }
  int st = NNCP_OK;
  if (hipEventRecord(e0, s) != hipSuccess) st = NNCP_EDEVICE;
  // the first tree op of the mode (a root partial MTTKRP for modes 1 and s+1)
  const int node = P->L.nsched[mode] > 0 ? P->L.sched[mode][0] : -1;
  for (int i = 0; st == NNCP_OK && node >= 0 && i < reps; ++i)
    if (tree_op(P, node, true, s, nullptr, nullptr) != hipSuccess) st = NNCP_EDEVICE;
  float ms = 0.f;
  if (st == NNCP_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    st = NNCP_EDEVICE;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *ms_avg = (double)ms / reps;
  return st;
}

int nncp_plan_time_mttkrp(nncp_plan* P, int reps, double* ms_avg) {
  if (!P || !ms_avg || reps < 1) return NNCP_EINVAL;
  hipStream_t s = P->user_stream;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return NNCP_EDEVICE;
  }
  int st = NNCP_OK;
  if (hipEventRecord(e0, s) != hipSuccess) st = NNCP_EDEVICE;
  for (int i = 0; st == NNCP_OK && i < reps; ++i)
    for (int n = 0; st == NNCP_OK && n < P->p.N; ++n) {
      const void* M = nullptr;
      int m_f64 = 1;
      if (P->p.no_tree) {
        if (direct_mttkrp(P, n, true, s, &M, &m_f64) != hipSuccess) st = NNCP_EDEVICE;
      } else if (tree_mode(P, n, true, s, &M, &m_f64) != hipSuccess) {
        st = NNCP_EDEVICE;
      }
    }
  float ms = 0.f;
  if (st == NNCP_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
    st = NNCP_EDEVICE;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *ms_avg = (double)ms / reps;
  return st;
}

int nncp_autotune_split(const void* X, int dtype, int N, const int64_t* dims, int R, float* const* H,
                        const nncp_options* opt, int reps, int* best_split, double* ms, void* stream) {
  if (!X || !H || !dims || !best_split || reps < 1 || N < 2 || N > kMaxModes) return NNCP_EINVAL;
  nncp_options o{};
  if (opt) o = *opt;
  o.no_graph = 1;  // no iteration is run: nothing to capture
  int best = 0, st_any = NNCP_ENOMEM;
  double best_ms = 0.0;
  for (int s = 1; s < N; ++s) {
    if (ms) ms[s - 1] = -1.0;
    o.split = s;
    nncp_plan* P = nullptr;
    int st = nncp_plan_create(&P, X, dtype, N, dims, R, NNCP_HALS, H, nullptr, nullptr, 0, &o, stream);
    if (st == NNCP_ENOMEM) {
      (void)hipGetLastError();
      continue;
    }
    if (st != NNCP_OK) return st;
    double warm = 0.0, t = 0.0;
    st = nncp_plan_time_mttkrp(P, 1, &warm);
    if (st == NNCP_OK) st = nncp_plan_time_mttkrp(P, reps, &t);
    nncp_plan_destroy(P);
    if (st != NNCP_OK) return st;
    st_any = NNCP_OK;
    if (ms) ms[s - 1] = t;
    if (best == 0 || t < best_ms) {
      best = s;
      best_ms = t;
    }
  }
  if (best == 0) return st_any;
  *best_split = best;
  return NNCP_OK;
}

int nncp_autotune_tree(const void* X, int dtype, int N, const int64_t* dims, int R, float* const* H,
                       const nncp_options* opt, int reps, int cap, int* splits, unsigned long long* peels,
                       double* ms, int* count, int* best, void* stream) {
  if (!X || !H || !dims || !splits || !peels || !ms || !count || !best || reps < 1 || cap < 1 || N < 2 ||
      N > kMaxModes)
    return NNCP_EINVAL;
  *count = 0;
  *best = -1;
  // every tree of every root split, in order: root split s, then the shapes of
  // the left half and of the right half (peel-first before peel-last at each node)
  std::vector<std::pair<int, uint64_t>> cand;
  std::function<void(int, int, uint64_t, std::vector<uint64_t>&)> shapes = [&](int a, int b, uint64_t m,
                                                                               std::vector<uint64_t>& out) {
    if (b - a < 2) {
      out.push_back(m);
      return;
    }
    shapes(a + 1, b, m, out);                               // {a} | {a+1..b}
    shapes(a, b - 1, m | (1ull << (a * 8 + b)), out);       // {a..b-1} | {b}
  };
  for (int s = 1; s < N; ++s) {
    std::vector<uint64_t> left, right;
    shapes(0, s - 1, 0, left);
    shapes(s, N - 1, 0, right);
    for (uint64_t l : left)
      for (uint64_t r : right) cand.push_back({s, l | r});
  }
  nncp_options o{};
  if (opt) o = *opt;
  o.no_graph = 1;  // no iteration is run: nothing to capture
  o.no_tree = 0;
  int st_any = NNCP_ENOMEM;
  double best_ms = 0.0;
  for (size_t c = 0; c < cand.size() && *count < cap; ++c) {
    o.split = cand[c].first;
    o.tree_peel = cand[c].second;
    nncp_plan* P = nullptr;
    int st = nncp_plan_create(&P, X, dtype, N, dims, R, NNCP_HALS, H, nullptr, nullptr, 0, &o, stream);
    if (st == NNCP_ENOMEM) {
      (void)hipGetLastError();
      continue;
    }
    if (st != NNCP_OK) return st;
    double warm = 0.0, t = 0.0;
    st = nncp_plan_time_mttkrp(P, 1, &warm);
    if (st == NNCP_OK) st = nncp_plan_time_mttkrp(P, reps, &t);
    nncp_plan_destroy(P);
    if (st != NNCP_OK) return st;
    st_any = NNCP_OK;
    const int k = (*count)++;
    splits[k] = cand[c].first;
    peels[k] = cand[c].second;
    ms[k] = t;
    if (*best < 0 || t < best_ms) {
      *best = k;
      best_ms = t;
    }
  }
  return *best < 0 ? st_any : NNCP_OK;
}

int nncp_plan_set_stream(nncp_plan* P, void* stream) {
  if (!P) return NNCP_EINVAL;
  P->user_stream = (hipStream_t)stream;
  return NNCP_OK;
}

int nncp_plan_destroy(nncp_plan* P) {
  if (!P) return NNCP_EINVAL;
  destroy_graph(P);
  if (P->cap_stream) hipStreamDestroy(P->cap_stream);
  for (auto& e : P->ev)
    if (e) hipEventDestroy(e);
  if (P->own_ws && P->ws) hipFree(P->ws);
  delete P;
  return NNCP_OK;
}

int nncp_plan_run(nncp_plan* P, int iters, double* fit, int* iters_done) {
  if (!P || iters < 0) return NNCP_EINVAL;
  if (iters_done) *iters_done = 0;
  if (iters == 0) return NNCP_OK;
  hipStream_t us = P->user_stream;
  int done = 0;
  double prev_fit = NAN;
  std::vector<double> hfit;
  while (done < iters) {
    int chunk = std::min(iters - done, kFitCap);
    if (P->tol > 0) chunk = 1;
    if (fill_u32_launch((unsigned*)P->iter(), 1, 0u, us) != hipSuccess) return NNCP_EDEVICE;
    if (P->use_graph) {
      if (!P->gexec) {
        int r = build_graph(P);
        if (r != NNCP_OK) return r;
      }
      HIPCHK(hipEventRecord(P->ev[0], us));
      HIPCHK(hipStreamWaitEvent(P->cap_stream, P->ev[0], 0));
      for (int i = 0; i < chunk; ++i) HIPCHK(hipGraphLaunch(P->gexec, P->cap_stream));
      HIPCHK(hipEventRecord(P->ev[1], P->cap_stream));
      HIPCHK(hipStreamWaitEvent(us, P->ev[1], 0));
    } else if (P->phase_timers) {
      for (int i = 0; i < chunk; ++i) {
        std::vector<std::pair<int, hipEvent_t>> marks;
        hipError_t e = enqueue_iteration(P, sink_of(us), &marks);
        if (e == hipSuccess) e = hipStreamSynchronize(us);
        for (size_t j = 0; j + 1 < marks.size(); ++j) {
          float ms = 0.f;
          if (e == hipSuccess && hipEventElapsedTime(&ms, marks[j].second, marks[j + 1].second) == hipSuccess &&
              marks[j].first >= 0)
            P->phase_ms[marks[j].first] += ms;
        }
        if (e == hipSuccess && marks.size() >= 2) {
          float ms = 0.f;
          if (hipEventElapsedTime(&ms, marks.front().second, marks.back().second) == hipSuccess)
            P->phase_ms[PH_TOTAL] += ms;
        }
        for (auto& m : marks) hipEventDestroy(m.second);
        if (e != hipSuccess) return NNCP_EDEVICE;
      }
    } else {
      for (int i = 0; i < chunk; ++i)
        if (enqueue_iteration(P, sink_of(us), nullptr) != hipSuccess) return NNCP_EDEVICE;
    }
    hfit.resize(chunk);
    HIPCHK(hipMemcpyAsync(hfit.data(), P->fit(), sizeof(double) * chunk, hipMemcpyDeviceToHost, us));
    HIPCHK(hipStreamSynchronize(us));
    if (fit) std::memcpy(fit + done, hfit.data(), sizeof(double) * chunk);
    done += chunk;
    if (P->tol > 0) {
      double f = hfit[chunk - 1];
      if (!std::isnan(prev_fit) && std::fabs(f - prev_fit) < P->tol) break;
      prev_fit = f;
    }
  }
  if (iters_done) *iters_done = done;
  return NNCP_OK;
}

int nncp_plan_finish(nncp_plan* P, double* lambda) {
  if (!P || !lambda) return NNCP_EINVAL;
  hipStream_t s = P->user_stream;
  const Problem& p = P->p;
  for (int k = 0; k < p.N; ++k)
    if (normalize_out_launch(P->H[k], p.dims[k], p.R, P->lam() + (int64_t)k * p.R, s) != hipSuccess)
      return NNCP_EDEVICE;
  if (unit_lambda_launch(P->lam(), (int64_t)p.N * p.R, s) != hipSuccess) return NNCP_EDEVICE;
  HIPCHK(hipMemcpyAsync(lambda, P->lam_model(), sizeof(double) * p.R, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return NNCP_OK;
}

int nncp_plan_phase_ms(const nncp_plan* P, double* ms) {
  if (!P || !ms) return NNCP_EINVAL;
  for (int i = 0; i < 6; ++i) ms[i] = P->phase_ms[i];
  return NNCP_OK;
}

int nncp(const void* X, int dtype, int N, const int64_t* dims, int R, int iters, int update,
         float* const* H, double* lambda, double* fit, int* iters_done, void* workspace,
         size_t ws_bytes, const nncp_options* opt, void* stream) {
  if (iters < 0 || !lambda) return NNCP_EINVAL;
  nncp_plan* P = nullptr;
  int st = nncp_plan_create(&P, X, dtype, N, dims, R, update, H, lambda, workspace, ws_bytes, opt, stream);
  if (st != NNCP_OK) return st;
  std::vector<double> f(iters > 0 ? iters : 1, NAN);
  int done = 0;
  st = nncp_plan_run(P, iters, f.data(), &done);
  if (st == NNCP_OK) st = nncp_plan_finish(P, lambda);
  if (st == NNCP_OK && fit) {
    if (opt && opt->no_record_fit) fit[0] = done > 0 ? f[done - 1] : NAN;
    else std::memcpy(fit, f.data(), sizeof(double) * (size_t)done);
  }
  if (iters_done) *iters_done = done;
  nncp_plan_destroy(P);
  return st;
}

// ---- steps ----

int nncp_quantize(const float* src, void* dst, int dtype, int64_t n, void* stream) {
  if (!src || !dst || n < 0 || (dtype != NNCP_BF16 && dtype != NNCP_F16)) return NNCP_EINVAL;
  if (n == 0) return NNCP_OK;
  return quantize_launch(src, dst, dtype, n, (hipStream_t)stream) == hipSuccess ? NNCP_OK : NNCP_EDEVICE;
}

int nncp_norm_sq(const void* X, int dtype, int64_t n, double* out_dev, void* stream) {
  if (!X || !out_dev || n < 1 || (dtype < 0 || dtype > 2)) return NNCP_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int nb = norm_sq_blocks(n);
  void* scratch = nullptr;
  if (hipMalloc(&scratch, sizeof(double) * nb + 256) != hipSuccess) return NNCP_ENOMEM;
  unsigned* ctr = (unsigned*)((char*)scratch + align256(sizeof(double) * nb));
  int st = NNCP_OK;
  if (fill_u32_launch(ctr, 1, 0u, s) != hipSuccess ||
      norm_sq_launch(X, dtype, n, out_dev, (double*)scratch, ctr, nb, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    st = NNCP_EDEVICE;
  hipFree(scratch);
  return st;
}

// A throw-away plan-like context for the step entry points (no lambda scaling).
struct StepCtx {
  nncp_plan P;
  void* mem = nullptr;
  ~StepCtx() {
    if (mem) hipFree(mem);
  }
};

static int step_ctx(StepCtx& c, const void* X, int dtype, int N, const int64_t* dims, int s, float* const* H,
                    int R) {
  int st = fill_problem(c.P.p, N, dims, R, dtype, NNCP_HALS, s);
  if (st != NNCP_OK) return st;
  c.P.L = make_layout(c.P.p);
  c.P.X = X;
  for (int k = 0; k < N; ++k) {
    if (!H[k]) return NNCP_EINVAL;
    c.P.H[k] = H[k];
  }
  if (hipMalloc(&c.mem, c.P.L.total) != hipSuccess) return NNCP_ENOMEM;
  c.P.ws = (char*)c.mem;
  if (fill_u32_launch(c.P.counters(), c.P.L.ncounters, 0u, nullptr) != hipSuccess) return NNCP_EDEVICE;
  if (fill_u32_launch(c.P.zeros(), 64, 0u, nullptr) != hipSuccess) return NNCP_EDEVICE;
  return NNCP_OK;
}

int nncp_partial_mttkrp(const void* X, int dtype, int N, const int64_t* dims, int s, int side,
                        float* const* H, int R, double* T, void* stream) {
  if (!X || !H || !T || (side != 0 && side != 1) || s < 1) return NNCP_EINVAL;
  StepCtx c;
  int st = step_ctx(c, X, dtype, N, dims, s, H, R);
  if (st != NNCP_OK) return st;
  hipStream_t hs = (hipStream_t)stream;
  if (hipDeviceSynchronize() != hipSuccess) return NNCP_EDEVICE;
  if (run_pm(&c.P, side, T, 1, X, false, hs) != hipSuccess) return NNCP_EDEVICE;
  if (hipStreamSynchronize(hs) != hipSuccess) return NNCP_EDEVICE;
  return NNCP_OK;
}

int nncp_mttv(const double* T, int nm, const int64_t* node_dims, int kind, float* const* Hf, int R,
              double* out, void* stream) {
  if (!T || !node_dims || !Hf || !out || nm < 2 || nm > kMaxModes || R < 1 || R > kMaxRank ||
      (kind != 0 && kind != 1))
    return NNCP_EINVAL;
  for (int k = 0; k < nm; ++k)
    if (node_dims[k] < 1 || node_dims[k] > INT32_MAX) return NNCP_EINVAL;
  MttvArgs a{};
  a.T = T;
  a.t_f64 = 1;
  a.Ia = node_dims[0];
  a.J = 1;
  for (int k = 1; k < nm; ++k) a.J *= node_dims[k];
  if (a.J > (int64_t)UINT32_MAX) return NNCP_EINVAL;
  a.R = R;
  a.out = out;
  a.out_f64 = 1;
  a.krp.lam = nullptr;
  if (kind == 0) {
    a.krp.nm = nm - 1;
    for (int j = 0; j < nm - 1; ++j) {
      if (!Hf[j]) return NNCP_EINVAL;
      a.krp.f[j] = Hf[j];
      a.krp.dim[j] = (int)node_dims[j + 1];
      a.krp.mode[j] = j;
    }
  } else {
    if (!Hf[0]) return NNCP_EINVAL;
    a.krp.nm = 1;
    a.krp.f[0] = Hf[0];
    a.krp.dim[0] = (int)node_dims[0];
  }
  hipStream_t hs = (hipStream_t)stream;
  hipError_t e = kind == 0 ? mttv_trail_launch(a, hs) : mttv_lead_launch(a, hs);
  if (e != hipSuccess) return NNCP_EDEVICE;
  return hipStreamSynchronize(hs) == hipSuccess ? NNCP_OK : NNCP_EDEVICE;
}

int nncp_mttkrp(const void* X, int dtype, int N, const int64_t* dims, int s, int n, float* const* H, int R,
                double* M, void* stream) {
  if (!X || !H || !M || s < 1 || n < 0 || n >= N) return NNCP_EINVAL;
  StepCtx c;
  int st = step_ctx(c, X, dtype, N, dims, s, H, R);
  if (st != NNCP_OK) return st;
  hipStream_t hs = (hipStream_t)stream;
  if (hipDeviceSynchronize() != hipSuccess) return NNCP_EDEVICE;
  // the schedules of n's half from its first mode up to n: every node on the
  // path to leaf n is computed (with the given factors) by the time n's runs
  const Problem& p = c.P.p;
  const void* Mp = nullptr;
  int m_f64 = 1;
  for (int k = n < p.s ? 0 : p.s; k <= n; ++k)
    if (tree_mode(&c.P, k, false, hs, &Mp, &m_f64) != hipSuccess) return NNCP_EDEVICE;
  const int64_t cnt = p.dims[n] * R;
  if ((m_f64 ? copy_f64_launch(M, (const double*)Mp, cnt, hs) : widen_f32_launch(M, (const float*)Mp, cnt, hs)) !=
      hipSuccess)
    return NNCP_EDEVICE;
  return hipStreamSynchronize(hs) == hipSuccess ? NNCP_OK : NNCP_EDEVICE;
}

int nncp_gram(const float* H, int64_t I, int R, double* G, void* stream) {
  if (!H || !G || I < 1 || R < 1 || R > kMaxRank) return NNCP_EINVAL;
  hipStream_t hs = (hipStream_t)stream;
  int rpc;
  const int chunks = finalize_chunks(I, R, &rpc);
  const size_t RR = (size_t)R * R;
  size_t bytes = align256(sizeof(double) * chunks * (RR + 1)) + align256(sizeof(double) * RR) +
                 align256(sizeof(double) * R) * 2 + 256;
  char* mem = nullptr;
  if (hipMalloc(&mem, bytes) != hipSuccess) return NNCP_ENOMEM;
  size_t o = 0;
  double* part = (double*)(mem + o);
  o += align256(sizeof(double) * chunks * (RR + 1));
  double* Gn = (double*)(mem + o);
  o += align256(sizeof(double) * RR);
  double* lam = (double*)(mem + o);
  o += align256(sizeof(double) * R);
  double* lamm = (double*)(mem + o);
  FinalizeArgs f{};
  f.W = H;
  f.I = I;
  f.R = R;
  f.N = 1;
  f.mode = 0;
  f.G = Gn;
  f.lam = lam;
  f.lam_model = lamm;
  f.next_mode = -1;
  f.gram_raw = G;
  f.partial = part;
  f.nchunks = chunks;
  f.rows_per_chunk = rpc;
  int st = NNCP_OK;
  if (finalize_launch(f, hs) != hipSuccess || hipStreamSynchronize(hs) != hipSuccess) st = NNCP_EDEVICE;
  hipFree(mem);
  return st;
}

int nncp_nls_update(const double* M, float* H, int64_t I, int R, const double* S, double* lambda, int update,
                    double* G, void* stream) {
  return nncp_nls_solve(M, H, I, R, S, lambda, update, 1, 0.0, nullptr, G, stream);
}

int nncp_nls_solve(const double* M, float* H, int64_t I, int R, const double* S, double* lambda, int update,
                   int max_sweeps, double tol, double* W_out, double* G, void* stream) {
  if (!M || !H || !S || !lambda || !G || I < 1 || R < 1 || R > kMaxRank ||
      (update != NNCP_HALS && update != NNCP_MU) || max_sweeps < 1 || max_sweeps > NNCP_MAX_SWEEPS ||
      !(tol >= 0.0) || !std::isfinite(tol))
    return NNCP_EINVAL;
  hipStream_t hs = (hipStream_t)stream;
  int rpc;
  const int chunks = finalize_chunks(I, R, &rpc);
  const size_t RR = (size_t)R * R;
  size_t bytes = align256(sizeof(double) * chunks * (RR + 1)) + align256(sizeof(double) * R) * 2 + 256;
  char* mem = nullptr;
  if (hipMalloc(&mem, bytes) != hipSuccess) return NNCP_ENOMEM;
  double* part = (double*)mem;
  double* ones = (double*)(mem + align256(sizeof(double) * chunks * (RR + 1)));
  int st = NNCP_OK;
  UpdateArgs u{};
  u.M = M;
  u.m_f64 = 1;
  u.W = H;
  u.I = I;
  u.R = R;
  u.S = S;
  u.lam_model = lambda;
  u.lam_self = ones;
  u.update = update;
  u.sweeps = max_sweeps;
  u.tol = tol;
  u.W64 = W_out;
  FinalizeArgs f{};
  f.W = H;
  f.I = I;
  f.R = R;
  f.N = 1;
  f.mode = 0;
  f.G = G;
  f.lam = lambda;
  f.lam_model = lambda;
  f.next_mode = -1;
  f.partial = part;
  f.nchunks = chunks;
  f.rows_per_chunk = rpc;
  if (fill_f64_launch(ones, R, 1.0, hs) != hipSuccess ||
      update_launch(u, hs) != hipSuccess || finalize_launch(f, hs) != hipSuccess ||
      normalize_out_launch(H, I, R, lambda, hs) != hipSuccess || hipStreamSynchronize(hs) != hipSuccess)
    st = NNCP_EDEVICE;
  hipFree(mem);
  return st;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched plans: one outer iteration of every member plan per tick.
//
// Each member's iteration is recorded once as launch records (the kernels,
// grids and arguments its stand-alone run would launch). The records of all
// members are grouped by stage (mode, step) and kernel family; every group
// becomes one launch of a persistent work-list kernel whose items are the
// (op, tile) pairs of all members. Stages run in order, so each member's
// chain of kernels keeps its order, and members never share a buffer, so a
// member's results do not depend on who else is in the batch. The sequence of
// launches of one tick is captured into a HIP graph and replayed.
// ---------------------------------------------------------------------------
struct nncp_batch {
  hipStream_t st = nullptr;   // caller's stream
  hipStream_t cap = nullptr;  // capture / replay stream
  hipEvent_t ev[2] = {nullptr, nullptr};
  std::vector<nncp_plan*> plans;
  bool dirty = true;
  // Device work lists. Their addresses are baked into the captured graph; a
  // membership change rewrites their contents in place between ticks.
  KOp* d_ops = nullptr;
  size_t cap_ops = 0;
  BItem* d_items = nullptr;
  size_t cap_items = 0;
  int* d_grp = nullptr;  // per captured launch: {first item, item count}
  size_t cap_grp = 0;
  struct Launch {
    int stage, kid, kind, variant;
  };
  std::vector<Launch> launches;  // captured launches, in stage order
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  size_t n_items = 0;
  int64_t captures = 0, list_updates = 0;
  double rebuild_s = 0.0, graph_s = 0.0;  // host time: list rewrites (graph builds included), graph builds
};

namespace {

int device_cus() {
  static int n = [] {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      return 256;
    return cus;
  }();
  return n;
}

template <typename T>
int ensure_dev(T** p, size_t* cap, size_t n, size_t floor, bool* moved) {
  if (n <= *cap && *p) return NNCP_OK;
  if (*p) hipFree(*p);
  *p = nullptr;
  *cap = 0;
  *moved = true;
  // headroom, so that members joining later rarely need a larger list: at
  // least `floor` entries, else half again the current need
  size_t want = n < floor ? floor : n + n / 2;
  if (hipMalloc((void**)p, want * sizeof(T)) != hipSuccess) return NNCP_ENOMEM;
  *cap = want;
  return NNCP_OK;
}

void batch_drop_graph(nncp_batch* B) {
  if (B->gexec) hipGraphExecDestroy(B->gexec);
  if (B->graph) hipGraphDestroy(B->graph);
  B->gexec = nullptr;
  B->graph = nullptr;
}

// Records one iteration of every member, groups the records into the launches
// of one tick (stage order; within a stage one launch per batched kernel) and
// writes the device work lists. The tick's graph is captured again only when a
// launch is needed that the captured graph does not have, or a list outgrows
// its device buffer; otherwise the captured graph runs the new lists as they
// are (launches with no items of the current members find a count of zero).
int batch_build(nncp_batch* B) {
  std::vector<KOp> all;
  for (nncp_plan* P : B->plans) {
    std::vector<KOp> rec;
    Sink sk;
    sk.rec = &rec;
    if (enqueue_iteration(P, sk, nullptr) != hipSuccess) return NNCP_EDEVICE;
    all.insert(all.end(), rec.begin(), rec.end());
  }
  auto key_of = [](int stage, int kid) { return ((int64_t)stage << 32) | (uint32_t)kid; };
  std::map<int64_t, nncp_batch::Launch> need;
  for (const KOp& o : all) {
    const int kid = batch_kernel_id(o.kind, o.variant);
    need.emplace(key_of(o.stage, kid), nncp_batch::Launch{o.stage, kid, o.kind, o.variant});
  }
  std::map<int64_t, nncp_batch::Launch> have;
  for (const auto& l : B->launches) have.emplace(key_of(l.stage, l.kid), l);
  bool recapture = !B->gexec;
  for (const auto& kv : need)
    if (!have.count(kv.first)) {
      have.emplace(kv.first, kv.second);
      recapture = true;
    }
  // launches no member uses any more still run (with no items) every tick;
  // once they outnumber the used ones, the graph is built for the used ones only
  if (!recapture && have.size() > 2 * need.size() + 16) {
    have = need;
    recapture = true;
  }
  // launch order: by stage, then by kernel (the map's key order)
  std::vector<nncp_batch::Launch> L;
  std::map<int64_t, int> slot;
  for (const auto& kv : have) {
    slot[kv.first] = (int)L.size();
    L.push_back(kv.second);
  }
  // Items of each launch, contiguous. A batch item of a small op runs `coarse`
  // of its stand-alone work-groups in turn, so that an item carries enough work
  // to amortise fetching its descriptor (the blocks of these ops are tiny) --
  // but only while the launch still has several items per persistent group.
  {
    std::vector<double> blocks(L.size(), 0.0);
    for (const KOp& o : all)
      blocks[slot[key_of(o.stage, batch_kernel_id(o.kind, o.variant))]] += (double)o.gx * (double)o.gy;
    const double cus = (double)device_cus();
    for (KOp& o : all) {
      o.coarse = 1;
      const int kid = batch_kernel_id(o.kind, o.variant);
      if (kid < 100 || kid >= 1000) continue;  // small ops only
      const double groups = (double)batch_kernel_for(o.kind, o.variant).per_cu * cus;
      const double c = blocks[slot[key_of(o.stage, kid)]] / (4.0 * groups);
      const unsigned want = c >= 8.0 ? 8u : (c >= 1.0 ? (unsigned)c : 1u);
      o.coarse = want < o.gx ? want : (o.gx > 0 ? o.gx : 1u);
    }
  }
  std::vector<std::vector<BItem>> per(L.size());
  for (size_t i = 0; i < all.size(); ++i) {
    const KOp& o = all[i];
    auto& v = per[slot[key_of(o.stage, batch_kernel_id(o.kind, o.variant))]];
    const unsigned nx = (o.gx + o.coarse - 1) / o.coarse;
    for (unsigned by = 0; by < o.gy; ++by)
      for (unsigned bx = 0; bx < nx; ++bx) v.push_back(BItem{(int)i, (int)bx, (int)by});
  }
  // A persistent group takes items g, g + grid, g + 2 grid, ...: partial-MTTKRP
  // items in order of decreasing share of the tensor, so the largest start first
  // and the launch's tail is made of small ones.
  for (size_t g = 0; g < L.size(); ++g) {
    if (L[g].kind != K_PM_F32 && L[g].kind != K_PM_16) continue;
    auto share = [&](const BItem& it) {
      const KOp& o = all[it.op];
      return (double)o.u.pm.IL * (double)o.u.pm.IR / ((double)o.gx * (double)o.gy);
    };
    std::stable_sort(per[g].begin(), per[g].end(),
                     [&](const BItem& x, const BItem& y) { return share(x) > share(y); });
  }
  std::vector<BItem> items;
  std::vector<int> grp(2 * L.size());
  for (size_t g = 0; g < L.size(); ++g) {
    grp[2 * g] = (int)items.size();
    grp[2 * g + 1] = (int)per[g].size();
    items.insert(items.end(), per[g].begin(), per[g].end());
  }
  bool moved = false;
  if (recapture || all.size() > B->cap_ops || items.size() > B->cap_items || grp.size() > B->cap_grp)
    batch_drop_graph(B);  // the graph must not outlive the buffers it points at
  int r;
  // (at least 2048 ops, 32768 items and 256 launches: a batch of a few dozen
  // members never has to grow its lists, so joining and leaving never capture)
  if ((r = ensure_dev(&B->d_ops, &B->cap_ops, all.size(), 2048, &moved)) != NNCP_OK) return r;
  if ((r = ensure_dev(&B->d_items, &B->cap_items, items.size(), 32768, &moved)) != NNCP_OK) return r;
  if ((r = ensure_dev(&B->d_grp, &B->cap_grp, grp.size(), 512, &moved)) != NNCP_OK) return r;
  if (moved) recapture = true;
  if (!all.empty())
    HIPCHK(hipMemcpyAsync(B->d_ops, all.data(), all.size() * sizeof(KOp), hipMemcpyHostToDevice, B->cap));
  if (!items.empty())
    HIPCHK(hipMemcpyAsync(B->d_items, items.data(), items.size() * sizeof(BItem), hipMemcpyHostToDevice, B->cap));
  if (!grp.empty())
    HIPCHK(hipMemcpyAsync(B->d_grp, grp.data(), grp.size() * sizeof(int), hipMemcpyHostToDevice, B->cap));
  HIPCHK(hipStreamSynchronize(B->cap));
  B->n_items = items.size();
  ++B->list_updates;
  B->dirty = false;
  if (!recapture) return NNCP_OK;

  // The tick's graph is built node by node (no stream capture, so work that
  // other threads enqueue meanwhile, such as a serving loader's uploads and
  // allocations, cannot interfere with it): one kernel node per launch. The ops
  // of one stage are independent (different members, or independent ops of one
  // member), so a stage's launches depend only on all launches of the stage
  // before and may overlap one another's tails.
  const auto tg = std::chrono::steady_clock::now();
  batch_drop_graph(B);
  B->launches = L;
  const unsigned cus = (unsigned)device_cus();
  hipGraph_t gr = nullptr;
  HIPCHK(hipGraphCreate(&gr, 0));
  hipError_t e = hipSuccess;
  std::vector<hipGraphNode_t> before, cur;
  for (size_t g = 0; g < L.size() && e == hipSuccess; ++g) {
    if (g == 0 || L[g].stage != L[g - 1].stage) {
      if (!cur.empty()) before.swap(cur);
      cur.clear();
    }
    const BatchKernel bk = batch_kernel_for(L[g].kind, L[g].variant);
    if (!bk.fn) {
      e = hipErrorInvalidValue;
      break;
    }
    const BItem* it = B->d_items;
    const int* gp = B->d_grp + 2 * g;
    const KOp* ops = B->d_ops;
    void* args[] = {(void*)&it, (void*)&gp, (void*)&ops};
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(bk.fn);
    kp.gridDim = dim3((unsigned)bk.per_cu * cus);
    kp.blockDim = dim3(bk.threads);
    kp.sharedMemBytes = (unsigned)bk.lds;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipGraphNode_t node = nullptr;
    e = hipGraphAddKernelNode(&node, gr, before.empty() ? nullptr : before.data(), before.size(), &kp);
    if (e == hipSuccess) cur.push_back(node);
  }
  if (e != hipSuccess) {
    note_device_error((int)e, __LINE__);
    hipGraphDestroy(gr);
    B->launches.clear();
    return NNCP_EDEVICE;
  }
  B->graph = gr;
  if ((e = hipGraphInstantiate(&B->gexec, gr, nullptr, nullptr, 0)) != hipSuccess) {
    note_device_error((int)e, __LINE__);
    batch_drop_graph(B);
    B->launches.clear();
    return NNCP_EDEVICE;
  }
  ++B->captures;
  B->graph_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - tg).count();
  return NNCP_OK;
}

}  // namespace

namespace nncpk {

namespace {
std::atomic<uint64_t> g_last_device_error{0};
}

void note_device_error(int hip_error, int where) {
  g_last_device_error.store(((uint64_t)(uint32_t)hip_error << 32) | (uint32_t)where, std::memory_order_relaxed);
}

uint64_t last_device_error() { return g_last_device_error.load(std::memory_order_relaxed); }

int batch_kernel_id(int kind, int variant) {
  switch (kind) {
    case K_PM_F32: return 1000000 + variant;
    case K_PM_16: return 2000000 + variant;
    case K_PACK16: return 3000000 + variant;
    case K_FIN1K: case K_GRAM1K: case K_TAIL1K: return 2;
    case K_UPDATE: return 200 + variant;  // one kernel per register variant
    default: return 100 + kind;           // small ops: one kernel per kind
  }
}

namespace {
// Work-groups of a persistent launch per CU: as many as fit at once (at most
// cap); looked up once per kernel.
int groups_per_cu(const void* fn, int threads, size_t lds, int cap) {
  static std::mutex mu;
  static std::map<const void*, int> known;
  std::lock_guard<std::mutex> lk(mu);
  auto it = known.find(fn);
  if (it != known.end()) return it->second;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, threads, lds) != hipSuccess || n < 1) {
    (void)hipGetLastError();
    n = 1;
  }
  if (n > cap) n = cap;
  known.emplace(fn, n);
  return n;
}
}  // namespace

BatchKernel batch_kernel_for(int kind, int variant) {
  BatchKernel k;
  switch (kind) {
    case K_PM_F32:
      k.fn = pm_f32_batch_kernel(variant);
      k.threads = 256;
      k.lds = pm_variant_max_lds(kind, variant);
      k.per_cu = k.lds <= 80 * 1024 ? 2 : 1;  // the FP32 kernels are built for two groups per CU
      break;
    case K_PM_16:
      k.fn = pm16_batch_kernel(variant);
      k.threads = 256;
      k.lds = pm_variant_max_lds(kind, variant);
      k.per_cu = 1;
      break;
    case K_PACK16:
      k.fn = pm16_pack_batch_kernel(variant);
      k.threads = 256;
      k.per_cu = 4;
      break;
    case K_SCTAB:
      k.fn = pm_sctab_batch_kernel();
      k.threads = 256;
      k.per_cu = groups_per_cu(k.fn, 256, 0, 8);
      break;
    case K_FIN1K: case K_GRAM1K: case K_TAIL1K:
      k.fn = fin_batch_kernel_ptr();
      k.threads = 1024;
      k.lds = fin_batch_max_lds();
      k.per_cu = 1;
      break;
    default:
      // (the R > 64 forms, which need dynamic LDS, never run in a batch)
      if ((kind == K_UPDATE && variant <= 2) || kind == K_FIN_FUSED || kind == K_GRAM_CHUNKS || kind == K_FIN_TAIL)
        break;
      k.fn = small_batch_kernel_ptr(kind, variant);
      k.threads = 256;
      k.per_cu = k.fn ? groups_per_cu(k.fn, 256, 0, 8) : 1;
      break;
  }
  return k;
}

}  // namespace nncpk

extern "C" {

int nncp_batch_create(nncp_batch** out, void* stream) {
  if (!out) return NNCP_EINVAL;
  *out = nullptr;
  nncp_batch* B = new (std::nothrow) nncp_batch();
  if (!B) return NNCP_ENOMEM;
  B->st = (hipStream_t)stream;
  if (hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&B->ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&B->ev[1], hipEventDisableTiming) != hipSuccess) {
    nncp_batch_destroy(B);
    return NNCP_EDEVICE;
  }
  *out = B;
  return NNCP_OK;
}

int nncp_batch_add(nncp_batch* B, nncp_plan* P) {
  if (!B || !P) return NNCP_EINVAL;
  if (P->p.R > kPmMaxCols) return NNCP_EINVAL;  // one column chunk per partial MTTKRP
  for (nncp_plan* q : B->plans)
    if (q == P) return NNCP_EINVAL;
  try {
    B->plans.push_back(P);
  } catch (...) {
    return NNCP_ENOMEM;
  }
  B->dirty = true;
  return NNCP_OK;
}

int nncp_batch_remove(nncp_batch* B, nncp_plan* P) {
  if (!B || !P) return NNCP_EINVAL;
  auto it = std::find(B->plans.begin(), B->plans.end(), P);
  if (it == B->plans.end()) return NNCP_ENOTFOUND;
  B->plans.erase(it);
  B->dirty = true;
  return NNCP_OK;
}

int nncp_batch_size(const nncp_batch* B) { return B ? (int)B->plans.size() : 0; }

int nncp_batch_run(nncp_batch* B, int ticks) {
  if (!B || ticks < 0) return NNCP_EINVAL;
  if (ticks == 0 || B->plans.empty()) return NNCP_OK;
  if (B->dirty) {
    // members may have been set up on the caller's stream
    HIPCHK(hipStreamSynchronize(B->st));
    const auto t0 = std::chrono::steady_clock::now();
    int r = batch_build(B);
    B->rebuild_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (r != NNCP_OK) return r;
  }
  HIPCHK(hipEventRecord(B->ev[0], B->st));
  HIPCHK(hipStreamWaitEvent(B->cap, B->ev[0], 0));
  for (int t = 0; t < ticks; ++t) HIPCHK(hipGraphLaunch(B->gexec, B->cap));
  HIPCHK(hipEventRecord(B->ev[1], B->cap));
  HIPCHK(hipStreamWaitEvent(B->st, B->ev[1], 0));
  HIPCHK(hipStreamSynchronize(B->st));
  return NNCP_OK;
}

int nncp_batch_stats(const nncp_batch* B, int* launches, int64_t* items) {
  if (!B) return NNCP_EINVAL;
  if (launches) *launches = (int)B->launches.size();
  if (items) *items = (int64_t)B->n_items;
  return NNCP_OK;
}

int nncp_batch_captures(const nncp_batch* B, int64_t* captures, int64_t* list_updates) {
  if (!B) return NNCP_EINVAL;
  if (captures) *captures = B->captures;
  if (list_updates) *list_updates = B->list_updates;
  return NNCP_OK;
}

int nncp_batch_build_time(const nncp_batch* B, double* rebuild_s, double* graph_s) {
  if (!B) return NNCP_EINVAL;
  if (rebuild_s) *rebuild_s = B->rebuild_s;
  if (graph_s) *graph_s = B->graph_s;
  return NNCP_OK;
}

int nncp_batch_destroy(nncp_batch* B) {
  if (!B) return NNCP_EINVAL;
  batch_drop_graph(B);
  if (B->d_ops) hipFree(B->d_ops);
  if (B->d_items) hipFree(B->d_items);
  if (B->d_grp) hipFree(B->d_grp);
  if (B->cap) hipStreamDestroy(B->cap);
  for (auto& e : B->ev)
    if (e) hipEventDestroy(e);
  delete B;
  return NNCP_OK;
}

int nncp_plan_fits(nncp_plan* P, double* fit, int cap, int* count) {
  if (!P || !count || cap < 0 || (cap > 0 && !fit)) return NNCP_EINVAL;
  int it = 0;
  hipStream_t s = P->user_stream;
  HIPCHK(hipMemcpyAsync(&it, P->iter(), sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  *count = it;
  const int n = std::min(std::min(it, cap), kFitCap);
  if (n > 0) {
    HIPCHK(hipMemcpyAsync(fit, P->fit(), sizeof(double) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  return NNCP_OK;
}

}  // extern "C"
