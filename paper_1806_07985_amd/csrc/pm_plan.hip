// Tile and split-K plan of a partial-MTTKRP launch, and dispatch by tensor dtype.
#include <cmath>
#include <mutex>
#include <vector>

#include "pm_common.hpp"

namespace nncpk {

static int num_cus() {
  static int n = [] {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      return 256;
    return cus;
  }();
  return n;
}

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Work-groups a launch aims for: one per CU at most (measured on the 128^4
// rank-32 workload, one group of four waves per CU, each with three k-steps of
// loads in flight, streams X faster than two or three co-resident groups, and
// it keeps the split-K partial traffic small), and at least wg_kib KiB of X per
// group, so a small tensor is not cut into tiles whose LDS staging outweighs
// their share of X. The count depends on the job alone.
static int64_t target_wgs(int64_t x_bytes, int wg_kib) {
  const int64_t per = (int64_t)(wg_kib > 0 ? wg_kib : 256) * 1024;
  int64_t t = x_bytes / per;
  if (t < 1) t = 1;
  if (t > num_cus()) t = num_cus();
  return t;
}

// LDS budget of the i1 block of H_1: FP32 rows in ~48 KB (two groups may share a
// CU; `wide`: 140 KB, one group per CU; `xs`: 96 KB beside the X staging tiles),
// or the 16-bit term rows in up to 128 KB (two terms) or 150 KB (three terms;
// one group per CU).
static int lds_rows(int dtype, int RP, int ks, bool wide = false, bool xs = false, bool jone = false) {
  const bool f32 = dtype == NNCP_F32;
  const int row_bytes = f32 ? RP * 4 : RP * 2 * pm16_terms(dtype);
  const int budget = f32 ? (xs ? 96 * 1024 : (wide ? 140 * 1024 : (jone ? 72 * 1024 : 48 * 1024)))
                         : (pm16_terms(dtype) == 2 ? 128 * 1024 : 150 * 1024);
  int maxrows = budget / row_bytes / ks * ks;
  return maxrows < ks ? ks : maxrows;
}

static size_t lds_for(int dtype, int RP, int i1blk, int jblk) {
  if (dtype == NNCP_F32) return (size_t)RP * (i1blk + 4) * sizeof(float) + 8 + (size_t)jblk * RP * sizeof(double);
  return (size_t)pm16_terms(dtype) * RP * (i1blk + 8) * sizeof(unsigned short) + (size_t)jblk * RP * sizeof(float);
}

// Most j values whose per-(j, column) scales fit in LDS beside an i1 block of
// i1blk rows, at most `lim`: a 16-bit or wide FP32 group never asks for more
// than kPmMaxLds, an xs group for more than kPmMaxLds less its staging tiles
// (xs_tiles bytes), another FP32 group for more than half of it (two FP32
// groups share a CU).
static int jblk_cap(int dtype, int RP, int i1blk, int lim = 64, bool wide = false, size_t xs_tiles = 0) {
  const size_t maxl = xs_tiles ? kPmMaxLds - xs_tiles : ((dtype == NNCP_F32 && !wide) ? kPmMaxLds / 2 : kPmMaxLds);
  const size_t base = lds_for(dtype, RP, i1blk, 0);
  const size_t per = lds_for(dtype, RP, i1blk, 1) - base;
  const int64_t cap = base >= maxl ? 0 : (int64_t)((maxl - base) / per);
  return cap < lim ? (int)cap : lim;
}

// xs: plan the FP32 right node's LDS-staged form; the result has xs == 0 when
// the shape does not suit it (the caller then plans the direct form).
static PmLaunch plan_impl(int side, int dtype, int64_t IL, int64_t IR, int I1, int R, int wg_kib, bool xs) {
  PmLaunch L{};
  L.side = side;
  L.dtype = dtype;
  const int Rc = R < kPmMaxCols ? R : kPmMaxCols;
  L.nb = Rc <= 16 ? 1 : (Rc <= 32 ? 2 : 4);
  const int RP = 16 * L.nb;
  const bool f32 = dtype == NNCP_F32;
  xs = xs && f32 && side == 1 && I1 % pm_f32_kstep(1, true) == 0 && pm_f32_xs_ok(IL, L.nb);
  L.xs = xs ? 1 : 0;
  const size_t xs_tiles = xs ? pm_f32_xs_tile_lds(L.nb) : 0;
  const int64_t Mtot = side == 0 ? IL : IR;
  const int64_t Ktot = side == 0 ? IR : IL;
  const int ks = f32 ? pm_f32_kstep(side, xs) : pm_16_kstep(side);
  // a tall 16-bit right node with J == 1 uses the specialised kernel (wider waves)
  L.j1 = (!f32 && side == 1 && Ktot / I1 == 1 && cdiv(Mtot, 4 * pm_16_wave_rows(1, L.nb, 1)) >= 64) ? 1 : 0;
  const int wave_rows = f32 ? pm_f32_wave_rows(side, L.nb, xs) : pm_16_wave_rows(side, L.nb, L.j1);
  const int64_t target = target_wgs(IL * IR * (f32 ? 4 : 2), wg_kib);

  L.I1 = I1;
  L.J = Ktot / I1;
  L.I1pad = (int)cdiv(I1, ks) * ks;
  // (an FP32 launch with J == 1 keeps one j of scales: its H_1 block may take 72 KB)
  int maxrows = lds_rows(dtype, RP, ks, false, xs, L.J == 1);
  // An FP32 right node whose whole first contracted mode fits one CU's LDS but
  // not half of it takes the CU alone (wide): one i1 block, so no restaging
  // of LDS and no split K across i1 blocks (1024^3: the right node 1.18 ->
  // 1.06 ms). Where two blocks or more remain, two groups per CU are faster.
  L.wide = 0;
  if (!xs && f32 && side == 1 && (int)cdiv(I1, ks) * ks > maxrows &&
      (int)cdiv(I1, ks) * ks <= lds_rows(dtype, RP, ks, true)) {
    L.wide = 1;
    maxrows = lds_rows(dtype, RP, ks, true);
  }
  L.n_i1blk = (int)cdiv(L.I1pad, maxrows);
  L.i1blk = (int)cdiv(cdiv(L.I1pad, L.n_i1blk), ks) * ks;
  L.n_i1blk = (int)cdiv(L.I1pad, L.i1blk);

  // waves along M per group: four, unless the output is short; a left node
  // whose one-wave M tiles alone fill the GPU takes one wave along M and its
  // four waves split K inside the group (no split-K partials, no reduction)
  int wm = 4;
  if (cdiv(Mtot, 4 * wave_rows) < 64) wm = 1;
  if (side == 0 && cdiv(Mtot, wave_rows) >= target) wm = 1;
  if (L.j1) wm = 4;
  L.wm = wm;
  L.mtile = wm * wave_rows;
  L.mtiles = (int)cdiv(Mtot, L.mtile);

  // A right node with a tall output and several i1 blocks walks the blocks
  // inside each work-group (restaging LDS) instead of splitting K: the split-K
  // partials of a tall output would cost more HBM traffic than X.
  L.istages = 1;
  if (side == 1 && wm == 4 && L.n_i1blk > 1 && L.mtiles >= target) L.istages = L.n_i1blk;
  // the xs form has four waves along M and one i1 block per group
  if (xs && (wm != 4 || L.istages != 1)) {
    L.xs = 0;
    return L;
  }
  const int n_i1grp = L.n_i1blk / L.istages;

  // Many short tiles (one i1 block, at least as many four-wave tiles as the
  // target group count): four waves along M, and each group streams several
  // consecutive tiles, so a wave keeps its loads in flight across tile
  // boundaries and the group stages H_1 and the scales once for all of them,
  // instead of a group per tile whose few k-steps per wave are mostly load
  // latency.
  L.mper = 1;
  {
    const int64_t t4 = cdiv(Mtot, 4 * wave_rows);
    if (!L.j1 && L.n_i1blk == 1 && t4 >= target) {
      wm = 4;
      L.mtile = 4 * wave_rows;
      L.mtiles = (int)t4;
      L.mper = (int)cdiv(t4, target);
    } else if (L.j1 && L.istages == 1 && L.mtiles >= target && L.nb < 4) {
      // (the J == 1 kernel at four column blocks has no registers to spare for it)
      L.mper = (int)cdiv(L.mtiles, target);
    }
  }
  L.wm = wm;
  L.mgroups = (int)cdiv(L.mtiles, L.mper);

  const int64_t steps_per_j = L.i1blk / ks;
  int64_t want_splits = target / L.mgroups;
  if (want_splits < 1) want_splits = 1;
  // never more groups than the target: a second partial round of groups (one
  // group fills a CU's LDS) would double the kernel's time for a few groups
  int64_t n_jblk = want_splits / n_i1grp;
  if (n_jblk < 1) n_jblk = 1;
  // each wave should own a few k-steps, and the per-(j, column) scales fit LDS
  const int64_t min_j = cdiv(8 * (4 / wm), steps_per_j);
  int64_t jblk = cdiv(L.J, n_jblk < 1 ? 1 : n_jblk);
  if (jblk < min_j) jblk = min_j;
  // at most 64 j per group (a group's scales are a prologue of jblk * RP
  // values: copied from the launch's table, or computed where there is none),
  // or 128 for an FP32 launch that still has two rounds of groups or more with
  // it (the 64^5 left node: 4096 -> 2048 groups, 0.85 -> 0.76 ms; fewer groups
  // than that would leave CUs unevenly loaded), unless that leaves a few groups
  // beyond the target -- a second, mostly idle round for a 16-bit kernel (one
  // group per CU): then up to 128
  int jlim = 64;
  if (f32 && L.mgroups * n_i1grp * cdiv(L.J, jblk_cap(dtype, RP, L.i1blk, 128, L.wide, xs_tiles)) >= 2 * 2 * target)
    jlim = 128;
  if (jblk > jblk_cap(dtype, RP, L.i1blk, jlim, L.wide, xs_tiles)) {
    const int64_t over = L.mgroups * n_i1grp * cdiv(L.J, jblk_cap(dtype, RP, L.i1blk, jlim, L.wide, xs_tiles));
    const int64_t room = target / (L.mgroups * n_i1grp);
    if (dtype != NNCP_F32 && over > target && over < 2 * target && room >= 1 &&
        cdiv(L.J, room) <= jblk_cap(dtype, RP, L.i1blk, 128, L.wide, xs_tiles))
      jblk = cdiv(L.J, room);
    else
      jblk = jblk_cap(dtype, RP, L.i1blk, jlim, L.wide, xs_tiles);
  }
  if (jblk > L.J) jblk = L.J;
  if (jblk < 1) jblk = 1;
  L.jblk = (int)jblk;
  // FP32 partial sums span `fold` k-steps (fold*ks products) before they are
  // added into FP64. A running FP32 sum of c products over a reduction of K
  // terms leaves a relative error of about 0.3 u c / sqrt(3 K) once the chunks
  // are summed exactly; fold keeps c <= 0.6 sqrt(3 K), i.e. under ~0.2 u.
  // (The 16-bit kernels add each j's FP32 sum into FP32 accumulators.)
  {
    const double cmax = 0.6 * std::sqrt(3.0 * (double)Ktot);
    int fmax = (int)(cmax / ks);
    if (fmax < 1) fmax = 1;
    int f = 1;
    for (int d = 1; d <= steps_per_j && d <= fmax; ++d)
      if (steps_per_j % d == 0) f = d;
    L.fold = f;
  }
  L.n_jblk = (int)cdiv(L.J, jblk);
  L.nsplit = n_i1grp * L.n_jblk;
  L.lds_bytes = lds_for(dtype, RP, L.i1blk, L.jblk) + xs_tiles;
  L.pack_bytes =
      f32 ? 0 : (size_t)pm16_terms(dtype) * RP * L.I1pad * sizeof(unsigned short) + 256 + (size_t)RP * sizeof(float);
  L.partial_doubles = L.nsplit > 1 ? (size_t)L.nsplit * RP * (size_t)L.mtiles * L.mtile : 0;
  L.ncounters = L.mtiles;
  return L;
}

PmLaunch pm_plan(int side, int dtype, int64_t IL, int64_t IR, int I1, int R, int wg_kib) {
  if (dtype == NNCP_F32 && side == 1) {
    const PmLaunch L = plan_impl(side, dtype, IL, IR, I1, R, wg_kib, true);
    if (L.xs) return L;
  }
  return plan_impl(side, dtype, IL, IR, I1, R, wg_kib, false);
}

void pm_fill_args(const PmLaunch& L, PmArgs& a) {
  a.I1 = L.I1;
  a.I1pad = L.I1pad;
  a.i1blk = L.i1blk;
  a.n_i1blk = L.n_i1blk;
  a.J = L.J;
  a.jblk = L.jblk;
  a.n_jblk = L.n_jblk;
  a.fold = L.fold;
  a.nsplit = L.nsplit;
  a.istages = L.istages;
  a.wm = L.wm;
  a.mtiles = L.mtiles;
  a.mper = L.mper;
}

size_t pm_variant_max_lds(int kind, int variant) {
  const bool f32 = kind == K_PM_F32;
  const int dtype = f32 ? NNCP_F32 : (((variant / 10000) % 10) ? NNCP_BF16 : NNCP_F16);
  const int side = (variant / 1000) % 10, nb = (variant / 100) % 10;
  const bool wide = f32 && (variant / 10000) % 10;
  const bool xs = f32 && (variant / 100000) % 10;
  const size_t xs_tiles = xs ? pm_f32_xs_tile_lds(nb) : 0;
  const int RP = 16 * nb;
  const int ks = f32 ? pm_f32_kstep(side, xs) : pm_16_kstep(side);
  size_t lds = 0;
  for (int rows = ks; rows <= lds_rows(dtype, RP, ks, wide, xs); rows += ks) {
    const size_t b = lds_for(dtype, RP, rows, jblk_cap(dtype, RP, rows, 128, wide, xs_tiles)) + xs_tiles;
    if (b > lds) lds = b;
  }
  // launches with J == 1: one j of scales beside a possibly larger H_1 block
  for (int rows = ks; rows <= lds_rows(dtype, RP, ks, wide, xs, true); rows += ks) {
    const size_t b = lds_for(dtype, RP, rows, 1) + xs_tiles;
    if (b > lds) lds = b;
  }
  const size_t red = f32 ? pm_f32_reduce_lds(side, nb, 1) : pm_16_reduce_lds(side, nb, 1);
  return lds > red ? lds : red;
}

void pm_allow_lds(const void* k, size_t bytes) {
  static std::mutex mu;
  static std::vector<const void*> done;
  std::lock_guard<std::mutex> lk(mu);
  for (const void* d : done)
    if (d == k) return;
  if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess)
    (void)hipGetLastError();
  done.push_back(k);
}

hipError_t pm_launch(const PmLaunch& L, const PmArgs& a, const Sink& sk) {
  hipError_t e = (L.dtype == NNCP_F32) ? pm_launch_f32(L, a, sk) : pm_launch_16(L, a, sk);
  if (e != hipSuccess || L.nsplit <= 1) return e;
  ReduceArgs r{};
  r.part = a.partial;
  r.T = a.T;
  r.t_f64 = a.t_f64;
  r.Mtot = L.side == 0 ? a.IL : a.IR;
  r.Mpad = (int64_t)L.mtiles * L.mtile;
  r.RP = 16 * L.nb;
  r.R = a.R;
  r.col0 = a.col0;
  r.nsplit = L.nsplit;
  return pm_reduce_launch(r, sk);
}

hipError_t pm_launch(const PmLaunch& L, const PmArgs& a, hipStream_t st) {
  Sink sk;
  sk.st = st;
  return pm_launch(L, a, sk);
}

}  // namespace nncpk
