// Host-side check of the partial-MTTKRP kernels' addressing (test
// infrastructure, not part of the library). For the plan nncpk::pm_plan makes
// for a shape, it walks every work-group, wave, lane and vector or element load
// the kernels issue (including the loads a wave prefetches past the end of its
// range, and a group's walk over several M tiles and i1 stages) and every
// output row they store, the way pm_kernels.hip and pm16_body.hpp compute the
// addresses, and counts elements that fall outside the tensor or the output.
// The tile geometry below (rows per wave, k-step, loads in flight) mirrors the
// kernels' constants.
//
// stdin: one case per line, "dtype IL IR I1_left I1_right R" (dtype 0 FP32,
// 1 BF16, 2 FP16); stdout: one line per case, then a summary; exit status 1 if
// any access is out of bounds.
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <vector>
#include "nncp_internal.hpp"
using namespace nncpk;

static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
static long long bad = 0, nchk = 0;
static void chk(int64_t e, int64_t n, const char* what) {
  ++nchk;
  if (e < 0 || e >= n) { if (bad < 5) printf("  OOB %s: %lld of %lld\n", what, (long long)e, (long long)n); ++bad; }
}
static void wave_range(int n, int wk, int WK, int* b, int* e) {
  const int per = (n + WK - 1) / WK;
  *b = wk * per < n ? wk * per : n;
  *e = (wk + 1) * per < n ? (wk + 1) * per : n;
}

// side 0: left. f32: KS=16, TR, lanes load 4 columns (4lq+u) TR rows; 16-bit: KS=32, 8 columns (8lq+e).
static void emu_left(const PmLaunch& L, int64_t IL, int64_t IR, bool f32, bool fast) {
  const int nb = L.nb;
  // rows per lane and k-step from the library; columns per lane load and k-steps
  // in flight as in the kernels
  const int TR = (f32 ? pm_f32_wave_rows(0, nb) : pm_16_wave_rows(0, nb)) / 16;
  const int KS = f32 ? pm_f32_kstep(0) : pm_16_kstep(0);
  const int NCOL = f32 ? 4 : 8, D = f32 ? (nb == 2 ? 3 : 4) : 3;
  const int WM = L.wm, WK = 4 / WM, WROWS = 16 * TR;
  const int64_t Mtot = IL, Ktot = IR, I = IL * IR;
  const int64_t vec_lim = Mtot * Ktot - (TR - 1);
  if (L.mtile != WM * WROWS || (L.mper > 1 && WM != 4)) { printf("  bad tile geometry\n"); ++bad; }
  const int64_t Mpad = (int64_t)L.mtiles * L.mtile;
  for (int by = 0; by < L.nsplit; ++by)
    for (int bx = 0; bx < L.mgroups; ++bx)
      for (int wave = 0; wave < 4; ++wave) {
        const int wm = wave % WM, wk = wave / WM;
        const int tile0 = bx * L.mper, ntile = std::min(L.mper, L.mtiles - tile0);
        if (ntile < 1) { printf("  empty group\n"); ++bad; continue; }
        int tileL = 0;
        int64_t mw = (int64_t)tile0 * L.mtile + wm * WROWS;
        const int ib = by % L.n_i1blk, jb = by / L.n_i1blk;
        const int i1_0 = ib * L.i1blk;
        const int i1n = std::min(L.i1blk, L.I1pad - i1_0);
        const int64_t j0 = (int64_t)jb * L.jblk;
        const int jn = (int)std::min((int64_t)L.jblk, L.J - j0);
        if (jn <= 0) { printf("  empty j block\n"); ++bad; continue; }
        const int S1 = i1n / KS;
        int sb, se;
        wave_range(S1 * jn, wk, WK, &sb, &se);
        se += (ntile - 1) * S1 * jn;
        const int jrot = (WK == 1 && jn > 1) ? (int)(((unsigned)bx * 5u) % (unsigned)jn) : 0;
        int jcntL = sb / S1;
        int jl = jcntL + jrot, tl = sb - jcntL * S1;
        if (jl >= jn) jl -= jn;
        // stores of every tile of the group (wave wk == 0)
        if (wk == 0)
          for (int t = 0; t < ntile; ++t)
            for (int lane = 0; lane < 64; ++lane) {
              const int lq = lane >> 4;
              for (int v = 0; v < 4; ++v) {
                const int64_t m0 = (int64_t)(tile0 + t) * L.mtile + wm * WROWS + TR * (4 * lq + v);
                chk(m0 + TR - 1, Mpad, "store");
              }
            }
        const int ilim = L.I1 - i1_0;
        // number of load calls: D initial + one per computed step in the main loop
        int nloads = D;
        { int s = sb; for (; s + D - 1 < se; s += D) nloads += D; }
        for (int q = 0; q < nloads; ++q) {
          const int64_t colbase = (int64_t)L.I1 * (j0 + jl) + i1_0 + KS * tl;
          const bool vec = fast || Mtot * (colbase + KS) <= vec_lim;
          for (int lane = 0; lane < 64; ++lane) {
            const int li = lane & 15, lq = lane >> 4;
            const int64_t m = mw + TR * li, mload = m < Mtot ? m : 0;
            for (int u = 0; u < NCOL; ++u) {
              const int64_t col = colbase + NCOL * lq + u;
              if (vec) { chk(Mtot * col + mload, I, "vec lo"); chk(Mtot * col + mload + TR - 1, I, "vec hi"); }
              else {
                const bool kv = (KS * tl + NCOL * lq + u) < ilim;
                for (int e = 0; e < TR; ++e) if (kv && m + e < Mtot) chk(Mtot * col + m + e, I, "elem");
              }
            }
          }
          if (++tl == S1) { tl = 0; if (++jl == jn) jl = 0;
            if (++jcntL == jn) { jcntL = 0; if (++tileL == ntile) tileL = 0; mw = (int64_t)(tile0 + tileL) * L.mtile + wm * WROWS; } }
        }
      }
}

static void emu_right(const PmLaunch& L, int64_t IL, int64_t IR, bool f32, bool fast) {
  const int nb = L.nb;
  // column groups per wave and k-step from the library; lane vector width and
  // k-steps in flight as in the kernels
  const int MC = (f32 ? pm_f32_wave_rows(1, nb) : pm_16_wave_rows(1, nb, L.j1)) / 16;
  const int KS = f32 ? pm_f32_kstep(1) : pm_16_kstep(1), VW = f32 ? 4 : 8, HS = KS / 2;
  const int D = f32 ? 3 : (L.j1 ? (nb >= 4 ? 2 : 3) : 3);
  const int WM = L.wm, WK = 4 / WM;
  const int64_t Mtot = IR, Ktot = IL, I = IL * IR;
  const int n_i1grp = L.n_i1blk / L.istages;
  if (L.mtile != WM * 16 * MC || (L.mper > 1 && (WM != 4 || L.istages != 1))) { printf("  bad tile geometry\n"); ++bad; }
  const int64_t Mpad = (int64_t)L.mtiles * L.mtile;
  for (int by = 0; by < L.nsplit; ++by)
    for (int bx = 0; bx < L.mgroups; ++bx)
      for (int wave = 0; wave < 4; ++wave) {
        const int wm = wave % WM, wk = wave / WM;
        const int tile0 = bx * L.mper, ntile = std::min(L.mper, L.mtiles - tile0);
        if (ntile < 1) { printf("  empty group\n"); ++bad; continue; }
        int tileL = 0;
        int64_t cw = (int64_t)tile0 * L.mtile + wm * 16 * MC;
        const int ib0 = (by % n_i1grp) * L.istages, jb = by / n_i1grp;
        const int64_t j0 = (int64_t)jb * L.jblk;
        const int jn = (int)std::min((int64_t)L.jblk, L.J - j0);
        auto stage_rows = [&](int st) { return std::min(L.i1blk, L.I1pad - (ib0 + st) * L.i1blk); };
        int total = 0;
        for (int st = 0; st < L.istages; ++st) total += (stage_rows(st) / KS) * jn;
        int sb, se;
        wave_range(total, wk, WK, &sb, &se);
        se += (ntile - 1) * total;
        int64_t cmax = std::min(cw + 16 * MC - 1, Mtot - 1);
        int64_t vec_lim = Mtot * Ktot - Ktot * cmax - KS;
        if (wk == 0)
          for (int t = 0; t < ntile; ++t)
            for (int lane = 0; lane < 64; ++lane) {
              const int lq = lane >> 4;
              for (int g = 0; g < MC; ++g) {
                const int64_t m0 = (int64_t)(tile0 + t) * L.mtile + wm * 16 * MC + 16 * g + 4 * lq;
                chk(m0 + 3, Mpad, "rstore");
              }
            }
        const int jrot = (WK == 1 && jn > 1) ? (int)(((unsigned)bx * 5u) % (unsigned)jn) : 0;
        int stL = 0, S1L = stage_rows(0) / KS;
        int jcntL = sb / S1L, tl = sb - jcntL * S1L, jl = jcntL + jrot;
        if (jl >= jn) jl -= jn;
        int nloads = D;
        { int s = sb; for (; s + D - 1 < se; s += D) nloads += D; }
        for (int q = 0; q < nloads; ++q) {
          const int i1s = (ib0 + stL) * L.i1blk;
          const int64_t lbase = (int64_t)L.I1 * (j0 + jl) + i1s + KS * tl;
          const bool vec = fast || lbase <= vec_lim;
          const int ilimL = L.I1 - i1s;
          for (int lane = 0; lane < 64; ++lane) {
            const int li = lane & 15, lq = lane >> 4;
            for (int g = 0; g < MC; ++g) {
              const int64_t c = cw + 16 * g + li, cc = c < Mtot ? c : 0;
              const int64_t colp = Ktot * cc + VW * lq;
              for (int h = 0; h < 2; ++h) {
                if (vec) { chk(colp + lbase + HS * h, I, "rvec lo"); chk(colp + lbase + HS * h + VW - 1, I, "rvec hi"); }
                else {
                  const int off = KS * tl + HS * h + VW * lq;
                  for (int e = 0; e < VW; ++e) if (off + e < ilimL) chk(colp + lbase + HS * h + e, I, "relem");
                }
              }
            }
          }
          if (++tl == S1L) { tl = 0; if (++jl == jn) jl = 0; if (++jcntL == jn) { jcntL = 0;
              if (++stL == L.istages) { stL = 0;
                if (ntile > 1) { if (++tileL == ntile) tileL = 0; cw = (int64_t)(tile0 + tileL) * L.mtile + wm * 16 * MC;
                  cmax = std::min(cw + 16 * MC - 1, Mtot - 1); vec_lim = Mtot * Ktot - Ktot * cmax - KS; } }
              S1L = stage_rows(stL) / KS; } }
        }
      }
}

// The FP32 right node's LDS-staged (xs) form: load instruction i of a step reads
// column cw + 4i + lq at k offset 4li, 64 k per step; each wave writes its tile
// [16 MC columns][kXsRow] after the H_1 block and the scales, and reads it back
// at column 16g + li, k 16h + 4lq. B operands: H_1 rows of the step's k.
static void emu_right_xs(const PmLaunch& L, int64_t IL, int64_t IR) {
  const int nb = L.nb, RP = 16 * nb;
  const int MC = pm_f32_wave_rows(1, nb, true) / 16;
  const int KS = pm_f32_kstep(1, true), ROW = KS + 4, D = 3, NI = 4 * MC;
  const int64_t Mtot = IR, Ktot = IL, I = IL * IR;
  if (L.wm != 4 || L.istages != 1 || L.I1 % KS != 0 || L.mtile != 4 * 16 * MC) { printf("  bad xs geometry\n"); ++bad; return; }
  // LDS: H_1 block, scales, four tiles
  const int hp = L.i1blk + 4;
  const int64_t xt0 = (int64_t)RP * hp * 4 + (int64_t)L.jblk * RP * 8;  // bytes
  const int64_t tile_bytes = (int64_t)16 * MC * ROW * 4;
  chk(xt0 + 4 * tile_bytes - 1, (int64_t)L.lds_bytes, "xs lds");
  chk((int64_t)L.lds_bytes - 1, (int64_t)kPmMaxLds, "xs lds max");
  if (xt0 % 16) { printf("  xs tile misaligned\n"); ++bad; }
  for (int lane = 0; lane < 64; ++lane) {
    const int li = lane & 15, lq = lane >> 4;
    for (int i = 0; i < NI; ++i) {
      chk((4 * i + lq) * ROW + 4 * li, 16 * MC * ROW, "xs stage lo");
      chk((4 * i + lq) * ROW + 4 * li + 3, 16 * MC * ROW, "xs stage hi");
    }
    for (int g = 0; g < MC; ++g)
      for (int h = 0; h < 4; ++h) chk((16 * g + li) * ROW + 16 * h + 4 * lq + 3, 16 * MC * ROW, "xs read");
  }
  const int64_t Mpad = (int64_t)L.mtiles * L.mtile;
  for (int by = 0; by < L.nsplit; ++by)
    for (int bx = 0; bx < L.mgroups; ++bx)
      for (int wave = 0; wave < 4; ++wave) {
        const int tile0 = bx * L.mper, ntile = std::min(L.mper, L.mtiles - tile0);
        if (ntile < 1) { printf("  empty group\n"); ++bad; continue; }
        const int ib = by % L.n_i1blk, jb = by / L.n_i1blk;
        const int i1_0 = ib * L.i1blk;
        const int i1n = std::min(L.i1blk, L.I1pad - i1_0);
        const int64_t j0 = (int64_t)jb * L.jblk;
        const int jn = (int)std::min((int64_t)L.jblk, L.J - j0);
        if (jn <= 0 || i1n % KS) { printf("  bad xs block\n"); ++bad; continue; }
        const int S1 = i1n / KS;
        const int se = ntile * S1 * jn;
        for (int t = 0; t < ntile; ++t)
          for (int lane = 0; lane < 64; ++lane) {
            const int lq = lane >> 4;
            for (int g = 0; g < MC; ++g)
              chk((int64_t)(tile0 + t) * L.mtile + wave * 16 * MC + 16 * g + 4 * lq + 3, Mpad, "xs store");
          }
        const int jrot = jn > 1 ? (int)(((unsigned)bx * 5u) % (unsigned)jn) : 0;
        int tileL = 0, jcntL = 0, tl = 0, jl = jrot;
        int64_t cw = (int64_t)tile0 * L.mtile + wave * 16 * MC;
        // D loads, one more for step D, then one for each step that has a successor
        const int nloads = D + se;
        for (int q = 0; q < nloads; ++q) {
          // buffer loads: base e0 (the step's first element of the wave's first
          // column), range min(I - e0, 2^30 - 1) elements, lane offset
          // (4i + lq) Ktot + 4li; reads at or past the range return zeros
          const int64_t e0 = Ktot * cw + (int64_t)L.I1 * (j0 + jl) + i1_0 + KS * tl;
          const int64_t rem = I - e0;
          const int64_t nrec = rem <= 0 ? 0 : std::min<int64_t>(rem, 0x3fffffff);
          for (int lane = 0; lane < 64; ++lane) {
            const int li = lane & 15, lq = lane >> 4;
            for (int i = 0; i < NI; ++i) {
              const int64_t c = cw + 4 * i + lq;
              const int64_t off = (int64_t)(4 * i + lq) * Ktot + 4 * li;
              chk(off * 4 + 15, (int64_t)1 << 31, "xs voffset");
              if (off + 3 < nrec) { chk(e0 + off, I, "xs vec lo"); chk(e0 + off + 3, I, "xs vec hi"); }
              else if (off < nrec) { printf("  xs load straddles the range\n"); ++bad; }
              if (c < Mtot && !(off + 3 < nrec)) { printf("  xs load of a real column suppressed\n"); ++bad; }
            }
          }
          if (++tl == S1) { tl = 0; if (++jl == jn) jl = 0;
            if (ntile > 1 && ++jcntL == jn) { jcntL = 0; if (++tileL == ntile) tileL = 0;
              cw = (int64_t)(tile0 + tileL) * L.mtile + wave * 16 * MC; } }
        }
      }
}

static int run_case(int dt, int64_t IL, int64_t IR, int I1l, int I1r, int R) {
  const bool f32 = dt == 0;
  const long long bad0 = bad;
  for (int side = 0; side < 2; ++side) {
    const int Rc = std::min(R, 64);
    PmLaunch L = pm_plan(side, dt, IL, IR, side == 0 ? I1l : I1r, Rc, 0);
    if ((int64_t)L.mgroups * L.nsplit * 64 * 4 > 400000000LL) continue;  // too large to walk here
    const int I1 = side == 0 ? I1l : I1r;
    const bool fast = f32 ? pm_f32_fast(side, IL, I1, L.nb, L.xs) : pm16_fast(side, IL, I1, L.nb);
    if (side == 0) emu_left(L, IL, IR, f32, fast);
    else if (L.xs) emu_right_xs(L, IL, IR);
    else emu_right(L, IL, IR, f32, fast);
    {
      // a batched launch of this plan's kernel variant reserves at least the
      // plan's LDS (the variant's maximum over every plan it can run)
      const int kind = f32 ? K_PM_F32 : K_PM_16;
      const int var = f32 ? (L.xs ? 100000 : 0) + (L.wide ? 10000 : 0) + side * 1000 + L.nb * 100
                          : (L.j1 ? 100000 : 0) + (dt == NNCP_BF16 ? 10000 : 0) + side * 1000 + L.nb * 100;
      chk((int64_t)L.lds_bytes - 1, (int64_t)pm_variant_max_lds(kind, var), "batch variant lds");
    }
    if (!f32 && side == 1) {
      // 16-bit right node: the staged factor terms (RP columns each, pitch
      // i1blk + 8) and the j block's scales, as the kernel lays them out, fit
      // the launch's LDS
      const int RP = 16 * L.nb;
      const int64_t need = (int64_t)pm16_terms(dt) * RP * (L.i1blk + 8) * 2 + (int64_t)L.jblk * RP * 4;
      chk(need - 1, (int64_t)L.lds_bytes, "16-bit right lds");
      chk((int64_t)L.lds_bytes - 1, (int64_t)kPmMaxLds, "lds max");
    }
  }
  return bad == bad0 ? 0 : 1;
}

int main() {
  int dt, I1l, I1r, R;
  long long IL, IR;
  int cases = 0, failed = 0;
  while (scanf("%d %lld %lld %d %d %d", &dt, &IL, &IR, &I1l, &I1r, &R) == 6) {
    ++cases;
    const int f = run_case(dt, IL, IR, I1l, I1r, R);
    failed += f;
    printf("%s dtype %d IL %lld IR %lld I1 %d/%d R %d\n", f ? "FAIL" : "ok", dt, IL, IR, I1l, I1r, R);
  }
  printf("%d cases, %lld accesses checked, %lld out of bounds, %d cases failed\n", cases, nchk, bad, failed);
  return failed ? 1 : 0;
}
