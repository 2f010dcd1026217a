// Partial MTTKRP on MFMA for FP32 tensors: the root edges of the dimension tree
// (Section IV-A, Figure 2a), T = X_[L] * K (left node {1..s}) or
// T = X_[L]^T * K (right node {s+1..N}), where X_[L] is the tensor viewed as the
// column-major I_L x I_R matrix and K the Khatri-Rao product of the other
// side's factors (first contracted mode fastest).
//
// Design (gfx950, wave64):
//  * The reduction index is split as k = i1 + I1*j (i1: first contracted mode).
//    K(k, :) = H_1(i1, :) * Krest(j, :), so a work-group keeps the H_1 rows of
//    its i1 block in LDS (the MFMA B operand), and applies Krest(j, :) as a
//    per-column factor when it folds the FP32 MFMA sums into FP64 accumulators
//    (one v_fma_f64 per output). The Khatri-Rao product is never formed.
//  * X streams from HBM straight into VGPRs with vector loads (8 or 16 bytes per
//    lane), several k-steps ahead of the MFMAs (v_mfma_f32_16x16x4_f32), for any
//    shape: a load of padded i1 (>= I1) reads the next j's columns, which meet
//    zero rows of H_1 in LDS; a load of rows past the output reads into the next
//    column and only feeds outputs that are never stored. The one k-step that
//    could read past the end of the tensor loads element by element.
//  * Precision: each MFMA chain covers at most `fold` k-steps (16 or 32 products
//    per output each) before it is added into FP64; split-K partials, the
//    cross-wave reduction and the output are FP64.
//  * Split-K over (i1 block, j block) pairs: each work-group writes an FP64
//    partial; a separate reduction kernel sums them in split order, so results
//    do not depend on scheduling and no cross-XCD fence is needed. A right node
//    with a tall output walks its i1 blocks inside the work-group instead
//    (restaging LDS), so it writes only its output.
#include "pm_common.hpp"

namespace nncpk {
namespace {

// Rows per left wave = 16 * left_tr(NB); columns per right wave = 16 * right_mc(NB).
// Chosen so that the FP64 accumulators (2 VGPRs per output) leave room for
// several k-steps of X in flight without spilling. PF = k-steps in flight.
constexpr int left_tr(int nb) { return nb >= 4 ? 2 : 4; }
constexpr int right_mc(int nb) { return nb >= 4 ? 2 : 4; }
constexpr int left_pf(int nb) { return nb == 2 ? 3 : 4; }
constexpr int right_pf(int nb) { return 3; }

// ----------------------------------------------------------------------------
// Left side: T(m, r) = sum_k X[m + IL*k] K(k, r); m is contiguous in X.
// A wave covers 16*TR rows m. In a k-step (16 consecutive i1 of one j), lane
// (li, lq) loads rows TR*li .. TR*li+TR-1 of the columns i1 = base + 4*lq + u,
// u = 0..3; MFMA chain tt uses row TR*li + tt of every load.
// ----------------------------------------------------------------------------
template <int NB, int D, bool FAST, bool MT, bool NTL>
__device__ __forceinline__ void pm_left_f32_body(const PmArgs& a, int bx, int by) {
  constexpr int RP = NB * 16;
  constexpr int TR = left_tr(NB);
  constexpr int KS = 16;
  constexpr int NACC = TR * NB;
  constexpr int WROWS = 16 * TR;
  using vT = f32v<TR>;
  extern __shared__ double lds_d[];
  const int hp = a.i1blk + 4;
  float* hs = (float*)lds_d;
  double* sc = lds_d + (RP * hp + 1) / 2;

  const int WM = a.wm, WK = 4 / WM;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave % WM, wk = wave / WM;
  const int li = lane & 15, lq = lane >> 4;
  const int64_t Mtot = a.IL, Ktot = a.IR;
  const int mtile = WM * WROWS;
  // the group's M tiles tile0 .. tile0 + ntile - 1 (ntile > 1 only with WK == 1):
  // one continuous stream of k-steps per wave, the loads of a tile's first steps
  // issued while the previous tile's last steps are computed
  const int tile0 = MT ? bx * a.mper : bx;
  const int ntile = MT ? min(a.mper, a.mtiles - tile0) : 1;
  const int ib = by % a.n_i1blk, jb = by / a.n_i1blk;
  const int i1_0 = ib * a.i1blk;
  const int i1n = min(a.i1blk, a.I1pad - i1_0);
  const int64_t j0 = (int64_t)jb * a.jblk;
  const int jn = (int)min((int64_t)a.jblk, a.J - j0);
  const float* X = (const float*)a.X;

  pm_prologue(a, hs, hp, sc, RP, i1_0, i1n, j0, jn);
  __syncthreads();

  const int S1 = i1n / KS;
  int sb, se;
  wave_range(S1 * jn, wk, WK, &sb, &se);
  se += (ntile - 1) * S1 * jn;

  double acc[NACC][4];
#pragma unroll
  for (int v = 0; v < NACC; ++v)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[v][e] = 0.0;

  // lane's first row in the tile being loaded; a row group wholly past the
  // output reads row 0
  int64_t m = (int64_t)tile0 * mtile + wm * WROWS + TR * li;
  int64_t mload = m < Mtot ? m : 0;
  const int ilim = a.I1 - i1_0;            // lane i1 offsets >= ilim are padding
  const float* zeros = (const float*)a.zeros;
  int64_t lane_col[4];                     // lane part of the address of column (colbase + 4*lq + u)
#pragma unroll
  for (int u = 0; u < 4; ++u) lane_col[u] = Mtot * (int64_t)(4 * lq + u);
  // The vector loads of a step read elements up to Mtot * (colbase + KS) + TR - 2
  // (row group start <= Mtot - 1, TR rows, in the step's last column): all of
  // them lie inside the tensor while Mtot * (colbase + KS) <= vec_lim.
  const int64_t vec_lim = Mtot * Ktot - (TR - 1);

  // load cursor (uniform): step = jl * S1 + tl. With one wave along K the group
  // starts at a j rotated by its M tile, so groups that share a split do not all
  // request the same addresses modulo the column stride at the same time.
  const int jrot = (WK == 1 && jn > 1) ? (int)(((unsigned)bx * 5u) % (unsigned)jn) : 0;
  int jcntL = sb / S1, tileL = 0;
  int jl = jcntL + jrot, tl = sb - jcntL * S1;
  if (jl >= jn) jl -= jn;  // an empty range (sb == S1 * jn) starts at the block's first j
  // The cursor stays inside the group's j block and tiles (it wraps), so loads
  // of steps past the wave's range read valid memory and are simply not used.
  auto load = [&](vT (&A)[4]) {
    const int64_t colbase = (int64_t)a.I1 * (j0 + jl) + i1_0 + KS * tl;
    const float* base = X + Mtot * colbase;
    if (FAST || Mtot * (colbase + KS) <= vec_lim) {  // uniform
#pragma unroll
      for (int u = 0; u < 4; ++u) A[u] = tload<NTL>((const vT*)(base + lane_col[u] + mload));
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        // per lane: the whole row group of a real column in one vector load,
        // else element by element (rows past the output, padded i1: zero)
        const bool kv = (KS * tl + 4 * lq + u) < ilim;
        vT v;
        if (kv && m + TR <= Mtot) {
          v = *(const vT*)(base + lane_col[u] + m);
        } else {
#pragma unroll
          for (int e = 0; e < TR; ++e) {
            const float* p = (kv && m + e < Mtot) ? base + lane_col[u] + m + e : zeros;
            v[e] = *p;
          }
        }
        A[u] = v;
      }
    }
    if (++tl == S1) {
      tl = 0;
      if (++jl == jn) jl = 0;
      if (MT && ++jcntL == jn) {
        jcntL = 0;
        if (++tileL == ntile) tileL = 0;
        m = (int64_t)(tile0 + tileL) * mtile + wm * WROWS + TR * li;
        mload = m < Mtot ? m : 0;
      }
    }
  };

  // acc[tt*NB+nb][v]: row mw + TR*(4*lq + v) + tt, rank column 16nb + li.
  const bool direct = (a.nsplit == 1);
  const int64_t Mpad = (int64_t)a.mtiles * mtile;
  auto store_tile = [&](int64_t mw) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double o[TR];
#pragma unroll
        for (int tt = 0; tt < TR; ++tt) o[tt] = acc[tt * NB + nb][v];
        pm_store_rows<TR>(a, direct, Mtot, Mpad, RP, by, 16 * nb + li, mw + TR * (4 * lq + v), o);
      }
  };

  // FP32 partial sums (one 16x16 block per (tt, nb)) live for `fold` k-steps and
  // are then added into the FP64 accumulators with the chunk's column scale.
  f4 c32[TR][NB];
#pragma unroll
  for (int tt = 0; tt < TR; ++tt)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) c32[tt][nb] = f4{0.f, 0.f, 0.f, 0.f};
  int jc = jl, tc = tl, jcntC = jcntL, tileC = 0, fc = tl % a.fold, sc_left = se - sb;
  auto compute = [&](const vT (&A)[4]) {
    const int kk = KS * tc + 4 * lq;
    f4 B[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) B[nb] = *(const f4*)&hs[(16 * nb + li) * hp + kk];
    // u-major: consecutive MFMAs go to different accumulators
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int tt = 0; tt < TR; ++tt)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) c32[tt][nb] = mfma4(A[u][tt], B[nb][u], c32[tt][nb]);
    --sc_left;
    // fold every `fold` k-steps, at the end of each j (the last i1 block can be
    // shorter than the others, so fold need not divide its steps) and at the end
    if (++fc == a.fold || tc + 1 == S1 || sc_left == 0) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const double scl = sc[jc * RP + 16 * nb + li];
#pragma unroll
        for (int tt = 0; tt < TR; ++tt) {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            acc[tt * NB + nb][e] = __builtin_fma((double)c32[tt][nb][e], scl, acc[tt * NB + nb][e]);
          c32[tt][nb] = f4{0.f, 0.f, 0.f, 0.f};
        }
      }
      fc = 0;
    }
    if (++tc == S1) {
      tc = 0;
      if (++jc == jn) jc = 0;
      if (MT && ++jcntC == jn) {
        jcntC = 0;
        if (tileC + 1 < ntile) {  // a tile done (its last j folded above): store it, start the next
          store_tile((int64_t)(tile0 + tileC) * mtile + wm * WROWS);
#pragma unroll
          for (int v = 0; v < NACC; ++v)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[v][e] = 0.0;
          ++tileC;
        }
      }
    }
  };

  // D k-steps of X in flight: the loads of step s+D are issued right after step
  // s is consumed. sched_barrier keeps the compiler from sinking them. The first
  // D loads are issued unconditionally so every path into the loop has the same
  // loads in flight and the compiler's wait counts stay precise.
  vT A[D][4];
  int s = sb;
#pragma unroll
  for (int d = 0; d < D; ++d) load(A[d]);
  for (; s + D - 1 < se; s += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      compute(A[d]);
      __builtin_amdgcn_sched_barrier(0);
      load(A[d]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int d = 0; d < D - 1; ++d)
    if (s + d < se) compute(A[d]);

  __syncthreads();  // LDS is reused by the cross-wave reduction
  wave_reduce_k<NACC>(acc, lds_d, wk, wm, WK);
  if (wk != 0) return;
  store_tile((int64_t)(tile0 + ntile - 1) * mtile + wm * WROWS);
}

// ----------------------------------------------------------------------------
// Right side: T(c, r) = sum_k X[k + IL*c] K(k, r); k is contiguous in X.
// A wave covers MC groups of 16 columns c. In a k-step (32 consecutive i1 of
// one j), lane (li, lq) loads k = base + 16h + 4*lq + u (u = 0..3 in one
// 16-byte load, h = 0..1) of column c = group + li. The work-group walks
// `istages` i1 blocks (j inside each), restaging LDS between them; istages > 1
// only with every wave on its own columns (WM = 4).
// ----------------------------------------------------------------------------
template <int NB, int D, bool FAST, bool MT, bool NTL>
__device__ __forceinline__ void pm_right_f32_body(const PmArgs& a, int bx, int by) {
  constexpr int RP = NB * 16;
  constexpr int MC = right_mc(NB);
  constexpr int KS = 32;
  constexpr int NACC = MC * NB;
  using vT = f32v<4>;
  extern __shared__ double lds_d[];
  const int hp = a.i1blk + 4;
  float* hs = (float*)lds_d;
  double* sc = lds_d + (RP * hp + 1) / 2;

  const int WM = a.wm, WK = 4 / WM;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave % WM, wk = wave / WM;
  const int li = lane & 15, lq = lane >> 4;
  const int64_t Mtot = a.IR, Ktot = a.IL;
  const int mtile = WM * 16 * MC;
  // the group's M tiles tile0 .. tile0 + ntile - 1 (ntile > 1 only with WK == 1
  // and istages == 1), streamed as one sequence of k-steps per wave
  const int tile0 = MT ? bx * a.mper : bx;
  const int ntile = MT ? min(a.mper, a.mtiles - tile0) : 1;
  const int n_i1grp = a.n_i1blk / a.istages;
  const int ib0 = (by % n_i1grp) * a.istages, jb = by / n_i1grp;
  const int64_t j0 = (int64_t)jb * a.jblk;
  const int jn = (int)min((int64_t)a.jblk, a.J - j0);
  const float* X = (const float*)a.X;

  // stage geometry: all stages have i1blk rows except possibly the last
  auto stage_rows = [&](int st) { return min(a.i1blk, a.I1pad - (ib0 + st) * a.i1blk); };

  pm_prologue(a, hs, hp, sc, RP, ib0 * a.i1blk, stage_rows(0), j0, jn);
  __syncthreads();

  int total = 0;
  for (int st = 0; st < a.istages; ++st) total += (stage_rows(st) / KS) * jn;
  int sb, se;
  wave_range(total, wk, WK, &sb, &se);  // istages > 1 implies WK == 1: the whole range
  se += (ntile - 1) * total;

  double acc[NACC][4];
#pragma unroll
  for (int v = 0; v < NACC; ++v)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[v][e] = 0.0;

  // Columns of the tile being loaded (columns past the output read column 0).
  // The vector loads of a step read elements up to Ktot * cmax + lbase + KS - 1
  // (cmax: the wave's last column that is read, lane offsets up to KS - 1): all
  // of them lie inside the tensor while lbase <= vec_lim. Only the steps that
  // run past the end of a column near the tensor's end fail this.
  const float* colp[MC];
  int64_t vec_lim;
  auto set_tile = [&](int t) {
    const int64_t cw = (int64_t)(tile0 + t) * mtile + wm * 16 * MC;
#pragma unroll
    for (int g = 0; g < MC; ++g) {
      const int64_t c = cw + 16 * g + li;
      colp[g] = X + Ktot * (c < Mtot ? c : 0) + 4 * lq;
    }
    const int64_t cmax = min(cw + 16 * MC - 1, Mtot - 1);
    vec_lim = Mtot * Ktot - Ktot * cmax - KS;  // wave-uniform
  };
  set_tile(0);
  const float* zeros = (const float*)a.zeros;

  // cursor (stage, j, t): t over the stage's k-steps, j over the block (rotated
  // start with one wave along K), stages in order. The load cursor runs D steps
  // ahead and wraps to the start after the last step, so it stays in bounds.
  const int jrot = (WK == 1 && jn > 1) ? (int)(((unsigned)bx * 5u) % (unsigned)jn) : 0;
  int stL = 0, S1L = stage_rows(0) / KS, tileL = 0;
  int jcntL = sb / S1L;  // sb > 0 only when istages == 1
  int tl = sb - jcntL * S1L;
  int jl = jcntL + jrot;
  if (jl >= jn) jl -= jn;
  auto load = [&](vT (&A)[MC][2]) {
    const int i1s = (ib0 + stL) * a.i1blk;
    const int64_t lbase = (int64_t)a.I1 * (j0 + jl) + i1s + KS * tl;
    if (FAST || lbase <= vec_lim) {  // uniform
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int g = 0; g < MC; ++g) A[g][h] = tload<NTL>((const vT*)(colp[g] + lbase + 16 * h));
    } else {
      const int ilimL = a.I1 - i1s;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int off = KS * tl + 16 * h + 4 * lq;
#pragma unroll
        for (int g = 0; g < MC; ++g) {
          // per lane: four real k in one vector load, else element by element
          // (padded i1 reads zero)
          vT v;
          if (off + 4 <= ilimL) {
            v = *(const vT*)(colp[g] + lbase + 16 * h);
          } else {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const float* p = (off + e < ilimL) ? colp[g] + lbase + 16 * h + e : zeros;
              v[e] = *p;
            }
          }
          A[g][h] = v;
        }
      }
    }
    if (++tl == S1L) {
      tl = 0;
      if (++jl == jn) jl = 0;
      if (++jcntL == jn) {
        jcntL = 0;
        if (++stL == a.istages) {
          stL = 0;
          if (MT) {
            if (++tileL == ntile) tileL = 0;
            set_tile(tileL);
          }
        }
        S1L = stage_rows(stL) / KS;
      }
    }
  };

  // acc[g*NB+nb][v]: column c = cw + 16g + 4*lq + v, rank column 16nb + li.
  const bool direct = (a.nsplit == 1);
  const int64_t Mpad = (int64_t)a.mtiles * mtile;
  auto store_tile = [&](int64_t cw) {
#pragma unroll
    for (int g = 0; g < MC; ++g)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        double o[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) o[v] = acc[g * NB + nb][v];
        pm_store_rows<4>(a, direct, Mtot, Mpad, RP, by, 16 * nb + li, cw + 16 * g + 4 * lq, o);
      }
  };

  f4 c32[MC][NB];
#pragma unroll
  for (int g = 0; g < MC; ++g)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) c32[g][nb] = f4{0.f, 0.f, 0.f, 0.f};
  int stC = 0, S1C = S1L, jc = jl, tc = tl, jcntC = jcntL, tileC = 0, fc = tl % a.fold, sc_left = se - sb;
  auto compute = [&](const vT (&A)[MC][2]) {
    const int kk = KS * tc + 4 * lq;
    f4 B[2][NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int h = 0; h < 2; ++h) B[h][nb] = *(const f4*)&hs[(16 * nb + li) * hp + kk + 16 * h];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int g = 0; g < MC; ++g)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb) c32[g][nb] = mfma4(A[g][h][u], B[h][nb][u], c32[g][nb]);
    --sc_left;
    // fold every `fold` k-steps, at the end of each j (and so of each stage) and
    // at the end of the range
    if (++fc == a.fold || tc + 1 == S1C || sc_left == 0) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const double scl = sc[jc * RP + 16 * nb + li];
#pragma unroll
        for (int g = 0; g < MC; ++g) {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            acc[g * NB + nb][e] = __builtin_fma((double)c32[g][nb][e], scl, acc[g * NB + nb][e]);
          c32[g][nb] = f4{0.f, 0.f, 0.f, 0.f};
        }
      }
      fc = 0;
    }
    if (++tc == S1C) {
      tc = 0;
      if (++jc == jn) jc = 0;
      if (++jcntC == jn) {
        jcntC = 0;
        if (++stC < a.istages && sc_left > 0) {
          // next i1 block: every wave of the group gets here at the same step
          __syncthreads();
          pm_stage_h1(a, hs, hp, RP, (ib0 + stC) * a.i1blk, stage_rows(stC));
          __syncthreads();
          S1C = stage_rows(stC) / KS;
        } else if (MT && tileC + 1 < ntile) {  // a tile done (istages == 1): store it, start the next
          stC = 0;
          store_tile((int64_t)(tile0 + tileC) * mtile + wm * 16 * MC);
#pragma unroll
          for (int v = 0; v < NACC; ++v)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[v][e] = 0.0;
          ++tileC;
        }
      }
    }
  };

  vT A[D][MC][2];
  int s = sb;
#pragma unroll
  for (int d = 0; d < D; ++d) load(A[d]);
  for (; s + D - 1 < se; s += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      compute(A[d]);
      __builtin_amdgcn_sched_barrier(0);
      load(A[d]);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int d = 0; d < D - 1; ++d)
    if (s + d < se) compute(A[d]);

  __syncthreads();
  wave_reduce_k<NACC>(acc, lds_d, wk, wm, WK);
  if (wk != 0) return;
  store_tile((int64_t)(tile0 + ntile - 1) * mtile + wm * 16 * MC);
}

// ----------------------------------------------------------------------------
// Right side with X staged through LDS (the "xs" form). The direct loads above
// give each lane's 16-byte load its own column (the MFMA row index), so one
// load instruction reads sixteen columns, 64 bytes from each; measured on this
// chip, HBM serves that pattern at ~6.0 TB/s against ~6.8 TB/s for four columns
// of 256 bytes. Here load instruction i of a step reads columns 4i .. 4i+3 of
// the wave, 64 consecutive k (256 bytes) each (lane (li, lq): column 4i + lq,
// k 4li .. 4li+3); the wave writes every lane's 16 bytes into its own padded
// [column][k] tile in LDS and reads them back in the MFMA layout (lane (li, lq):
// column li, k 16h + 4lq .. +3). A tile is written and read by one wave only,
// and a wave's LDS operations execute in order, so there is no barrier and one
// tile per wave is enough. Shapes: I1 a multiple of 64 (each step is 64 real
// i1 of one j, so every load lies inside the tensor), four waves along M and
// one i1 block per group (the plan falls back to the direct form otherwise).
// ----------------------------------------------------------------------------
constexpr int kXsKs = 64;            // k per step
constexpr int kBufWord3 = 0x00020000;  // buffer resource word 3: raw 32-bit data
constexpr int kBufNt = 2;              // buffer load cache policy: nontemporal
constexpr int kXsRow = kXsKs + 4;    // floats per staged column in LDS (padded)
constexpr int xs_mc(int nb) { return nb >= 4 ? 1 : 2; }
constexpr int xs_pf(int nb) { return 3; }

template <int NB, int D, bool MT>
__device__ __forceinline__ void pm_right_f32_xs_body(const PmArgs& a, int bx, int by) {
  constexpr int RP = NB * 16;
  constexpr int MC = xs_mc(NB);
  constexpr int KS = kXsKs;
  constexpr int NI = 4 * MC;  // load instructions per step
  constexpr int NACC = MC * NB;
  extern __shared__ double lds_d[];
  const int hp = a.i1blk + 4;
  float* hs = (float*)lds_d;
  double* sc = lds_d + (RP * hp + 1) / 2;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int li = lane & 15, lq = lane >> 4;
  // the wave's staging tile, after the scales (16-byte aligned: RP * hp and
  // jblk * RP are multiples of 64 floats)
  float* xt = (float*)(sc + (size_t)a.jblk * RP) + wave * (16 * MC * kXsRow);
  const int64_t Mtot = a.IR, Ktot = a.IL;
  const int mtile = 4 * 16 * MC;
  const int tile0 = MT ? bx * a.mper : bx;
  const int ntile = MT ? min(a.mper, a.mtiles - tile0) : 1;
  const int ib = by % a.n_i1blk, jb = by / a.n_i1blk;
  const int i1_0 = ib * a.i1blk;
  const int i1n = min(a.i1blk, a.I1pad - i1_0);
  const int64_t j0 = (int64_t)jb * a.jblk;
  const int jn = (int)min((int64_t)a.jblk, a.J - j0);
  const float* X = (const float*)a.X;

  pm_prologue(a, hs, hp, sc, RP, i1_0, i1n, j0, jn);
  __syncthreads();

  const int S1 = i1n / KS;
  const int se = ntile * S1 * jn;  // every wave walks all steps of its columns

  double acc[NACC][4];
#pragma unroll
  for (int v = 0; v < NACC; ++v)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[v][e] = 0.0;

  // Loads are buffer loads: the wave-uniform resource starts at the step's
  // first element of the wave's first column and ends at the tensor's end, so
  // lanes of columns past the output read zeros (the buffer range check) and
  // the per-lane byte offsets, column 4i + lq and k 4li, are fixed.
  const int64_t IX = Mtot * Ktot;
  uint32_t voff[NI];
#pragma unroll
  for (int i = 0; i < NI; ++i) voff[i] = (uint32_t)((((int64_t)(4 * i + lq)) * Ktot + 4 * li) * 4);
  int64_t cwk = 0;  // first element of the wave's columns in the tile being loaded
  auto set_tile = [&](int t) { cwk = ((int64_t)(tile0 + t) * mtile + wave * 16 * MC) * Ktot; };
  set_tile(0);

  // cursor (tile, j, t); j starts rotated by the group, the load cursor runs D
  // steps ahead and wraps inside the group's tiles and j block
  const int jrot = jn > 1 ? (int)(((unsigned)bx * 5u) % (unsigned)jn) : 0;
  int tileL = 0, jcntL = 0, tl = 0, jl = jrot;
  auto load = [&](f4 (&A)[NI]) {
    const int64_t e0 = cwk + (int64_t)a.I1 * (j0 + jl) + i1_0 + KS * tl;
    const int64_t rem = IX - e0;
    const int nrec = rem <= 0 ? 0 : (rem >= (int64_t)0x3fffffff ? (int)0xfffffffc : (int)(rem * 4));
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)(X + e0), (short)0, nrec, kBufWord3);
#pragma unroll
    for (int i = 0; i < NI; ++i) A[i] = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)voff[i], 0, kBufNt));
    if (++tl == S1) {
      tl = 0;
      if (++jl == jn) jl = 0;
      if (MT && ++jcntL == jn) {
        jcntL = 0;
        if (++tileL == ntile) tileL = 0;
        set_tile(tileL);
      }
    }
  };
  auto stage = [&](const f4 (&A)[NI]) {
#pragma unroll
    for (int i = 0; i < NI; ++i) *(f4*)&xt[(4 * i + lq) * kXsRow + 4 * li] = A[i];
  };

  // acc[g*NB+nb][v]: column c = cw + 16g + 4*lq + v, rank column 16nb + li.
  const bool direct = (a.nsplit == 1);
  const int64_t Mpad = (int64_t)a.mtiles * mtile;
  auto store_tile = [&](int64_t cw) {
#pragma unroll
    for (int g = 0; g < MC; ++g)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        double o[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) o[v] = acc[g * NB + nb][v];
        pm_store_rows<4>(a, direct, Mtot, Mpad, RP, by, 16 * nb + li, cw + 16 * g + 4 * lq, o);
      }
  };

  // MFMA operands of one h (16 k) of a step: the tile's four k of each column
  // group and the H_1 values of the same k for each column block
  struct Ops {
    f4 x[MC], b[NB];
  };
  auto read_ops = [&](int t, int h, Ops& o) {
#pragma unroll
    for (int g = 0; g < MC; ++g) o.x[g] = *(const f4*)&xt[(16 * g + li) * kXsRow + 16 * h + 4 * lq];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) o.b[nb] = *(const f4*)&hs[(16 * nb + li) * hp + KS * t + 4 * lq + 16 * h];
  };
  using Acc32 = f4[MC][NB];
  // `first`: the step's first products, which start the sums (zero input)
  auto mma = [&](const Ops& o, Acc32& c, bool first) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int g = 0; g < MC; ++g)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          c[g][nb] = mfma4(o.x[g][u], o.b[nb][u], (first && u == 0) ? f4{0.f, 0.f, 0.f, 0.f} : c[g][nb]);
  };
  // FP32 sums of one step (64 products per output) into FP64 with the step's
  // per-(j, column) scale
  auto fold = [&](const Acc32& c, const double (&scl)[NB]) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int g = 0; g < MC; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[g * NB + nb][e] = __builtin_fma((double)c[g][nb][e], scl[nb], acc[g * NB + nb][e]);
  };
  auto read_scales = [&](int j, double (&scl)[NB]) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) scl[nb] = sc[j * RP + 16 * nb + li];
  };

  // Each step sums into its own FP32 set (two sets, alternating with the step's
  // parity) and is folded into FP64 during the next step, after that step's
  // first MFMAs: the fold's reads of the MFMA results then find them complete.
  // A set that holds nothing to fold is zero (so the fold is unconditional).
  Acc32 c32[2];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int g = 0; g < MC; ++g)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) c32[q][g][nb] = f4{0.f, 0.f, 0.f, 0.f};
  int jc = jl, tc = 0, jcntC = 0, tileC = 0, jprev = 0;
  // One step, in four scheduling regions, one per h (16 k). On entry the tile
  // holds the step and p0 its h = 0 operands. The LDS reads of h + 1 go out
  // before the MFMAs of h; with `next`, the following step (registers An,
  // loaded D steps ago) is written to the tile and the loads D steps ahead go
  // out into An during the MFMAs of h = 2, and its h = 0 operands are read
  // before the MFMAs of h = 3 (a wave's LDS operations run in order, so the
  // tile is rewritten only after this step's reads). sched_group_barrier
  // spreads the LDS and memory instructions between the MFMAs, so that the
  // matrix pipe keeps busy while the LDS takes the writes.
  constexpr int NR = MC + NB;  // LDS reads of one h
  Ops p0, p1;
  auto step = [&](f4 (&An)[NI], bool next, Acc32& cc, Acc32& cp) {
    double sp[NB];
    read_scales(jprev, sp);
    read_ops(tc, 1, p1);
    mma(p0, cc, true);
    fold(cp, sp);
#pragma unroll
    for (int i = 0; i < NR + NB; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // LDS read
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // MFMA
    }
#pragma unroll
    for (int i = 0; i < 4 * MC * NB - NR - NB; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x002, 3, 0);  // VALU
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
    read_ops(tc, 2, p0);
    mma(p1, cc, false);
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 1);
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 1);
    }
    __builtin_amdgcn_sched_barrier(0);
    read_ops(tc, 3, p1);
    mma(p0, cc, false);
    if (next) {
      stage(An);
      load(An);
    }
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 2);
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 2);
    }
#pragma unroll
    for (int i = 0; i < NI; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x200, 1, 2);  // LDS write
      __builtin_amdgcn_sched_group_barrier(0x020, 1, 2);  // memory read
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 2);
    }
    __builtin_amdgcn_sched_barrier(0);
    if (next) read_ops(tc + 1 == S1 ? 0 : tc + 1, 0, p0);
    mma(p1, cc, false);
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 3);
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 3);
    }
    __builtin_amdgcn_sched_barrier(0);
    jprev = jc;
    if (++tc == S1) {
      tc = 0;
      if (++jc == jn) jc = 0;
      if (MT && ++jcntC == jn) {
        jcntC = 0;
        if (tileC + 1 < ntile) {  // a tile done: fold its last step now, store it, start the next
          double sl[NB];
          read_scales(jprev, sl);
          fold(cc, sl);
#pragma unroll
          for (int g = 0; g < MC; ++g)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) cc[g][nb] = f4{0.f, 0.f, 0.f, 0.f};
          store_tile((int64_t)(tile0 + tileC) * mtile + wave * 16 * MC);
#pragma unroll
          for (int v = 0; v < NACC; ++v)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[v][e] = 0.0;
          ++tileC;
        }
      }
    }
  };

  // D steps of X in flight in registers: step s + 1 is staged from ring slot
  // (s + 1) % D while step s is computed, and that slot then loads step s + 1 + D
  // (the cursor wraps inside the group's tiles and j block, so loads past the
  // end read valid memory that is never used). The loop body covers 2D steps so
  // that ring slots and FP32 sets are both fixed per unrolled step.
  f4 A[D][NI];
#pragma unroll
  for (int d = 0; d < D; ++d) load(A[d]);
  stage(A[0]);
  __builtin_amdgcn_sched_barrier(0);
  load(A[0]);
  __builtin_amdgcn_sched_barrier(0);
  read_ops(0, 0, p0);
  int s = 0;
  for (; s + 2 * D < se; s += 2 * D) {
#pragma unroll
    for (int d = 0; d < 2 * D; ++d) step(A[(d + 1) % D], true, c32[d % 2], c32[(d + 1) % 2]);
  }
#pragma unroll
  for (int d = 0; d < 2 * D; ++d)
    if (s + d < se) step(A[(d + 1) % D], s + d + 1 < se, c32[d % 2], c32[(d + 1) % 2]);
  {  // the last step (its set: parity of se - 1)
    double sl[NB];
    read_scales(jprev, sl);
    if ((se - 1) % 2 == 0) fold(c32[0], sl);
    else fold(c32[1], sl);
  }
  store_tile((int64_t)(tile0 + ntile - 1) * mtile + wave * 16 * MC);
}

// FAST: the shape guarantees that every vector load of every step lies inside
// the tensor (pm_f32_fast), so the loads need no per-step check. MT: a group
// streams several M tiles (a separate form, so that the one-tile kernels keep
// their register budget).
// NTL: tensor loads with the nontemporal (streaming) hint. The stand-alone
// kernels stream one large tensor and use it; the batched kernels do not: their
// items are a few hundred KB of many small tensors, several launches stream at
// once, and with the hint the caches dropped lines (or line halves) that the
// next k-step still needed (256-job batch: 11.2 -> 9.0 GB fetched per tick,
// 3.24 -> 2.56 ms; the 128^4 left node alone is 0.18 ms with the hint, 0.20
// without).
template <int NB, bool FAST, bool MT, bool NTL>
__device__ __forceinline__ void pm_f32_body(int side, const PmArgs& a, int bx, int by) {
  if (side == 0) pm_left_f32_body<NB, left_pf(NB), FAST, MT, NTL>(a, bx, by);
  else pm_right_f32_body<NB, right_pf(NB), FAST, MT, NTL>(a, bx, by);
}

// Stand-alone kernels: one work-group per (M tile group, split).
template <int SIDE, int NB, bool FAST, bool MT>
__global__ __launch_bounds__(NT, 2) void pm_f32(PmArgs a) {
  pm_f32_body<NB, FAST, MT, true>(SIDE, a, blockIdx.x, blockIdx.y);
}

// Persistent batched form of the same kernel: work-group b takes the items
// grp[0] + b, grp[0] + b + gridDim.x, ... below grp[0] + grp[1]; each item is one
// (M tile group, split) work-group of a recorded stand-alone launch of this variant.
template <int SIDE, int NB, bool FAST, bool MT>
__global__ __launch_bounds__(NT, 2) void pm_f32_items(const BItem* __restrict__ items, const int* __restrict__ grp,
                                                      const KOp* __restrict__ ops) {
  const int off = grp[0], n = grp[1];
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const BItem it = items[off + i];
    const KOp& op = ops[it.op];
    pm_f32_body<NB, FAST, MT, false>(SIDE, op.u.pm, it.bx, it.by);
    __syncthreads();  // LDS is reused by the next item
  }
}

// The xs form (right side only; FAST shapes by construction).
template <int NB, bool MT>
__global__ __launch_bounds__(NT, 2) void pm_f32_xs(PmArgs a) {
  pm_right_f32_xs_body<NB, xs_pf(NB), MT>(a, blockIdx.x, blockIdx.y);
}
template <int NB, bool MT>
__global__ __launch_bounds__(NT, 2) void pm_f32_xs_items(const BItem* __restrict__ items, const int* __restrict__ grp,
                                                         const KOp* __restrict__ ops) {
  const int off = grp[0], n = grp[1];
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const BItem it = items[off + i];
    const KOp& op = ops[it.op];
    pm_right_f32_xs_body<NB, xs_pf(NB), MT>(op.u.pm, it.bx, it.by);
    __syncthreads();  // LDS is reused by the next item
  }
}

// The scale table of a launch: sctab[j * RP + r] = Krest(j, col0 + r) times
// the column's 1/lambda product (0 for r >= R), j < J. The same function of
// (j, column) the work-groups otherwise evaluate themselves.
__device__ __forceinline__ void scale_table_block(const PmArgs& a, int RP, int64_t n, int64_t blk) {
  const int64_t e = blk * NT + threadIdx.x;
  if (e >= n) return;
  const int64_t j = e / RP;
  const int r = (int)(e - j * RP);
  a.sctab[e] = r < a.R ? krp_scale_entry(a.krp, (uint32_t)j, a.col0 + r) : 0.0;
}
__global__ __launch_bounds__(NT) void pm_scale_table_kernel(PmArgs a, int RP, int64_t n) {
  scale_table_block(a, RP, n, blockIdx.x);
}
// Batched form: an item runs `coarse` consecutive blocks of one recorded table.
__global__ __launch_bounds__(NT) void pm_scale_table_items(const BItem* __restrict__ items,
                                                           const int* __restrict__ grp,
                                                           const KOp* __restrict__ ops) {
  const int off = grp[0], n = grp[1];
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const BItem it = items[off + i];
    const KOp& op = ops[it.op];
    const int RP = op.variant;
    const int64_t tot = op.u.pm.J * RP;
    for (unsigned c = 0; c < op.coarse; ++c) {
      const int64_t b = (int64_t)it.bx * op.coarse + c;
      if (b < (int64_t)op.gx) scale_table_block(op.u.pm, RP, tot, b);
    }
  }
}

template <bool MT>
const void* pick_xs(int nb, bool batch) {
  switch (nb) {
    case 1: return batch ? (const void*)pm_f32_xs_items<1, MT> : (const void*)pm_f32_xs<1, MT>;
    case 2: return batch ? (const void*)pm_f32_xs_items<2, MT> : (const void*)pm_f32_xs<2, MT>;
    case 4: return batch ? (const void*)pm_f32_xs_items<4, MT> : (const void*)pm_f32_xs<4, MT>;
    default: return nullptr;
  }
}

template <int SIDE, bool FAST, bool MT>
const void* pick(int nb, bool batch) {
  switch (nb) {
    case 1: return batch ? (const void*)pm_f32_items<SIDE, 1, FAST, MT> : (const void*)pm_f32<SIDE, 1, FAST, MT>;
    case 2: return batch ? (const void*)pm_f32_items<SIDE, 2, FAST, MT> : (const void*)pm_f32<SIDE, 2, FAST, MT>;
    case 4: return batch ? (const void*)pm_f32_items<SIDE, 4, FAST, MT> : (const void*)pm_f32<SIDE, 4, FAST, MT>;
    default: return nullptr;
  }
}

template <int SIDE, bool MT>
const void* pick_fast(int nb, bool fast, bool batch) {
  return fast ? pick<SIDE, true, MT>(nb, batch) : pick<SIDE, false, MT>(nb, batch);
}

const void* kernel_for(int side, int nb, bool fast, bool mt, bool xs, bool batch) {
  if (xs) return side == 1 && fast ? (mt ? pick_xs<true>(nb, batch) : pick_xs<false>(nb, batch)) : nullptr;
  if (side == 0) return mt ? pick_fast<0, true>(nb, fast, batch) : pick_fast<0, false>(nb, fast, batch);
  return mt ? pick_fast<1, true>(nb, fast, batch) : pick_fast<1, false>(nb, fast, batch);
}

size_t reduce_lds(int side, int nb, int wm) {
  if (wm >= 4) return 0;
  const int nacc = side == 0 ? left_tr(nb) * nb : right_mc(nb) * nb;
  return (size_t)wm * nacc * 4 * 64 * sizeof(double);
}

}  // namespace

int pm_f32_wave_rows(int side, int nb, bool xs) {
  if (xs) return 16 * xs_mc(nb);
  return side == 0 ? 16 * left_tr(nb) : 16 * right_mc(nb);
}
int pm_f32_kstep(int side, bool xs) { return xs ? kXsKs : (side == 0 ? 16 : 32); }
size_t pm_f32_xs_tile_lds(int nb) { return (size_t)4 * 16 * xs_mc(nb) * kXsRow * sizeof(float); }
// the per-lane buffer offsets (up to 16 MC columns of Ktot elements) fit 31 bits
bool pm_f32_xs_ok(int64_t Ktot, int nb) { return (int64_t)16 * xs_mc(nb) * Ktot * 4 + 256 < ((int64_t)1 << 31); }
size_t pm_f32_reduce_lds(int side, int nb, int wm) { return reduce_lds(side, nb, wm); }

// Every vector load of every step lies inside the tensor when the k-steps
// tile I1 exactly (no padded i1) and, on the left side, the row groups tile
// I_L exactly (no group straddles a column end).
bool pm_f32_fast(int side, int64_t IL, int I1, int nb, bool xs) {
  if (I1 % pm_f32_kstep(side, xs) != 0) return false;
  return side == 1 || IL % left_tr(nb) == 0;
}

hipError_t pm_launch_f32(const PmLaunch& L, const PmArgs& a, const Sink& sk) {
  const int wm = a.wm;
  const bool fast = pm_f32_fast(L.side, a.IL, a.I1, L.nb, L.xs);
  const bool mt = L.mper > 1;
  // variant = xs*100000 + wide*10000 + side*1000 + nb*100 + mt*10 + fast (wide: launched with more LDS)
  const int variant =
      (L.xs ? 100000 : 0) + (L.wide ? 10000 : 0) + L.side * 1000 + L.nb * 100 + (mt ? 10 : 0) + (fast ? 1 : 0);
  const void* k = kernel_for(L.side, L.nb, fast, mt, L.xs, false);
  if (!k || (wm != 1 && wm != 4)) return hipErrorInvalidValue;
  if (L.xs && (wm != 4 || a.istages != 1)) return hipErrorInvalidValue;
  size_t lds = L.lds_bytes;
  if (reduce_lds(L.side, L.nb, wm) > lds) lds = reduce_lds(L.side, L.nb, wm);
  if (lds > kPmMaxLds) return hipErrorInvalidValue;
  if (sk.rec) {
    KOp op{};
    op.kind = K_PM_F32;
    op.variant = variant;
    op.gx = (unsigned)L.mgroups;
    op.gy = (unsigned)L.nsplit;
    op.lds = (unsigned)lds;
    op.u.pm = a;
    if (a.sctab) {
      hipError_t e = pm_scale_table_record(L, a, sk);
      if (e != hipSuccess) return e;
    }
    return sink_record(sk, op);
  }
  if (a.sctab) {
    hipError_t e = pm_scale_table_launch(L, a, sk.st);
    if (e != hipSuccess) return e;
  }
  if (lds > 64 * 1024) pm_allow_lds(k, 160 * 1024);
  void* args[] = {(void*)&a};
  return hipLaunchKernel(k, dim3(L.mgroups, L.nsplit), dim3(NT), args, lds, sk.st);
}

size_t pm_sctab_doubles(const PmLaunch& L) { return (size_t)L.J * 16 * L.nb; }

hipError_t pm_scale_table_record(const PmLaunch& L, const PmArgs& a, const Sink& sk) {
  const int RP = 16 * L.nb;
  const int64_t n = L.J * RP;
  KOp op{};
  op.kind = K_SCTAB;
  op.variant = RP;
  op.gx = (unsigned)((n + NT - 1) / NT);
  op.gy = 1;
  op.u.pm = a;
  return sink_record(sk, op);
}

const void* pm_sctab_batch_kernel() { return (const void*)pm_scale_table_items; }

hipError_t pm_scale_table_launch(const PmLaunch& L, const PmArgs& a, hipStream_t st) {
  int RP = 16 * L.nb;
  int64_t n = L.J * RP;
  PmArgs b = a;
  void* targs[] = {(void*)&b, (void*)&RP, (void*)&n};
  return hipLaunchKernel((const void*)pm_scale_table_kernel, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), targs, 0,
                         st);
}

const void* pm_f32_batch_kernel(int variant) {
  const int side = (variant / 1000) % 10, nb = (variant / 100) % 10;
  const void* k = kernel_for(side, nb, variant % 10 != 0, (variant / 10) % 10 != 0, (variant / 100000) % 10 != 0, true);
  if (k) pm_allow_lds(k, 160 * 1024);
  return k;
}

}  // namespace nncpk
