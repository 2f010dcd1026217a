// Partial MTTKRP on MFMA for FP32 tensors: the root edges of the dimension tree
// (Section IV-A, Figure 2a), T = X_[L] * K (left node {1..s}) or
// T = X_[L]^T * K (right node {s+1..N}), where X_[L] is the tensor viewed as the
// column-major I_L x I_R matrix and K the Khatri-Rao product of the other
// side's factors (first contracted mode fastest).
//
// Design (gfx950, wave64):
//  * The reduction index is split as k = i1 + I1*j (i1: first contracted mode).
//    K(k, :) = H_1(i1, :) * Krest(j, :), so a work-group keeps the H_1 rows of
//    its i1 block in LDS for the whole kernel (the MFMA B operand), and applies
//    Krest(j, :) as a per-column factor when it folds each k-step's FP32 MFMA
//    result into FP64 accumulators (one v_fma_f64 per output). The Khatri-Rao
//    product is never formed, and the main loop has no barrier.
//  * X streams from HBM straight into VGPRs with 8/16-byte loads, two k-steps
//    ahead of the MFMAs (v_mfma_f32_16x16x4_f32), with no branches around the
//    loads (out-of-range lanes read a valid address and are zeroed).
//  * Precision: each MFMA chain covers one k-step (16 or 32 products per
//    output) before it is added into FP64; split-K partials, the cross-wave
//    reduction and the output are FP64.
//  * Split-K over (i1 block, j block) pairs: each work-group writes an FP64
//    partial; a separate reduction kernel sums them in split order, so results
//    do not depend on scheduling and no cross-XCD fence is needed.
#include "pm_common.hpp"

namespace nncpk {
namespace {

// ----------------------------------------------------------------------------
// Left side: T(m, r) = sum_k X[m + IL*k] K(k, r); m is contiguous in X.
// A wave covers 16*TR rows m. In a k-step (16 consecutive i1 of one j), lane
// (li, lq) loads rows TR*li .. TR*li+TR-1 of the columns i1 = base + 4*lq + u,
// u = 0..3; MFMA chain tt uses row TR*li + tt of every load.
// ----------------------------------------------------------------------------
template <int NB, int TR, int WM, bool FAST, int D>
__device__ __forceinline__ void pm_left_f32_body(const PmArgs& a, int bx, int by, int gx) {
  constexpr bool VEC = FAST;
  constexpr int RP = NB * 16;
  constexpr int WK = 4 / WM;
  constexpr int KS = 16;
  constexpr int NACC = TR * NB;
  constexpr int WROWS = 16 * TR;
  typedef float vT __attribute__((ext_vector_type(TR)));
  extern __shared__ double lds_d[];
  const int hp = a.i1blk + 4;
  float* hs = (float*)lds_d;
  double* sc = lds_d + (RP * hp + 1) / 2;

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave % WM, wk = wave / WM;
  const int li = lane & 15, lq = lane >> 4;
  const int64_t Mtot = a.IL;
  const int mtile = WM * WROWS;
  const int64_t mbeg = (int64_t)bx * mtile;
  const int64_t mw = mbeg + wm * WROWS;
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

  double acc[NACC][4];
#pragma unroll
  for (int v = 0; v < NACC; ++v)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[v][e] = 0.0;

  const int64_t m = mw + TR * li;
  const int64_t mload = (m + TR <= Mtot) ? m : 0;
  const int ilim = a.I1 - i1_0;  // lane i1 offsets >= ilim are padding
  const float* zeros = (const float*)a.zeros;
  // lane part of the address of column (colbase + 4*lq + u): loop invariant
  int64_t lane_off[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) lane_off[u] = Mtot * (int64_t)(4 * lq + u) + (VEC ? mload : 0);

  // load cursor (uniform): step = jl * S1 + tl. With one wave along K the group
  // starts at a j rotated by its M tile, so groups that share a split do not all
  // request the same addresses modulo the column stride at the same time.
  const int jrot = (WK == 1 && jn > 1) ? (int)(((unsigned)bx * 5u) % (unsigned)jn) : 0;
  int jl = sb / S1 + jrot, tl = sb - (sb / S1) * S1;
  if (jl >= jn) jl -= jn;  // an empty range (sb == S1 * jn) starts at the block's first j
  // The cursor always stays inside the group's j block (it wraps), so loads of
  // steps past the wave's range read valid memory and are simply not used.
  auto load = [&](vT (&A)[4], bool sv) {
    (void)sv;
    const int64_t colbase = (int64_t)a.I1 * (j0 + jl) + i1_0 + KS * tl;
    const float* base = X + Mtot * colbase;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (FAST) {
        // I1 is a multiple of the k-step and rows are aligned: no padding lanes
        A[u] = __builtin_nontemporal_load((const vT*)(base + lane_off[u]));
      } else {
        const bool kv = (KS * tl + 4 * lq + u) < ilim;
        vT v;
#pragma unroll
        for (int e = 0; e < TR; ++e) {
          const float* p = (kv && m + e < Mtot) ? base + lane_off[u] + m + e : zeros;
          v[e] = *p;
        }
        A[u] = v;
      }
    }
    if (++tl == S1) {
      tl = 0;
      if (++jl == jn) jl = 0;
    }
  };

  // FP32 partial sums (one 16x16 block per (tt, nb)) live for `fold` k-steps and
  // are then added into the FP64 accumulators with the chunk's column scale.
  f4 c32[TR][NB];
#pragma unroll
  for (int tt = 0; tt < TR; ++tt)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) c32[tt][nb] = f4{0.f, 0.f, 0.f, 0.f};
  int jc = jl, tc = tl, fc = tl % a.fold, sc_left = se - sb;
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
          for (int e = 0; e < 4; ++e) acc[tt * NB + nb][e] = __builtin_fma((double)c32[tt][nb][e], scl, acc[tt * NB + nb][e]);
          c32[tt][nb] = f4{0.f, 0.f, 0.f, 0.f};
        }
      }
      fc = 0;
    }
    if (++tc == S1) {
      tc = 0;
      if (++jc == jn) jc = 0;
    }
  };

  // D k-steps of X in flight: the loads of step s+D are issued right after step
  // s is consumed. sched_barrier keeps the compiler from sinking them.
  // The first D loads are issued unconditionally (out-of-range steps read the
  // zero block) so every path into the loop has the same loads in flight and the
  // compiler's wait counts stay precise.
  vT A[D][4];
  int s = sb;
#pragma unroll
  for (int d = 0; d < D; ++d) load(A[d], sb + d < se);
  for (; s + D - 1 < se; s += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      compute(A[d]);
      __builtin_amdgcn_sched_barrier(0);
      load(A[d], s + D + d < se);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int d = 0; d < D - 1; ++d)
    if (s + d < se) compute(A[d]);

  __syncthreads();  // LDS is reused by the cross-wave reduction
  wave_reduce_k<NACC>(acc, lds_d, wk, wm, WK);
  if (wk != 0 && a.nsplit == 1) return;

  // acc[tt*NB+nb][v]: row mw + TR*(4*lq + v) + tt, rank column 16nb + li.
  const bool direct = (a.nsplit == 1);
  const int64_t Mpad = (int64_t)gx * mtile;
  (void)mbeg;
  if (wk == 0) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double o[TR];
#pragma unroll
        for (int tt = 0; tt < TR; ++tt) o[tt] = acc[tt * NB + nb][v];
        pm_store_rows<TR>(a, direct, Mtot, Mpad, RP, by, 16 * nb + li, mw + TR * (4 * lq + v), o);
      }
  }
}

// ----------------------------------------------------------------------------
// Right side: T(c, r) = sum_k X[k + IL*c] K(k, r); k is contiguous in X.
// A wave covers MC groups of 16 columns c. In a k-step (32 consecutive i1 of
// one j), lane (li, lq) loads k = base + 16h + 4*lq + u (u = 0..3 in one
// 16-byte load, h = 0..1) of column c = group + li.
// ----------------------------------------------------------------------------
template <int NB, int MC, int WM, bool FAST, int D>
__device__ __forceinline__ void pm_right_f32_body(const PmArgs& a, int bx, int by, int gx) {
  constexpr bool VEC = FAST;
  constexpr int RP = NB * 16;
  constexpr int WK = 4 / WM;
  constexpr int KS = 32;
  constexpr int NACC = MC * NB;
  extern __shared__ double lds_d[];
  const int hp = a.i1blk + 4;
  float* hs = (float*)lds_d;
  double* sc = lds_d + (RP * hp + 1) / 2;

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave % WM, wk = wave / WM;
  const int li = lane & 15, lq = lane >> 4;
  const int64_t Mtot = a.IR, Ktot = a.IL;
  const int mtile = WM * 16 * MC;
  const int64_t mbeg = (int64_t)bx * mtile;
  const int64_t cw = mbeg + wm * 16 * MC;
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

  double acc[NACC][4];
#pragma unroll
  for (int v = 0; v < NACC; ++v)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[v][e] = 0.0;

  const float* colp[MC];
#pragma unroll
  for (int g = 0; g < MC; ++g) {
    const int64_t c = cw + 16 * g + li;
    colp[g] = X + Ktot * (c < Mtot ? c : 0) + 4 * lq;
  }
  const int ilim = a.I1 - i1_0;
  const float* zeros = (const float*)a.zeros;

  const int jrot = (WK == 1 && jn > 1) ? (int)(((unsigned)bx * 5u) % (unsigned)jn) : 0;
  int jl = sb / S1 + jrot, tl = sb - (sb / S1) * S1;
  if (jl >= jn) jl -= jn;  // an empty range (sb == S1 * jn) starts at the block's first j
  auto load = [&](f4 (&A)[MC][2], bool sv) {
    (void)sv;
    const int64_t lbase = (int64_t)a.I1 * (j0 + jl) + i1_0 + KS * tl;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int off = KS * tl + 16 * h + 4 * lq;
#pragma unroll
      for (int g = 0; g < MC; ++g) {
        if (FAST) {
          A[g][h] = __builtin_nontemporal_load((const f4*)(colp[g] + lbase + 16 * h));
        } else {
          f4 v;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const bool kv = off + e < ilim;
            const float* p = kv ? colp[g] + lbase + 16 * h + e : zeros;
            v[e] = *p;
          }
          A[g][h] = v;
        }
      }
    }
    if (++tl == S1) {
      tl = 0;
      if (++jl == jn) jl = 0;
    }
  };

  f4 c32[MC][NB];
#pragma unroll
  for (int g = 0; g < MC; ++g)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) c32[g][nb] = f4{0.f, 0.f, 0.f, 0.f};
  int jc = jl, tc = tl, fc = tl % a.fold, sc_left = se - sb;
  auto compute = [&](const f4 (&A)[MC][2]) {
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
    // fold every `fold` k-steps, at the end of each j (the last i1 block can be
    // shorter than the others, so fold need not divide its steps) and at the end
    if (++fc == a.fold || tc + 1 == S1 || sc_left == 0) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const double scl = sc[jc * RP + 16 * nb + li];
#pragma unroll
        for (int g = 0; g < MC; ++g) {
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[g * NB + nb][e] = __builtin_fma((double)c32[g][nb][e], scl, acc[g * NB + nb][e]);
          c32[g][nb] = f4{0.f, 0.f, 0.f, 0.f};
        }
      }
      fc = 0;
    }
    if (++tc == S1) {
      tc = 0;
      if (++jc == jn) jc = 0;
    }
  };

  f4 A[D][MC][2];
  int s = sb;
#pragma unroll
  for (int d = 0; d < D; ++d) load(A[d], sb + d < se);
  for (; s + D - 1 < se; s += D) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      compute(A[d]);
      __builtin_amdgcn_sched_barrier(0);
      load(A[d], s + D + d < se);
      __builtin_amdgcn_sched_barrier(0);
    }
  }
#pragma unroll
  for (int d = 0; d < D - 1; ++d)
    if (s + d < se) compute(A[d]);

  __syncthreads();
  wave_reduce_k<NACC>(acc, lds_d, wk, wm, WK);
  if (wk != 0 && a.nsplit == 1) return;

  // acc[g*NB+nb][v]: column c = cw + 16g + 4*lq + v, rank column 16nb + li.
  const bool direct = (a.nsplit == 1);
  const int64_t Mpad = (int64_t)gx * mtile;
  (void)mbeg;
  if (wk == 0) {
#pragma unroll
    for (int g = 0; g < MC; ++g)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        double o[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) o[v] = acc[g * NB + nb][v];
        pm_store_rows<4>(a, direct, Mtot, Mpad, RP, by, 16 * nb + li, cw + 16 * g + 4 * lq, o);
      }
  }
}

// Rows per left wave = 16 * left_tr(NB); columns per right wave = 16 * right_mc(NB).
// Chosen so that the FP64 accumulators (2 VGPRs per output) leave room for
// several k-steps of X in flight without spilling. PF = k-steps in flight.
constexpr int left_tr(int nb) { return nb >= 4 ? 2 : 4; }
constexpr int right_mc(int nb) { return nb >= 4 ? 2 : 4; }
constexpr int left_pf(int nb) { return nb == 2 ? 3 : 4; }
constexpr int right_pf(int nb) { return nb >= 4 ? 3 : 3; }

// Stand-alone kernels: one work-group per (M tile, split).
template <int NB, int TR, int WM, bool FAST, int D>
__global__ __launch_bounds__(NT, 2) void pm_left_f32(PmArgs a) {
  pm_left_f32_body<NB, TR, WM, FAST, D>(a, blockIdx.x, blockIdx.y, gridDim.x);
}
template <int NB, int MC, int WM, bool FAST, int D>
__global__ __launch_bounds__(NT, 2) void pm_right_f32(PmArgs a) {
  pm_right_f32_body<NB, MC, WM, FAST, D>(a, blockIdx.x, blockIdx.y, gridDim.x);
}

template <int NB, int WM, bool VEC>
const void* kernel_ptr(int side) {
  if (side == 0) return (const void*)pm_left_f32<NB, left_tr(NB), WM, VEC, left_pf(NB)>;
  return (const void*)pm_right_f32<NB, right_mc(NB), WM, VEC, right_pf(NB)>;
}

// variant = side*1000 + nb*100 + wm*10 + vec
const void* select_variant(int v) {
  const int side = v / 1000;
  switch (v % 1000) {
    case 141: return kernel_ptr<1, 4, true>(side);
    case 140: return kernel_ptr<1, 4, false>(side);
    case 111: return kernel_ptr<1, 1, true>(side);
    case 110: return kernel_ptr<1, 1, false>(side);
    case 241: return kernel_ptr<2, 4, true>(side);
    case 240: return kernel_ptr<2, 4, false>(side);
    case 211: return kernel_ptr<2, 1, true>(side);
    case 210: return kernel_ptr<2, 1, false>(side);
    case 441: return kernel_ptr<4, 4, true>(side);
    case 440: return kernel_ptr<4, 4, false>(side);
    case 411: return kernel_ptr<4, 1, true>(side);
    case 410: return kernel_ptr<4, 1, false>(side);
    default: return nullptr;
  }
}

template <int NB, int WM, bool VEC>
__device__ __forceinline__ void body_for(int side, const PmArgs& a, int bx, int by, int gx) {
  if (side == 0) pm_left_f32_body<NB, left_tr(NB), WM, VEC, left_pf(NB)>(a, bx, by, gx);
  else pm_right_f32_body<NB, right_mc(NB), WM, VEC, right_pf(NB)>(a, bx, by, gx);
}

// Persistent batched form: work-group b takes items b, b + gridDim.x, ...; each
// item is one (M tile, split) work-group of a recorded stand-alone launch.
__global__ __launch_bounds__(NT, 1) void pm_f32_batch_kernel(const BItem* __restrict__ items,
                                                             const int* __restrict__ count,
                                                             const KOp* __restrict__ ops) {
  const int n = *count;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const BItem it = items[i];
    const KOp& op = ops[it.op];
    const int v = op.variant, side = v / 1000;
    switch (v % 1000) {
      case 141: body_for<1, 4, true>(side, op.u.pm, it.bx, it.by, op.gx); break;
      case 140: body_for<1, 4, false>(side, op.u.pm, it.bx, it.by, op.gx); break;
      case 111: body_for<1, 1, true>(side, op.u.pm, it.bx, it.by, op.gx); break;
      case 110: body_for<1, 1, false>(side, op.u.pm, it.bx, it.by, op.gx); break;
      case 241: body_for<2, 4, true>(side, op.u.pm, it.bx, it.by, op.gx); break;
      case 240: body_for<2, 4, false>(side, op.u.pm, it.bx, it.by, op.gx); break;
      case 211: body_for<2, 1, true>(side, op.u.pm, it.bx, it.by, op.gx); break;
      case 210: body_for<2, 1, false>(side, op.u.pm, it.bx, it.by, op.gx); break;
      case 441: body_for<4, 4, true>(side, op.u.pm, it.bx, it.by, op.gx); break;
      case 440: body_for<4, 4, false>(side, op.u.pm, it.bx, it.by, op.gx); break;
      case 411: body_for<4, 1, true>(side, op.u.pm, it.bx, it.by, op.gx); break;
      case 410: body_for<4, 1, false>(side, op.u.pm, it.bx, it.by, op.gx); break;
      default: break;
    }
    __syncthreads();  // LDS is reused by the next item
  }
}

size_t reduce_lds(int side, int nb, int wm) {
  if (wm >= 4) return 0;
  const int nacc = side == 0 ? left_tr(nb) * nb : right_mc(nb) * nb;
  return (size_t)wm * nacc * 4 * 64 * sizeof(double);
}

}  // namespace

int pm_f32_wave_rows(int side, int nb) { return side == 0 ? 16 * left_tr(nb) : 16 * right_mc(nb); }
int pm_f32_kstep(int side) { return side == 0 ? 16 : 32; }

static bool f32_vec(const PmArgs& a, int side) {
  // Fast path: vector loads with no masked lanes. Left: 16-byte row loads need an
  // aligned base and I_L % 4 == 0. Both sides: I1 must be a multiple of the
  // k-step so the zero-padded tail of H_1 never occurs.
  bool vec = ((uintptr_t)a.X % 16 == 0) && (a.IL % 4 == 0);
  return vec && (a.I1 % pm_f32_kstep(side) == 0);
}

hipError_t pm_launch_f32(const PmLaunch& L, const PmArgs& a, const Sink& sk) {
  const int wm = L.mtile / pm_f32_wave_rows(L.side, L.nb);
  const int variant = L.side * 1000 + L.nb * 100 + wm * 10 + (f32_vec(a, L.side) ? 1 : 0);
  const void* k = select_variant(variant);
  if (!k) return hipErrorInvalidValue;
  size_t lds = L.lds_bytes;
  if (reduce_lds(L.side, L.nb, wm) > lds) lds = reduce_lds(L.side, L.nb, wm);
  if (sk.rec) {
    KOp op{};
    op.kind = K_PM_F32;
    op.variant = variant;
    op.gx = (unsigned)L.mtiles;
    op.gy = (unsigned)L.nsplit;
    op.lds = (unsigned)lds;
    op.u.pm = a;
    return sink_record(sk, op);
  }
  void* args[] = {(void*)&a};
  return hipLaunchKernel(k, dim3(L.mtiles, L.nsplit), dim3(NT), args, lds, sk.st);
}

hipError_t batch_launch_pm_f32(const BItem* items, const int* count, const KOp* ops, unsigned grid, size_t lds,
                               hipStream_t st) {
  static bool attr = [] {
    (void)hipFuncSetAttribute((const void*)pm_f32_batch_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    (void)hipGetLastError();
    return true;
  }();
  (void)attr;
  hipLaunchKernelGGL(pm_f32_batch_kernel, dim3(grid), dim3(NT), lds, st, items, count, ops);
  return hipGetLastError();
}

}  // namespace nncpk
