// Partial MTTKRP on MFMA for BF16 / FP16 tensors (the root edges of the
// dimension tree, Section IV-A, Figure 2a), same contraction as the FP32
// kernels: T = X_[L] * K (left node) or T = X_[L]^T * K (right node).
// Included by one translation unit per storage type (pm16_bf16.hip,
// pm16_f16.hip), which instantiates the kernels for that type only.
//
// Design (gfx950, wave64, v_mfma_f32_16x16x32_{bf16,f16}):
//  * The tensor is streamed in its 16-bit storage type, halving HBM traffic; the
//    MFMA accumulates in FP32.
//  * The first contracted factor H_1 is the other MFMA operand. So that the
//    only rounding the 16-bit path adds is the tensor's own storage, H_1 is
//    split into a sum of values of the tensor's 16-bit type, one MFMA per term
//    and tile: hi + lo for FP16 (2 x 11 significant bits), hi + mid + lo for
//    BF16 (3 x 8 bits), each as exact as an FP32 value. Each column is first
//    scaled by a power of two that puts its largest entry near 2^14 (FP16
//    keeps full precision there; the scale is undone exactly in the column
//    factor). A small pack kernel writes the terms once per launch;
//    work-groups copy their i1 block of them into LDS.
//  * The rest of the Khatri-Rao row, Krest(j, :) times the 1/lambda column
//    scales, is applied per output column when the FP32 sum over one j's
//    i1 block is added into the FP32 accumulators.
//  * Left side: each lane loads 8 (or 4) consecutive rows m from each of 8
//    columns k of X and transposes them in registers into the MFMA's 8-k
//    operand. Right side: k is contiguous, so one 16-byte load is the operand.
//  * Loads are vector loads for any shape (element-aligned): padded i1 reads
//    the next j's columns against zero rows of H_1, rows past the output read
//    into the next column and feed outputs that are never stored; the one
//    k-step that could read past the tensor's end loads element by element.
//  * When one LDS block cannot hold all of I1 and the output is tall (the
//    right node of a tensor whose first mode is long), a work-group walks the
//    i1 blocks in turn and restages LDS between them, instead of splitting K
//    and paying for split-K partials of the tall output.
#pragma once

#include "pm_common.hpp"

namespace nncpk {
namespace pm16 {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));

template <int DT>
struct T16;
template <>
struct T16<NNCP_BF16> {
  static __device__ __forceinline__ f4 mfma(u4 a, u4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0,
                                                   0);
  }
  static __device__ __forceinline__ unsigned short enc(float x) {
    return __builtin_bit_cast(unsigned short, (__bf16)x);
  }
  static __device__ __forceinline__ float dec(unsigned short u) { return (float)__builtin_bit_cast(__bf16, u); }
};
template <>
struct T16<NNCP_F16> {
  static __device__ __forceinline__ f4 mfma(u4 a, u4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a), __builtin_bit_cast(h8, b), c, 0, 0, 0);
  }
  static __device__ __forceinline__ unsigned short enc(float x) {
    return __builtin_bit_cast(unsigned short, (_Float16)x);
  }
  static __device__ __forceinline__ float dec(unsigned short u) { return (float)__builtin_bit_cast(_Float16, u); }
};

// One block per packed column r (RP blocks). Column r of H_1 (r < R) is scaled by
// 2^e so that its largest magnitude lies in [2^13, 2^14), then split term by
// term: t_0 = round(v), t_1 = round(v - t_0), t_2 = round(v - t_0 - t_1) (each
// difference is exact in FP32); rows I1..I1pad-1 and columns r >= R are 0.
// hscale[r] = 2^-e.
template <int DT>
__device__ __forceinline__ void pack_body(const PackArgs& pa, int r) {
  __shared__ float red[256];
  const float* __restrict__ H1 = pa.H1;
  const int I1 = pa.I1, I1pad = pa.I1pad, R = pa.R, col0 = pa.col0, RP = pa.RP;
  unsigned short* __restrict__ pack = pa.pack;
  float* __restrict__ hscale = pa.hscale;
  const bool live = r < R;
  const float* h = H1 + (int64_t)I1 * (col0 + r);
  float mx = 0.f;
  if (live)
    for (int i = threadIdx.x; i < I1; i += 256) mx = fmaxf(mx, fabsf(h[i]));
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  mx = red[0];
  int e = 0;
  if (mx > 0.f) {
    int ex;
    (void)frexpf(mx, &ex);  // mx = f * 2^ex, f in [0.5, 1)
    e = 14 - ex;
    e = e < -120 ? -120 : (e > 120 ? 120 : e);
  }
  const float up = ldexpf(1.f, e);
  constexpr int NTM = pm16_terms(DT);
  for (int i = threadIdx.x; i < I1pad; i += 256) {
    float v = (live && i < I1) ? h[i] * up : 0.f;
#pragma unroll
    for (int t = 0; t < NTM; ++t) {
      const unsigned short u = T16<DT>::enc(v);
      pack[(size_t)(t * RP + r) * I1pad + i] = u;
      v -= T16<DT>::dec(u);
    }
  }
  if (threadIdx.x == 0) hscale[r] = live ? ldexpf(1.f, -e) : 0.f;
}

// Per-(j, column) factors of a work-group's j block: Krest(j0 + jj, col0 + r)
// times the column's 1/lambda product times the pack scale, in FP32: from the
// launch's FP64 scale table when there is one (the product and the rounding to
// FP32 are then done here, as pm_fill_scales does them), else computed here.
__device__ __forceinline__ void scales(const PmArgs& a, float* sc, int RP, int64_t j0, int jn) {
  if (!a.sctab) {
    pm_fill_scales<float>(a, sc, RP, j0, jn, a.hscale);
    return;
  }
  typedef double d2 __attribute__((ext_vector_type(2)));
  const d2* src = (const d2*)(a.sctab + j0 * RP);
  const int total = jn * RP / 2;  // RP is a multiple of 16
  constexpr int CH = 4;
  for (int e0 = threadIdx.x; e0 < total; e0 += NT * CH) {
    d2 v[CH];
    float hs[CH][2];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int e = e0 + NT * c < total ? e0 + NT * c : 0;
      v[c] = src[e];
      const int r = (2 * e) % RP;  // even: r and r + 1 lie in one row
      hs[c][0] = a.hscale[r < a.R ? r : 0];
      hs[c][1] = a.hscale[r + 1 < a.R ? r + 1 : 0];
    }
#pragma unroll
    for (int c = 0; c < CH; ++c)
      if (e0 + NT * c < total) {
        const int e = e0 + NT * c;
        const int r = (2 * e) % RP;
        sc[2 * e] = r < a.R ? (float)(v[c][0] * (double)hs[c][0]) : 0.f;
        sc[2 * e + 1] = r + 1 < a.R ? (float)(v[c][1] * (double)hs[c][1]) : 0.f;
      }
  }
}

// Copy rows [i1_0, i1_0 + i1n) of the NTM packed factor terms into LDS (pitch
// lp): 16-byte chunks, eight loads in flight per thread before they are stored
// (sixteen measured no faster on the tall right nodes).
template <int NTM>
__device__ __forceinline__ void stage(const PmArgs& a, unsigned short* hs, int lp, int RP, int i1_0, int i1n) {
  const int chunks = i1n >> 3;
  const int total = NTM * RP * chunks;
  constexpr int CH = 8;
  const int drow = NT / chunks, dc = NT - drow * chunks;
  int row = threadIdx.x / chunks, c = threadIdx.x - row * chunks;
  for (int e0 = threadIdx.x; e0 < total; e0 += NT * CH) {
    u4 v[CH];
    int dst[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const bool ok = e0 + NT * q < total;
      v[q] = *(const u4*)&a.hpack[ok ? (size_t)row * a.I1pad + i1_0 + 8 * c : 0];
      dst[q] = ok ? row * lp + 8 * c : -1;
      row += drow;
      c += dc;
      if (c >= chunks) {
        c -= chunks;
        ++row;
      }
    }
#pragma unroll
    for (int q = 0; q < CH; ++q)
      if (dst[q] >= 0) *(u4*)&hs[dst[q]] = v[q];
  }
}

// Sum the FP32 accumulators across the waves sharing an M range (in FP64).
template <int NACC>
__device__ __forceinline__ void reduce_waves(float (&accf)[NACC][4], double* lds, int wk, int wm, int WK) {
  if (WK == 1) return;
  double acc[NACC][4];
#pragma unroll
  for (int v = 0; v < NACC; ++v)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[v][e] = (double)accf[v][e];
  __syncthreads();
  wave_reduce_k<NACC>(acc, lds, wk, wm, WK);
#pragma unroll
  for (int v = 0; v < NACC; ++v)
#pragma unroll
    for (int e = 0; e < 4; ++e) accf[v][e] = (float)acc[v][e];
}

// Rows per left wave = 16 * TR, columns per right wave = 16 * MC.
constexpr int left_tr16(int nb) { return nb >= 4 ? 4 : 8; }
constexpr int right_mc16(int nb) { return 4; }
constexpr int right_mc16_j1(int nb) { return nb >= 4 ? 9 : 8; }
constexpr int right_pf16_j1(int nb) { return nb >= 4 ? 2 : 3; }
constexpr int left_pf16(int nb) { return 3; }
constexpr int right_pf16(int nb) { return 3; }

// ----------------------------------------------------------------------------
// Left side: T(m, r) = sum_k X[m + IL*k] K(k, r). A wave covers 16*TR rows m. In
// a k-step (32 consecutive i1 of one j) lane (li, lq) loads rows
// TR*li .. TR*li+TR-1 of the 8 columns i1 = base + 8*lq + e; MFMA tile tt takes
// row TR*li + tt of those 8 loads as its 8-k operand.
// ----------------------------------------------------------------------------
template <int DT, int NB, bool FAST, bool MT, bool NTL>
__device__ __forceinline__ void left_body(const PmArgs& a, int bx, int by) {
  constexpr int RP = NB * 16;
  constexpr int TR = left_tr16(NB);
  constexpr int D = left_pf16(NB);
  constexpr int KS = 32;
  constexpr int NACC = TR * NB;
  constexpr int WROWS = 16 * TR;
  constexpr int NTM = pm16_terms(DT);
  using vT = u16v<TR>;
  extern __shared__ double lds_d[];
  const int lp = a.i1blk + 8;
  unsigned short* hs = (unsigned short*)lds_d;
  float* sc = (float*)(hs + NTM * RP * lp);

  const int WM = a.wm, WK = 4 / WM;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave % WM, wk = wave / WM;
  const int li = lane & 15, lq = lane >> 4;
  const int64_t Mtot = a.IL, Ktot = a.IR;
  const int mtile = WM * WROWS;
  // the group's M tiles tile0 .. tile0 + ntile - 1 (ntile > 1 only with WK == 1),
  // streamed as one sequence of k-steps per wave
  const int tile0 = MT ? bx * a.mper : bx;
  const int ntile = MT ? min(a.mper, a.mtiles - tile0) : 1;
  const int ib = by % a.n_i1blk, jb = by / a.n_i1blk;
  const int i1_0 = ib * a.i1blk;
  const int i1n = min(a.i1blk, a.I1pad - i1_0);
  const int64_t j0 = (int64_t)jb * a.jblk;
  const int jn = (int)min((int64_t)a.jblk, a.J - j0);
  const unsigned short* X = (const unsigned short*)a.X;

  stage<NTM>(a, hs, lp, RP, i1_0, i1n);
  scales(a, sc, RP, j0, jn);
  __syncthreads();

  const int S1 = i1n / KS;
  int sb, se;
  wave_range(S1 * jn, wk, WK, &sb, &se);
  se += (ntile - 1) * S1 * jn;

  float acc[NACC][4];
#pragma unroll
  for (int v = 0; v < NACC; ++v)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[v][e] = 0.f;

  // lane's first row in the tile being loaded; a row group wholly past the
  // output reads row 0
  int64_t m = (int64_t)tile0 * mtile + wm * WROWS + TR * li;
  int64_t mload = m < Mtot ? m : 0;
  const int ilim = a.I1 - i1_0;
  const unsigned short* zeros = (const unsigned short*)a.zeros;
  // The vector loads of a step read elements up to Mtot * (colbase + KS) + TR - 2
  // (row group start <= Mtot - 1, TR rows, in the step's last column): all of
  // them lie inside the tensor while Mtot * (colbase + KS) <= vec_lim.
  const int64_t vec_lim = Mtot * Ktot - (TR - 1);

  const int jrot = (WK == 1 && jn > 1) ? (int)(((unsigned)bx * 5u) % (unsigned)jn) : 0;
  int jcntL = sb / S1, tileL = 0;
  int jl = jcntL + jrot, tl = sb - jcntL * S1;
  if (jl >= jn) jl -= jn;
  auto load = [&](vT (&A)[8]) {
    const int64_t colbase = (int64_t)a.I1 * (j0 + jl) + i1_0 + KS * tl;
    const unsigned short* base = X + Mtot * (colbase + 8 * lq);
    if (FAST || Mtot * (colbase + KS) <= vec_lim) {  // uniform
#pragma unroll
      for (int e = 0; e < 8; ++e) A[e] = tload<NTL>((const vT*)(base + Mtot * e + mload));
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        // per lane: the whole row group of a real column in one vector load,
        // else element by element (rows past the output, padded i1: zero)
        const bool kv = (KS * tl + 8 * lq + e) < ilim;
        vT v;
        if (kv && m + TR <= Mtot) {
          v = *(const vT*)(base + Mtot * e + m);
        } else {
#pragma unroll
          for (int t = 0; t < TR; ++t) {
            const unsigned short* p = (kv && m + t < Mtot) ? base + Mtot * e + m + t : zeros;
            v[t] = *p;
          }
        }
        A[e] = v;
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

  const bool direct = (a.nsplit == 1);
  const int64_t Mpad = (int64_t)a.mtiles * mtile;
  auto store_tile = [&](int64_t mw) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double o[TR];
#pragma unroll
        for (int tt = 0; tt < TR; ++tt) o[tt] = (double)acc[tt * NB + nb][v];
        pm_store_rows<TR>(a, direct, Mtot, Mpad, RP, by, 16 * nb + li, mw + TR * (4 * lq + v), o);
      }
  };

  f4 c32[TR][NB];
#pragma unroll
  for (int tt = 0; tt < TR; ++tt)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) c32[tt][nb] = f4{0.f, 0.f, 0.f, 0.f};
  int jc = jl, tc = tl, jcntC = jcntL, tileC = 0, left = se - sb;
  auto compute = [&](const vT (&A)[8]) {
    const int kk = KS * tc + 8 * lq;
    u4 B[NTM][NB];
#pragma unroll
    for (int t = 0; t < NTM; ++t)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) B[t][nb] = *(const u4*)&hs[(t * RP + 16 * nb + li) * lp + kk];
    u4 av[TR];
#pragma unroll
    for (int tt = 0; tt < TR; ++tt)
#pragma unroll
      for (int w = 0; w < 4; ++w) av[tt][w] = (unsigned)A[2 * w][tt] | ((unsigned)A[2 * w + 1][tt] << 16);
#pragma unroll
    for (int t = 0; t < NTM; ++t)
#pragma unroll
      for (int tt = 0; tt < TR; ++tt)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) c32[tt][nb] = T16<DT>::mfma(av[tt], B[t][nb], c32[tt][nb]);
    --left;
    if (tc + 1 == S1 || left == 0) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const float s = sc[jc * RP + 16 * nb + li];
#pragma unroll
        for (int tt = 0; tt < TR; ++tt) {
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[tt * NB + nb][e] = __builtin_fmaf(c32[tt][nb][e], s, acc[tt * NB + nb][e]);
          c32[tt][nb] = f4{0.f, 0.f, 0.f, 0.f};
        }
      }
    }
    if (++tc == S1) {
      tc = 0;
      if (++jc == jn) jc = 0;
      if (MT && ++jcntC == jn) {
        jcntC = 0;
        if (tileC + 1 < ntile) {  // a tile done (its last j scaled above): store it, start the next
          store_tile((int64_t)(tile0 + tileC) * mtile + wm * WROWS);
#pragma unroll
          for (int v = 0; v < NACC; ++v)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[v][e] = 0.f;
          ++tileC;
        }
      }
    }
  };

  vT A[D][8];
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

  reduce_waves<NACC>(acc, lds_d, wk, wm, WK);
  if (wk != 0) return;
  store_tile((int64_t)(tile0 + ntile - 1) * mtile + wm * WROWS);
}

// ----------------------------------------------------------------------------
// Right side: T(c, r) = sum_k X[k + IL*c] K(k, r); k is contiguous. A wave covers
// MC groups of 16 columns c. In a k-step (64 consecutive i1 of one j) lane
// (li, lq) loads k = base + 32h + 8*lq .. +7 (h = 0, 1) of column group + li.
// The work-group walks `istages` i1 blocks (j inside each), restaging LDS
// between them; istages > 1 only with every wave on its own columns (WM = 4).
// J1: the remaining contracted extent is 1, so the Khatri-Rao scale is one
// factor per column: the MFMA sums run over all of K (FP32) and are scaled once
// at the end, with no separate accumulators (every wave owns its columns).
// ----------------------------------------------------------------------------
template <int DT, int NB, bool J1, bool FAST, bool MT, bool NTL>
__device__ __forceinline__ void right_body(const PmArgs& a, int bx, int by) {
  constexpr int RP = NB * 16;
  constexpr int MC = J1 ? right_mc16_j1(NB) : right_mc16(NB);
  constexpr int D = J1 ? right_pf16_j1(NB) : right_pf16(NB);
  constexpr int KS = 64;
  constexpr int NACC = MC * NB;
  constexpr int NTM = pm16_terms(DT);
  using vT = u16v<8>;
  extern __shared__ double lds_d[];
  const int lp = a.i1blk + 8;
  unsigned short* hs = (unsigned short*)lds_d;
  float* sc = (float*)(hs + NTM * RP * lp);

  const int WM = J1 ? 4 : a.wm, WK = 4 / WM;
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
  const unsigned short* X = (const unsigned short*)a.X;

  // stage geometry: all stages have i1blk rows except possibly the last
  auto stage_rows = [&](int st) { return min(a.i1blk, a.I1pad - (ib0 + st) * a.i1blk); };

  stage<NTM>(a, hs, lp, RP, ib0 * a.i1blk, stage_rows(0));
  scales(a, sc, RP, j0, jn);
  __syncthreads();

  int total = 0;
  for (int st = 0; st < a.istages; ++st) total += (stage_rows(st) / KS) * jn;
  int sb, se;
  wave_range(total, wk, WK, &sb, &se);  // istages > 1 implies WK == 1: the whole range
  se += (ntile - 1) * total;

  float acc[NACC][4];
#pragma unroll
  for (int v = 0; v < NACC; ++v)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[v][e] = 0.f;

  // Columns of the tile being loaded (columns past the output read column 0).
  // The vector loads of a step read elements up to Ktot * cmax + lbase + KS - 1
  // (cmax: the wave's last column that is read, lane offsets up to KS - 1): all
  // of them lie inside the tensor while lbase <= vec_lim.
  const unsigned short* colp[MC];
  int64_t vec_lim;
  auto set_tile = [&](int t) {
    const int64_t cw = (int64_t)(tile0 + t) * mtile + wm * 16 * MC;
#pragma unroll
    for (int g = 0; g < MC; ++g) {
      const int64_t c = cw + 16 * g + li;
      colp[g] = X + Ktot * (c < Mtot ? c : 0) + 8 * lq;
    }
    const int64_t cmax = min(cw + 16 * MC - 1, Mtot - 1);
    vec_lim = Mtot * Ktot - Ktot * cmax - KS;  // wave-uniform
  };
  set_tile(0);
  const unsigned short* zeros = (const unsigned short*)a.zeros;

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
        for (int g = 0; g < MC; ++g) A[g][h] = tload<NTL>((const vT*)(colp[g] + lbase + 32 * h));
    } else {
      const int ilimL = a.I1 - i1s;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int off = KS * tl + 32 * h + 8 * lq;
#pragma unroll
        for (int g = 0; g < MC; ++g) {
          // per lane: eight real k in one vector load, else element by element
          // (padded i1 reads zero)
          vT v;
          if (off + 8 <= ilimL) {
            v = *(const vT*)(colp[g] + lbase + 32 * h);
          } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              const unsigned short* p = (off + e < ilimL) ? colp[g] + lbase + 32 * h + e : zeros;
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

  f4 c32[MC][NB];
#pragma unroll
  for (int g = 0; g < MC; ++g)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) c32[g][nb] = f4{0.f, 0.f, 0.f, 0.f};

  // J1: the MFMA sums of the whole K range times the one Khatri-Rao scale per column
  auto finish_j1 = [&]() {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const float s = sc[16 * nb + li];
#pragma unroll
      for (int g = 0; g < MC; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[g * NB + nb][e] = c32[g][nb][e] * s;
    }
  };
  const bool direct = (a.nsplit == 1);
  const int64_t Mpad = (int64_t)a.mtiles * mtile;
  auto store_tile = [&](int64_t cw) {
#pragma unroll
    for (int g = 0; g < MC; ++g)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        double o[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) o[v] = (double)acc[g * NB + nb][v];
        pm_store_rows<4>(a, direct, Mtot, Mpad, RP, by, 16 * nb + li, cw + 16 * g + 4 * lq, o);
      }
  };
  int stC = 0, S1C = S1L, jc = jl, tc = tl, jcntC = jcntL, tileC = 0, left = se - sb;
  auto compute = [&](const vT (&A)[MC][2]) {
    const int kk = KS * tc + 8 * lq;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      u4 B[NTM][NB];
#pragma unroll
      for (int t = 0; t < NTM; ++t)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) B[t][nb] = *(const u4*)&hs[(t * RP + 16 * nb + li) * lp + kk + 32 * h];
#pragma unroll
      for (int t = 0; t < NTM; ++t)
#pragma unroll
        for (int g = 0; g < MC; ++g)
#pragma unroll
          for (int nb = 0; nb < NB; ++nb)
            c32[g][nb] = T16<DT>::mfma(__builtin_bit_cast(u4, A[g][h]), B[t][nb], c32[g][nb]);
    }
    --left;
    if (!J1 && (tc + 1 == S1C || left == 0)) {
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const float s = sc[jc * RP + 16 * nb + li];
#pragma unroll
        for (int g = 0; g < MC; ++g) {
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[g * NB + nb][e] = __builtin_fmaf(c32[g][nb][e], s, acc[g * NB + nb][e]);
          c32[g][nb] = f4{0.f, 0.f, 0.f, 0.f};
        }
      }
    }
    if (++tc == S1C) {
      tc = 0;
      if (++jc == jn) jc = 0;
      if (++jcntC == jn) {
        jcntC = 0;
        if (++stC < a.istages && left > 0) {
          // next i1 block: every wave of the group gets here at the same step
          __syncthreads();
          stage<NTM>(a, hs, lp, RP, (ib0 + stC) * a.i1blk, stage_rows(stC));
          __syncthreads();
          S1C = stage_rows(stC) / KS;
        } else if (MT && tileC + 1 < ntile) {  // a tile done (istages == 1): store it, start the next
          stC = 0;
          if (J1) {
            finish_j1();
#pragma unroll
            for (int g = 0; g < MC; ++g)
#pragma unroll
              for (int nb = 0; nb < NB; ++nb) c32[g][nb] = f4{0.f, 0.f, 0.f, 0.f};
          }
          store_tile((int64_t)(tile0 + tileC) * mtile + wm * 16 * MC);
#pragma unroll
          for (int v = 0; v < NACC; ++v)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[v][e] = 0.f;
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

  if (J1) finish_j1();
  else reduce_waves<NACC>(acc, lds_d, wk, wm, WK);
  if (wk != 0) return;
  store_tile((int64_t)(tile0 + ntile - 1) * mtile + wm * 16 * MC);
}

// FAST: the shape guarantees that every vector load of every step lies inside
// the tensor (pm16_fast), so the loads need no per-step check. NTL: tensor loads
// with the streaming hint (stand-alone launches; see pm_f32_body).
template <int DT, int SIDE, int NB, bool J1, bool FAST, bool MT, bool NTL>
__device__ __forceinline__ void body(const PmArgs& a, int bx, int by) {
  if (SIDE == 0) left_body<DT, NB, FAST, MT, NTL>(a, bx, by);
  else right_body<DT, NB, J1, FAST, MT, NTL>(a, bx, by);
}

// Stand-alone kernels: one work-group per (M tile, split).
template <int DT, int SIDE, int NB, bool J1, bool FAST, bool MT>
__global__ __launch_bounds__(NT, 1) void pm16_kernel_std(PmArgs a) {
  body<DT, SIDE, NB, J1, FAST, MT, true>(a, blockIdx.x, blockIdx.y);
}
// Persistent batched form: items grp[0] + b, grp[0] + b + gridDim.x, ... below
// grp[0] + grp[1], each one (M tile, split) work-group of a recorded launch.
template <int DT, int SIDE, int NB, bool J1, bool FAST, bool MT>
__global__ __launch_bounds__(NT, 1) void pm16_kernel_items(const BItem* __restrict__ items,
                                                           const int* __restrict__ grp,
                                                           const KOp* __restrict__ ops) {
  const int off = grp[0], n = grp[1];
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const BItem it = items[off + i];
    const KOp& op = ops[it.op];
    body<DT, SIDE, NB, J1, FAST, MT, false>(op.u.pm, it.bx, it.by);
    __syncthreads();  // LDS is reused by the next item
  }
}

template <int DT>
__global__ __launch_bounds__(256) void pack_kernel_std(PackArgs pa) {
  pack_body<DT>(pa, blockIdx.x);
}
template <int DT>
__global__ __launch_bounds__(256) void pack_kernel_items(const BItem* __restrict__ items, const int* __restrict__ grp,
                                                         const KOp* __restrict__ ops) {
  const int off = grp[0], n = grp[1];
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const BItem it = items[off + i];
    pack_body<DT>(ops[it.op].u.pk, it.bx);
    __syncthreads();
  }
}

template <int DT, int SIDE, bool J1, bool FAST, bool MT>
const void* pick(int nb, bool batch) {
  switch (nb) {
    case 1:
      return batch ? (const void*)pm16_kernel_items<DT, SIDE, 1, J1, FAST, MT>
                   : (const void*)pm16_kernel_std<DT, SIDE, 1, J1, FAST, MT>;
    case 2:
      return batch ? (const void*)pm16_kernel_items<DT, SIDE, 2, J1, FAST, MT>
                   : (const void*)pm16_kernel_std<DT, SIDE, 2, J1, FAST, MT>;
    case 4:
      if constexpr (J1 && MT) {
        return nullptr;  // not planned: the J == 1 kernel at four column blocks has no registers to spare
      } else {
        return batch ? (const void*)pm16_kernel_items<DT, SIDE, 4, J1, FAST, MT>
                     : (const void*)pm16_kernel_std<DT, SIDE, 4, J1, FAST, MT>;
      }
    default: return nullptr;
  }
}

template <int DT, bool FAST, bool MT>
const void* pick_side(int side, int nb, int j1, bool batch) {
  if (j1) return side == 1 ? pick<DT, 1, true, FAST, MT>(nb, batch) : nullptr;
  return side == 0 ? pick<DT, 0, false, FAST, MT>(nb, batch) : pick<DT, 1, false, FAST, MT>(nb, batch);
}

template <int DT, bool MT>
const void* pick_fast(int side, int nb, int j1, int fast, bool batch) {
  return fast ? pick_side<DT, true, MT>(side, nb, j1, batch) : pick_side<DT, false, MT>(side, nb, j1, batch);
}

}  // namespace pm16

// Kernel of (side, column blocks, J == 1 form, unchecked loads), stand-alone or
// batched, in the one-tile (MT false) or several-tile form.
template <int DT, bool MT>
const void* pm16_kernel_form(int side, int nb, int j1, int fast, bool batch) {
  return pm16::pick_fast<DT, MT>(side, nb, j1, fast, batch);
}
template <int DT>
const void* pm16_pack_kernel(bool batch) {
  return batch ? (const void*)pm16::pack_kernel_items<DT> : (const void*)pm16::pack_kernel_std<DT>;
}

}  // namespace nncpk
