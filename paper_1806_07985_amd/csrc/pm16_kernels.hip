// Partial MTTKRP on MFMA for BF16 / FP16 tensors (the root edges of the
// dimension tree, Section IV-A, Figure 2a), same contraction as the FP32
// kernels: T = X_[L] * K (left node) or T = X_[L]^T * K (right node).
//
// Design (gfx950, wave64, v_mfma_f32_16x16x32_{bf16,f16}):
//  * The tensor is streamed in its 16-bit storage type, halving HBM traffic; the
//    MFMA accumulates in FP32.
//  * The first contracted factor H_1 is the other MFMA operand. So that the
//    only rounding the 16-bit path adds is the tensor's own storage, H_1 is
//    split into hi + lo values of the tensor's 16-bit type (two MFMAs per
//    tile), after scaling each column by a power of two that puts its largest
//    entry near 2^14 (FP16 keeps full precision there; the scale is undone
//    exactly in the column factor). A small pack kernel writes this pair once
//    per launch; work-groups copy their i1 block of it into LDS.
//  * The rest of the Khatri-Rao row, Krest(j, :) times the 1/lambda column
//    scales, is applied per output column when the FP32 sum over one j's
//    i1 block is added into the FP32 accumulators.
//  * Left side: each lane loads 8 consecutive rows m (16 bytes) from each of 8
//    columns k of X and transposes them in registers into the MFMA's 8-k
//    operand. Right side: k is contiguous, so one 16-byte load is the operand.
//  * When one LDS block cannot hold all of I1 and the output is tall (the
//    right node of a tensor whose first mode is long), a work-group walks the
//    i1 blocks in turn and restages LDS between them, instead of splitting K
//    and paying for split-K partials of the tall output.
#include "pm_common.hpp"

namespace nncpk {
namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));
typedef unsigned short us4 __attribute__((ext_vector_type(4)));

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
// 2^e so that its largest magnitude lies in [2^13, 2^14), then split as
// hi = round(v), lo = round(v - hi); rows I1..I1pad-1 and columns r >= R are 0.
// hscale[r] = 2^-e.
template <int DT>
__device__ __forceinline__ void pm16_pack_body(const PackArgs& pa, int r) {
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
  unsigned short* hi = pack + (size_t)r * I1pad;
  unsigned short* lo = pack + (size_t)(RP + r) * I1pad;
  for (int i = threadIdx.x; i < I1pad; i += 256) {
    const float v = (live && i < I1) ? h[i] * up : 0.f;
    const unsigned short uh = T16<DT>::enc(v);
    hi[i] = uh;
    lo[i] = T16<DT>::enc(v - T16<DT>::dec(uh));
  }
  if (threadIdx.x == 0) hscale[r] = live ? ldexpf(1.f, -e) : 0.f;
}

template <int DT>
__global__ __launch_bounds__(256) void pm16_pack_kernel(PackArgs pa) {
  pm16_pack_body<DT>(pa, blockIdx.x);
}

// Per-(j, column) factors of a work-group's j block: Krest(j0 + jj, col0 + r)
// times the column's 1/lambda product times the pack scale, in FP32.
__device__ __forceinline__ void pm16_scales(const PmArgs& a, float* sc, int RP, int64_t j0, int jn) {
  pm_fill_scales<float>(a, sc, RP, j0, jn, a.hscale);
}

// Copy rows [i1_0, i1_0 + i1n) of the packed hi/lo factor into LDS (pitch lp):
// 16-byte chunks, eight loads in flight per thread before they are stored.
__device__ __forceinline__ void pm16_stage(const PmArgs& a, unsigned short* hs, int lp, int RP, int i1_0, int i1n) {
  const int chunks = i1n >> 3;
  const int total = 2 * RP * chunks;
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

// Sum the FP32 accumulators across the waves sharing an M range and store.
template <int NACC>
__device__ __forceinline__ void pm16_reduce_store(const PmArgs& a, float (&accf)[NACC][4], double* lds, int wk, int wm,
                                                  int WK) {
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

// ----------------------------------------------------------------------------
// Left side: T(m, r) = sum_k X[m + IL*k] K(k, r). A wave covers 16*TR rows m. In
// a k-step (32 consecutive i1 of one j) lane (li, lq) loads rows
// TR*li .. TR*li+TR-1 of the 8 columns i1 = base + 8*lq + e; MFMA tile tt takes
// row TR*li + tt of those 8 loads as its 8-k operand.
// ----------------------------------------------------------------------------
template <int DT, int NB, int TR, int WM, bool FAST, int D>
__device__ __forceinline__ void pm_left_16_body(const PmArgs& a, int bx, int by, int gx) {
  constexpr int RP = NB * 16;
  constexpr int WK = 4 / WM;
  constexpr int KS = 32;
  constexpr int NACC = TR * NB;
  constexpr int WROWS = 16 * TR;
  typedef unsigned short vT __attribute__((ext_vector_type(TR)));
  extern __shared__ double lds_d[];
  const int lp = a.i1blk + 8;
  unsigned short* hs = (unsigned short*)lds_d;
  float* sc = (float*)(hs + 2 * RP * lp);

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave % WM, wk = wave / WM;
  const int li = lane & 15, lq = lane >> 4;
  const int64_t Mtot = a.IL;
  const int mtile = WM * WROWS;
  const int64_t mw = (int64_t)bx * mtile + wm * WROWS;
  const int ib = by % a.n_i1blk, jb = by / a.n_i1blk;
  const int i1_0 = ib * a.i1blk;
  const int i1n = min(a.i1blk, a.I1pad - i1_0);
  const int64_t j0 = (int64_t)jb * a.jblk;
  const int jn = (int)min((int64_t)a.jblk, a.J - j0);
  const unsigned short* X = (const unsigned short*)a.X;

  pm16_stage(a, hs, lp, RP, i1_0, i1n);
  pm16_scales(a, sc, RP, j0, jn);
  __syncthreads();

  const int S1 = i1n / KS;
  int sb, se;
  wave_range(S1 * jn, wk, WK, &sb, &se);

  float acc[NACC][4];
#pragma unroll
  for (int v = 0; v < NACC; ++v)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[v][e] = 0.f;

  const int64_t m = mw + TR * li;
  const int64_t mload = (m + TR <= Mtot) ? m : 0;
  const int ilim = a.I1 - i1_0;
  const unsigned short* zeros = (const unsigned short*)a.zeros;

  const int jrot = (WK == 1 && jn > 1) ? (int)(((unsigned)bx * 5u) % (unsigned)jn) : 0;
  int jl = sb / S1 + jrot, tl = sb - (sb / S1) * S1;
  if (jl >= jn) jl -= jn;
  // Without the unmasked path: on every k-step that lies inside I1, TR-row loads
  // where I_L % TR == 0, else 8-byte loads (4 rows) where I_L % 4 == 0 (every
  // 4-row group is then all in or all out of M); element loads only for the
  // ragged last k-step or odd I_L.
  const bool mid = !FAST && (Mtot % 4 == 0) && ((uintptr_t)a.X % 8 == 0);
  const bool wide = mid && (Mtot % TR == 0) && ((uintptr_t)a.X % (2 * TR) == 0);  // TR-row loads fit
  auto load = [&](vT (&A)[8]) {
    const int64_t colbase = (int64_t)a.I1 * (j0 + jl) + i1_0 + KS * tl + 8 * lq;
    const unsigned short* base = X + Mtot * colbase;
    const bool full = KS * tl + KS <= ilim;  // wave-uniform
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      if (FAST) {
        A[e] = __builtin_nontemporal_load((const vT*)(base + Mtot * e + mload));
      } else if (wide && full) {
        A[e] = __builtin_nontemporal_load((const vT*)(base + Mtot * e + mload));
      } else if (mid && full) {
        vT v;
#pragma unroll
        for (int h = 0; h < TR / 4; ++h) {
          const int64_t mm = (m + 4 * h + 4 <= Mtot) ? m + 4 * h : 0;
          const us4 q = __builtin_nontemporal_load((const us4*)(base + Mtot * e + mm));
#pragma unroll
          for (int t = 0; t < 4; ++t) v[4 * h + t] = q[t];
        }
        A[e] = v;
      } else {
        const bool kv = (KS * tl + 8 * lq + e) < ilim;
        vT v;
#pragma unroll
        for (int t = 0; t < TR; ++t) {
          const unsigned short* p = (kv && m + t < Mtot) ? base + Mtot * e + m + t : zeros;
          v[t] = *p;
        }
        A[e] = v;
      }
    }
    if (++tl == S1) {
      tl = 0;
      if (++jl == jn) jl = 0;
    }
  };

  f4 c32[TR][NB];
#pragma unroll
  for (int tt = 0; tt < TR; ++tt)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) c32[tt][nb] = f4{0.f, 0.f, 0.f, 0.f};
  int jc = jl, tc = tl, left = se - sb;
  auto compute = [&](const vT (&A)[8]) {
    const int kk = KS * tc + 8 * lq;
    u4 Bh[NB], Bl[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      Bh[nb] = *(const u4*)&hs[(16 * nb + li) * lp + kk];
      Bl[nb] = *(const u4*)&hs[(RP + 16 * nb + li) * lp + kk];
    }
    u4 av[TR];
#pragma unroll
    for (int tt = 0; tt < TR; ++tt)
#pragma unroll
      for (int w = 0; w < 4; ++w) av[tt][w] = (unsigned)A[2 * w][tt] | ((unsigned)A[2 * w + 1][tt] << 16);
#pragma unroll
    for (int tt = 0; tt < TR; ++tt)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) c32[tt][nb] = T16<DT>::mfma(av[tt], Bh[nb], c32[tt][nb]);
#pragma unroll
    for (int tt = 0; tt < TR; ++tt)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) c32[tt][nb] = T16<DT>::mfma(av[tt], Bl[nb], c32[tt][nb]);
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

  pm16_reduce_store<NACC>(a, acc, lds_d, wk, wm, WK);
  if (wk != 0) return;
  const bool direct = (a.nsplit == 1);
  const int64_t Mpad = (int64_t)gx * mtile;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double o[TR];
#pragma unroll
      for (int tt = 0; tt < TR; ++tt) o[tt] = (double)acc[tt * NB + nb][v];
      pm_store_rows<TR>(a, direct, Mtot, Mpad, RP, by, 16 * nb + li, mw + TR * (4 * lq + v), o);
    }
}

// ----------------------------------------------------------------------------
// Right side: T(c, r) = sum_k X[k + IL*c] K(k, r); k is contiguous. A wave covers
// MC groups of 16 columns c. In a k-step (64 consecutive i1 of one j) lane
// (li, lq) loads k = base + 32h + 8*lq .. +7 (h = 0, 1) of column group + li.
// The work-group walks `istages` i1 blocks (j inside each), restaging LDS
// between them; istages > 1 only with every wave on its own columns (WM = 4).
// ----------------------------------------------------------------------------
template <int DT, int NB, int MC, int WM, bool FAST, int D, bool J1 = false>
__device__ __forceinline__ void pm_right_16_body(const PmArgs& a, int bx, int by, int gx) {
  // J1: the remaining contracted extent is 1, so the Khatri-Rao scale is one
  // factor per column: the MFMA sums run over all of K (FP32) and are scaled
  // once at the end; no separate accumulators (every wave owns its columns).
  static_assert(!J1 || WM == 4, "J1 needs one wave per column range");
  constexpr int RP = NB * 16;
  constexpr int WK = 4 / WM;
  constexpr int KS = 64;
  constexpr int NACC = MC * NB;
  extern __shared__ double lds_d[];
  const int lp = a.i1blk + 8;
  unsigned short* hs = (unsigned short*)lds_d;
  float* sc = (float*)(hs + 2 * RP * lp);

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave % WM, wk = wave / WM;
  const int li = lane & 15, lq = lane >> 4;
  const int64_t Mtot = a.IR, Ktot = a.IL;
  const int mtile = WM * 16 * MC;
  const int64_t cw = (int64_t)bx * mtile + wm * 16 * MC;
  const int n_i1grp = a.n_i1blk / a.istages;
  const int ib0 = (by % n_i1grp) * a.istages, jb = by / n_i1grp;
  const int64_t j0 = (int64_t)jb * a.jblk;
  const int jn = (int)min((int64_t)a.jblk, a.J - j0);
  const unsigned short* X = (const unsigned short*)a.X;

  // stage geometry: all stages have i1blk rows except possibly the last
  auto stage_rows = [&](int st) { return min(a.i1blk, a.I1pad - (ib0 + st) * a.i1blk); };

  pm16_stage(a, hs, lp, RP, ib0 * a.i1blk, stage_rows(0));
  pm16_scales(a, sc, RP, j0, jn);
  __syncthreads();

  int total = 0;
  for (int st = 0; st < a.istages; ++st) total += (stage_rows(st) / KS) * jn;
  int sb, se;
  wave_range(total, wk, WK, &sb, &se);  // istages > 1 implies WK == 1: the whole range

  float acc[NACC][4];
#pragma unroll
  for (int v = 0; v < NACC; ++v)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[v][e] = 0.f;

  const unsigned short* colp[MC];
#pragma unroll
  for (int g = 0; g < MC; ++g) {
    const int64_t c = cw + 16 * g + li;
    colp[g] = X + Ktot * (c < Mtot ? c : 0) + 8 * lq;
  }
  const unsigned short* zeros = (const unsigned short*)a.zeros;

  // cursor (stage, j, t): t over the stage's k-steps, j over the block (rotated
  // start with one wave along K), stages in order. The load cursor runs D steps
  // ahead and wraps to the start after the last step, so it stays in bounds.
  const int jrot = (WK == 1 && jn > 1) ? (int)(((unsigned)bx * 5u) % (unsigned)jn) : 0;
  int stL = 0, S1L = stage_rows(0) / KS;
  int jl, tl, jcntL;
  {
    // position of step sb within stage 0 (sb > 0 only when istages == 1)
    jcntL = sb / S1L;
    tl = sb - jcntL * S1L;
    jl = jcntL + jrot;
    if (jl >= jn) jl -= jn;
  }
  // Without the unmasked path: on every k-step that lies inside I1, 16-byte loads
  // where column starts allow them (I_L % 8 == 0), else two 8-byte loads per 8 k
  // (I_L % 4 == 0); element loads only for the ragged last k-step or odd I_L.
  const bool mid = !FAST && (Ktot % 4 == 0) && ((uintptr_t)a.X % 8 == 0);
  const bool wide = mid && (Ktot % 8 == 0) && ((uintptr_t)a.X % 16 == 0);  // 16-byte loads fit
  auto load = [&](us8 (&A)[MC][2]) {
    const int ilimL = a.I1 - (ib0 + stL) * a.i1blk;
    const int64_t lbase = (int64_t)a.I1 * (j0 + jl) + (int64_t)(ib0 + stL) * a.i1blk + KS * tl;
    const bool full = KS * tl + KS <= ilimL;  // wave-uniform
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int off = KS * tl + 32 * h + 8 * lq;
#pragma unroll
      for (int g = 0; g < MC; ++g) {
        if (FAST) {
          A[g][h] = __builtin_nontemporal_load((const us8*)(colp[g] + lbase + 32 * h));
        } else if (wide && full) {
          A[g][h] = __builtin_nontemporal_load((const us8*)(colp[g] + lbase + 32 * h));
        } else if (mid && full) {
          const us4* p = (const us4*)(colp[g] + lbase + 32 * h);
          const us4 lo = __builtin_nontemporal_load(p), hi = __builtin_nontemporal_load(p + 1);
          A[g][h] = us8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
        } else {
          us8 v;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const unsigned short* p = (off + e < ilimL) ? colp[g] + lbase + 32 * h + e : zeros;
            v[e] = *p;
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
        if (++stL == a.istages) stL = 0;
        S1L = stage_rows(stL) / KS;
      }
    }
  };

  f4 c32[MC][NB];
#pragma unroll
  for (int g = 0; g < MC; ++g)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) c32[g][nb] = f4{0.f, 0.f, 0.f, 0.f};
  int stC = 0, S1C = S1L, jc = jl, tc = tl, jcntC = jcntL, left = se - sb;
  auto compute = [&](const us8 (&A)[MC][2]) {
    const int kk = KS * tc + 8 * lq;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      u4 Bh[NB], Bl[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        Bh[nb] = *(const u4*)&hs[(16 * nb + li) * lp + kk + 32 * h];
        Bl[nb] = *(const u4*)&hs[(RP + 16 * nb + li) * lp + kk + 32 * h];
      }
#pragma unroll
      for (int g = 0; g < MC; ++g)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          c32[g][nb] = T16<DT>::mfma(__builtin_bit_cast(u4, A[g][h]), Bh[nb], c32[g][nb]);
#pragma unroll
      for (int g = 0; g < MC; ++g)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          c32[g][nb] = T16<DT>::mfma(__builtin_bit_cast(u4, A[g][h]), Bl[nb], c32[g][nb]);
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
          pm16_stage(a, hs, lp, RP, (ib0 + stC) * a.i1blk, stage_rows(stC));
          __syncthreads();
          S1C = stage_rows(stC) / KS;
        }
      }
    }
  };

  us8 A[D][MC][2];
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

  if (J1) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const float s = sc[16 * nb + li];
#pragma unroll
      for (int g = 0; g < MC; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[g * NB + nb][e] = c32[g][nb][e] * s;
    }
  } else {
    pm16_reduce_store<NACC>(a, acc, lds_d, wk, wm, WK);
  }
  if (wk != 0) return;
  const bool direct = (a.nsplit == 1);
  const int64_t Mpad = (int64_t)gx * mtile;
#pragma unroll
  for (int g = 0; g < MC; ++g)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      double o[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) o[v] = (double)acc[g * NB + nb][v];
      pm_store_rows<4>(a, direct, Mtot, Mpad, RP, by, 16 * nb + li, cw + 16 * g + 4 * lq, o);
    }
}

// Rows per left wave = 16 * TR, columns per right wave = 16 * MC.
constexpr int left_tr16(int nb) { return nb >= 4 ? 4 : 8; }
constexpr int right_mc16(int nb) { return nb >= 4 ? 4 : 4; }
constexpr int right_mc16_j1(int nb) { return 8; }
constexpr int right_pf16_j1(int nb) { return nb >= 4 ? 2 : 3; }
constexpr int left_pf16(int nb) { return nb >= 4 ? 3 : 3; }
constexpr int right_pf16(int nb) { return nb >= 4 ? 3 : 3; }

template <int DT, int NB, int TR, int WM, bool FAST, int D>
__global__ __launch_bounds__(NT, 1) void pm_left_16(PmArgs a) {
  pm_left_16_body<DT, NB, TR, WM, FAST, D>(a, blockIdx.x, blockIdx.y, gridDim.x);
}
template <int DT, int NB, int MC, int WM, bool FAST, int D, bool J1>
__global__ __launch_bounds__(NT, 1) void pm_right_16(PmArgs a) {
  pm_right_16_body<DT, NB, MC, WM, FAST, D, J1>(a, blockIdx.x, blockIdx.y, gridDim.x);
}

template <int DT, int NB, int WM, bool VEC>
const void* kernel16(int side) {
  if (side == 0) return (const void*)pm_left_16<DT, NB, left_tr16(NB), WM, VEC, left_pf16(NB)>;
  return (const void*)pm_right_16<DT, NB, right_mc16(NB), WM, VEC, right_pf16(NB), false>;
}
template <int DT, int NB, bool VEC>
const void* kernel16_j1() {
  return (const void*)pm_right_16<DT, NB, right_mc16_j1(NB), 4, VEC, right_pf16_j1(NB), true>;
}

template <int DT>
const void* select16(int side, int nb, int wm, bool vec, bool j1) {
  if (j1) {  // planned only where the unmasked 16-byte path applies
    if (side != 1 || wm != 4 || !vec) return nullptr;
    switch (nb) {
      case 1: return kernel16_j1<DT, 1, true>();
      case 2: return kernel16_j1<DT, 2, true>();
      case 4: return kernel16_j1<DT, 4, true>();
      default: return nullptr;
    }
  }
  switch (nb * 100 + wm * 10 + (vec ? 1 : 0)) {
    case 141: return kernel16<DT, 1, 4, true>(side);
    case 140: return kernel16<DT, 1, 4, false>(side);
    case 111: return kernel16<DT, 1, 1, true>(side);
    case 110: return kernel16<DT, 1, 1, false>(side);
    case 241: return kernel16<DT, 2, 4, true>(side);
    case 240: return kernel16<DT, 2, 4, false>(side);
    case 211: return kernel16<DT, 2, 1, true>(side);
    case 210: return kernel16<DT, 2, 1, false>(side);
    case 441: return kernel16<DT, 4, 4, true>(side);
    case 440: return kernel16<DT, 4, 4, false>(side);
    case 411: return kernel16<DT, 4, 1, true>(side);
    case 410: return kernel16<DT, 4, 1, false>(side);
    default: return nullptr;
  }
}

template <int DT, int NB, int WM, bool VEC>
__device__ __forceinline__ void body16(int side, const PmArgs& a, int bx, int by, int gx) {
  if (side == 0) pm_left_16_body<DT, NB, left_tr16(NB), WM, VEC, left_pf16(NB)>(a, bx, by, gx);
  else pm_right_16_body<DT, NB, right_mc16(NB), WM, VEC, right_pf16(NB)>(a, bx, by, gx);
}
template <int DT, int NB, bool VEC>
__device__ __forceinline__ void body16_j1(const PmArgs& a, int bx, int by, int gx) {
  pm_right_16_body<DT, NB, right_mc16_j1(NB), 4, VEC, right_pf16_j1(NB), true>(a, bx, by, gx);
}

// variant = j1*100000 + bf16*10000 + side*1000 + nb*100 + wm*10 + vec
template <int DT>
__device__ __forceinline__ void dispatch16_j1(int v, const PmArgs& a, int bx, int by, int gx) {
  switch ((v % 1000) / 100) {
    case 1: body16_j1<DT, 1, true>(a, bx, by, gx); break;
    case 2: body16_j1<DT, 2, true>(a, bx, by, gx); break;
    case 4: body16_j1<DT, 4, true>(a, bx, by, gx); break;
    default: break;
  }
}

template <int DT>
__device__ __forceinline__ void dispatch16(int v, const PmArgs& a, int bx, int by, int gx) {
  const int side = (v / 1000) % 10;
  switch (v % 1000) {
    case 141: body16<DT, 1, 4, true>(side, a, bx, by, gx); break;
    case 140: body16<DT, 1, 4, false>(side, a, bx, by, gx); break;
    case 111: body16<DT, 1, 1, true>(side, a, bx, by, gx); break;
    case 110: body16<DT, 1, 1, false>(side, a, bx, by, gx); break;
    case 241: body16<DT, 2, 4, true>(side, a, bx, by, gx); break;
    case 240: body16<DT, 2, 4, false>(side, a, bx, by, gx); break;
    case 211: body16<DT, 2, 1, true>(side, a, bx, by, gx); break;
    case 210: body16<DT, 2, 1, false>(side, a, bx, by, gx); break;
    case 441: body16<DT, 4, 4, true>(side, a, bx, by, gx); break;
    case 440: body16<DT, 4, 4, false>(side, a, bx, by, gx); break;
    case 411: body16<DT, 4, 1, true>(side, a, bx, by, gx); break;
    case 410: body16<DT, 4, 1, false>(side, a, bx, by, gx); break;
    default: break;
  }
}

// Persistent batched form (pack ops and 16-bit partial-MTTKRP tiles).
__global__ __launch_bounds__(NT, 1) void pm16_batch_kernel(const BItem* __restrict__ items,
                                                           const int* __restrict__ count,
                                                           const KOp* __restrict__ ops) {
  const int n = *count;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const BItem it = items[i];
    const KOp& op = ops[it.op];
    if (op.kind == K_PACK16) {
      if (op.variant) pm16_pack_body<NNCP_BF16>(op.u.pk, it.bx);
      else pm16_pack_body<NNCP_F16>(op.u.pk, it.bx);
    } else if ((op.variant / 10000) % 10) {
      dispatch16<NNCP_BF16>(op.variant, op.u.pm, it.bx, it.by, op.gx);
    } else {
      dispatch16<NNCP_F16>(op.variant, op.u.pm, it.bx, it.by, op.gx);
    }
    __syncthreads();
  }
}

// The J == 1 right-node tiles of 16-bit tensors (a family of their own).
__global__ __launch_bounds__(NT, 1) void pm16j1_batch_kernel(const BItem* __restrict__ items,
                                                             const int* __restrict__ count,
                                                             const KOp* __restrict__ ops) {
  const int n = *count;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const BItem it = items[i];
    const KOp& op = ops[it.op];
    if ((op.variant / 10000) % 10) dispatch16_j1<NNCP_BF16>(op.variant, op.u.pm, it.bx, it.by, op.gx);
    else dispatch16_j1<NNCP_F16>(op.variant, op.u.pm, it.bx, it.by, op.gx);
    __syncthreads();
  }
}

size_t reduce_lds16(int side, int nb, int wm) {
  if (wm >= 4) return 0;  // (also every J1 launch: one wave per column range)
  const int nacc = side == 0 ? left_tr16(nb) * nb : right_mc16(nb) * nb;
  return (size_t)wm * nacc * 4 * 64 * sizeof(double);
}

}  // namespace

int pm_16_wave_rows(int side, int nb, int j1) {
  return side == 0 ? 16 * left_tr16(nb) : 16 * (j1 ? right_mc16_j1(nb) : right_mc16(nb));
}
int pm_16_kstep(int side) { return side == 0 ? 32 : 64; }

static bool vec16(const PmArgs& a, int side) {
  // Fast path: 16-byte loads with no masked lanes. Left: 8 rows per load need an
  // aligned base and I_L % 8 == 0. Right: 8 consecutive k per load need column
  // starts aligned (I_L % 8 == 0). Both: I1 a multiple of the k-step.
  const bool vec = ((uintptr_t)a.X % 16 == 0) && (a.IL % 8 == 0);
  return vec && (a.I1 % pm_16_kstep(side) == 0);
}

hipError_t pm_launch_16(const PmLaunch& L, const PmArgs& a, const Sink& sk) {
  const int RP = 16 * L.nb;
  if (!a.hpack || !a.hscale) return hipErrorInvalidValue;
  const bool bf = L.dtype == NNCP_BF16;
  PackArgs pa{a.krp.f[0], a.I1, a.I1pad, a.R, a.col0, RP, a.hpack, a.hscale};
  const int wm = L.mtile / pm_16_wave_rows(L.side, L.nb, L.j1);
  const bool v = vec16(a, L.side);
  const int variant = (L.j1 ? 100000 : 0) + (bf ? 10000 : 0) + L.side * 1000 + L.nb * 100 + wm * 10 + (v ? 1 : 0);
  const void* k = bf ? select16<NNCP_BF16>(L.side, L.nb, wm, v, L.j1 != 0)
                     : select16<NNCP_F16>(L.side, L.nb, wm, v, L.j1 != 0);
  if (!k) return hipErrorInvalidValue;
  size_t lds = L.lds_bytes;
  if (reduce_lds16(L.side, L.nb, wm) > lds) lds = reduce_lds16(L.side, L.nb, wm);
  if (sk.rec) {
    KOp op{};
    op.kind = K_PACK16;
    op.variant = bf ? 1 : 0;
    op.gx = (unsigned)RP;
    op.gy = 1;
    op.u.pk = pa;
    hipError_t e = sink_record(sk, op);
    if (e != hipSuccess) return e;
    KOp pm{};
    pm.kind = K_PM_16;
    pm.variant = variant;
    pm.gx = (unsigned)L.mtiles;
    pm.gy = (unsigned)L.nsplit;
    pm.lds = (unsigned)lds;
    pm.u.pm = a;
    return sink_record(sk, pm);
  }
  if (bf) hipLaunchKernelGGL(pm16_pack_kernel<NNCP_BF16>, dim3(RP), dim3(256), 0, sk.st, pa);
  else hipLaunchKernelGGL(pm16_pack_kernel<NNCP_F16>, dim3(RP), dim3(256), 0, sk.st, pa);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  static bool attr_done[2][2][2][3][2][2] = {};
  bool& done = attr_done[L.j1 != 0][bf][L.side][L.nb == 1 ? 0 : (L.nb == 2 ? 1 : 2)][wm == 4][v];
  if (!done) {
    if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) != hipSuccess)
      (void)hipGetLastError();
    done = true;
  }
  void* args[] = {(void*)&a};
  return hipLaunchKernel(k, dim3(L.mtiles, L.nsplit), dim3(NT), args, lds, sk.st);
}

hipError_t batch_launch_pm_16j1(const BItem* items, const int* count, const KOp* ops, unsigned grid, size_t lds,
                                hipStream_t st) {
  static bool attr = [] {
    (void)hipFuncSetAttribute((const void*)pm16j1_batch_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    (void)hipGetLastError();
    return true;
  }();
  (void)attr;
  hipLaunchKernelGGL(pm16j1_batch_kernel, dim3(grid), dim3(NT), lds, st, items, count, ops);
  return hipGetLastError();
}

hipError_t batch_launch_pm_16(const BItem* items, const int* count, const KOp* ops, unsigned grid, size_t lds,
                              hipStream_t st) {
  static bool attr = [] {
    (void)hipFuncSetAttribute((const void*)pm16_batch_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    (void)hipGetLastError();
    return true;
  }();
  (void)attr;
  hipLaunchKernelGGL(pm16_batch_kernel, dim3(grid), dim3(NT), lds, st, items, count, ops);
  return hipGetLastError();
}

}  // namespace nncpk
