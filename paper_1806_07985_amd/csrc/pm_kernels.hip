// Partial MTTKRP on MFMA (the root edges of the dimension tree, Section IV-A,
// Figure 2a): T = X_[L] * K (left node) or T = X_[L]^T * K (right node), where
// X_[L] is the tensor viewed as the column-major I_L x I_R matrix (modes 1..s
// on the rows) and K is the Khatri-Rao product of the other side's factors.
//
// Design (gfx950, wave64):
//  * The reduction index k runs over X's columns (left) or rows (right). The
//    Khatri-Rao operand is never materialised in HBM: each work-group forms a
//    BK x R tile of it in LDS from factor rows (double-buffered), and every wave
//    of the group reads its MFMA B operand from that tile.
//  * X is streamed straight from HBM into VGPRs with 16-byte loads, one k-step
//    ahead of the MFMAs. FP32 uses v_mfma_f32_16x16x4_f32. The K order inside a
//    16- or 32-wide super-step is permuted so that one 16-byte load per lane
//    feeds four MFMAs while A and B agree on which k sits in which slot.
//  * Split-K over work-groups with FP32 partials; the last work-group to finish
//    an output tile (device-scope counter) sums the partials in FP64 in split
//    order, so results do not depend on scheduling.
#include "nncp_internal.hpp"

namespace nncpk {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));

constexpr int BK = 128;          // Khatri-Rao tile depth (k rows per LDS tile)
constexpr int PITCH = BK + 4;    // floats per tile column in LDS
constexpr int NT = 256;          // threads per work-group (4 waves)

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Build rows [k0, k0+BK) of the Khatri-Rao operand into LDS tile `kt`
// (layout kt[col * PITCH + k]). Rows at or beyond kend are zero.
template <int NB>
__device__ __forceinline__ void build_tile(float* kt, const KrpDesc& krp, const double* cs,
                                           int64_t k0, int64_t kend, int R, int col0) {
  constexpr int RP = NB * 16;
  const int kl = threadIdx.x % BK;
  const int c0 = threadIdx.x / BK;  // 0 or 1
  const int64_t k = k0 + kl;
  int d[kMaxModes];
  bool valid = k < kend;
  if (valid) {
    uint32_t rem = (uint32_t)k;  // operand rows are < 2^32
#pragma unroll
    for (int j = 0; j < kMaxModes; ++j) {
      if (j < krp.nm) {
        uint32_t dj = (uint32_t)krp.dim[j];
        d[j] = (int)(rem % dj);
        rem /= dj;
      }
    }
  }
  for (int c = c0; c < RP; c += NT / BK) {
    float v = 0.f;
    if (valid && c < R) {
      double p = cs[c];
#pragma unroll
      for (int j = 0; j < kMaxModes; ++j)
        if (j < krp.nm) p *= (double)krp.f[j][(int64_t)d[j] + (int64_t)krp.dim[j] * (col0 + c)];
      v = (float)p;
    }
    kt[c * PITCH + kl] = v;
  }
}

// Deterministic split-K epilogue: write this group's partial, count, and let the
// last group of the M tile reduce all splits in FP64 into T.
__device__ void splitk_finish(const PmArgs& a, int64_t Mtot, int mtile, int64_t mbeg, int RP,
                              int64_t Mpad) {
  __shared__ int s_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned prev = __hip_atomic_fetch_add(&a.counters[blockIdx.x], 1u, __ATOMIC_ACQ_REL,
                                           __HIP_MEMORY_SCOPE_AGENT);
    s_last = (prev == (unsigned)(a.nsplit - 1));
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  const int64_t rows = (Mtot - mbeg) < mtile ? (Mtot - mbeg) : mtile;
  const int64_t total = rows * a.R;
  const size_t sstride = (size_t)RP * (size_t)Mpad;
  for (int64_t e = threadIdx.x; e < total; e += NT) {
    int r = (int)(e / rows);
    int64_t m = mbeg + (e - (int64_t)r * rows);
    const float* p = a.partial + (size_t)r * Mpad + m;
    double s = 0.0;
    for (int sp = 0; sp < a.nsplit; ++sp) s += (double)__builtin_nontemporal_load(p + sp * sstride);
    a.T[m + Mtot * (int64_t)(a.col0 + r)] = (float)s;
  }
  if (threadIdx.x == 0)
    __hip_atomic_store(&a.counters[blockIdx.x], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum the accumulators of the WK waves that share an M range (WK > 1) through LDS;
// wave wk == 0 ends with the total. `acc` is NACC f4 per lane.
template <int NACC>
__device__ __forceinline__ void wave_reduce_k(f4* acc, float* lds, int wk, int wm, int WK, int WM) {
  if (WK == 1) return;
  const int lane = threadIdx.x & 63;
  for (int src = 1; src < WK; ++src) {
    __syncthreads();
    if (wk == src) {
#pragma unroll
      for (int v = 0; v < NACC; ++v) *(f4*)&lds[((wm * NACC + v) * 64 + lane) * 4] = acc[v];
    }
    __syncthreads();
    if (wk == 0) {
#pragma unroll
      for (int v = 0; v < NACC; ++v) acc[v] += *(f4*)&lds[((wm * NACC + v) * 64 + lane) * 4];
    }
  }
}

// ----------------------------------------------------------------------------
// Left side, FP32: T(m, r) = sum_k X[m + IL*k] * K(k, r); m is contiguous in X.
// Wave tile: MR groups of 64 rows x all RP columns. Lane (i, q) loads rows
// 4i..4i+3 of a group for column k = base + 4q + u; MFMA t uses row 4i+t.
// ----------------------------------------------------------------------------
template <int NB, int MR, int WM, bool VEC>
__global__ __launch_bounds__(NT, 2) void pm_left_f32(PmArgs a) {
  constexpr int RP = NB * 16;
  constexpr int WK = 4 / WM;
  constexpr int KS = 16;                  // k per super-step
  constexpr int SPT = BK / WK / KS;       // super-steps per tile per wave
  constexpr int NACC = MR * 4 * NB;
  static_assert(SPT >= 1, "tile too shallow");
  extern __shared__ float lds[];
  float* kt0 = lds;
  float* kt1 = lds + RP * PITCH;
  double* cs = (double*)(lds + 2 * RP * PITCH);

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % WM, wk = wave / WM;
  const int li = lane & 15, lq = lane >> 4;
  const int64_t Mtot = a.IL, Ktot = a.IR;
  const int mtile = WM * 64 * MR;
  const int64_t mbeg = (int64_t)blockIdx.x * mtile;
  const int64_t mw = mbeg + wm * 64 * MR;
  const int64_t kbeg = (int64_t)blockIdx.y * a.kchunk;
  int64_t kend = kbeg + a.kchunk;
  if (kend > Ktot) kend = Ktot;
  const int ntiles = (int)((kend - kbeg + BK - 1) / BK);
  const float* X = (const float*)a.X;

  for (int c = threadIdx.x; c < RP; c += NT) cs[c] = (c < a.R) ? krp_colscale(a.krp, a.col0 + c) : 0.0;
  __syncthreads();

  f4 acc[NACC];
#pragma unroll
  for (int v = 0; v < NACC; ++v) acc[v] = f4{0.f, 0.f, 0.f, 0.f};

  auto load_step = [&](int s, f4 (&A)[MR][4]) {
    const int t = s / SPT, w = s % SPT;
    const int64_t kb = kbeg + (int64_t)t * BK + wk * (BK / WK) + w * KS + 4 * lq;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t k = kb + u;
      const bool kv = k < kend;
      const float* col = X + Ktot * 0 + Mtot * (kv ? k : 0);
#pragma unroll
      for (int g = 0; g < MR; ++g) {
        const int64_t m = mw + 64 * g + 4 * li;
        if (VEC) {
          if (kv && m < Mtot) A[g][u] = __builtin_nontemporal_load((const f4*)(col + m));
          else A[g][u] = f4{0.f, 0.f, 0.f, 0.f};
        } else {
          f4 v;
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] = (kv && m + e < Mtot) ? col[m + e] : 0.f;
          A[g][u] = v;
        }
      }
    }
  };

  build_tile<NB>(kt0, a.krp, cs, kbeg, kend, a.R, a.col0);
  __syncthreads();

  const int nsteps = ntiles * SPT;
  f4 Acur[MR][4], Anxt[MR][4];
  if (nsteps > 0) load_step(0, Acur);
  for (int t = 0; t < ntiles; ++t) {
    const float* kt = (t & 1) ? kt1 : kt0;
#pragma unroll
    for (int w = 0; w < SPT; ++w) {
      const int s = t * SPT + w;
      if (s + 1 < nsteps) load_step(s + 1, Anxt);
      const int kk = wk * (BK / WK) + w * KS + 4 * lq;
      f4 B[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) B[nb] = *(const f4*)&kt[(16 * nb + li) * PITCH + kk];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int g = 0; g < MR; ++g)
#pragma unroll
          for (int tt = 0; tt < 4; ++tt)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
              acc[(g * 4 + tt) * NB + nb] = mfma4(Acur[g][u][tt], B[nb][u], acc[(g * 4 + tt) * NB + nb]);
      if (s + 1 < nsteps) {
#pragma unroll
        for (int g = 0; g < MR; ++g)
#pragma unroll
          for (int u = 0; u < 4; ++u) Acur[g][u] = Anxt[g][u];
      }
    }
    if (t + 1 < ntiles)
      build_tile<NB>((t & 1) ? kt0 : kt1, a.krp, cs, kbeg + (int64_t)(t + 1) * BK, kend, a.R, a.col0);
    __syncthreads();
  }

  wave_reduce_k<NACC>(acc, lds, wk, wm, WK, WM);
  if (wk != 0 && a.nsplit == 1) return;

  // Output element of acc[(g*4+t)*NB+nb][v]: row mw + 64g + 16*lq + 4v + t, column 16nb + li.
  const bool direct = (a.nsplit == 1);
  const int64_t Mpad = (int64_t)gridDim.x * mtile;
  if (wk == 0) {
#pragma unroll
    for (int g = 0; g < MR; ++g)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int r = 16 * nb + li;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t m = mw + 64 * g + 16 * lq + 4 * v;
          f4 o = f4{acc[(g * 4 + 0) * NB + nb][v], acc[(g * 4 + 1) * NB + nb][v],
                    acc[(g * 4 + 2) * NB + nb][v], acc[(g * 4 + 3) * NB + nb][v]};
          if (direct) {
            if (r < a.R) {
              float* dst = a.T + Mtot * (int64_t)(a.col0 + r);
#pragma unroll
              for (int e = 0; e < 4; ++e)
                if (m + e < Mtot) dst[m + e] = o[e];
            }
          } else {
            *(f4*)&a.partial[((size_t)blockIdx.y * RP + r) * Mpad + m] = o;
          }
        }
      }
  }
  if (!direct) splitk_finish(a, Mtot, mtile, mbeg, RP, Mpad);
}

// ----------------------------------------------------------------------------
// Right side, FP32: T(c, r) = sum_k X[k + IL*c] * K(k, r); k is contiguous in X.
// Wave tile: MC groups of 16 columns c. Lane (i, q) loads k = base + 16h + 4q + u
// (u = 0..3 in one 16-byte load, h = 0..1) of column c = group + i.
// ----------------------------------------------------------------------------
template <int NB, int MC, int WM, bool VEC>
__global__ __launch_bounds__(NT, 2) void pm_right_f32(PmArgs a) {
  constexpr int RP = NB * 16;
  constexpr int WK = 4 / WM;
  constexpr int KS = 32;
  constexpr int SPT = BK / WK / KS;
  constexpr int NACC = MC * NB;
  static_assert(SPT >= 1, "tile too shallow");
  extern __shared__ float lds[];
  float* kt0 = lds;
  float* kt1 = lds + RP * PITCH;
  double* cs = (double*)(lds + 2 * RP * PITCH);

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % WM, wk = wave / WM;
  const int li = lane & 15, lq = lane >> 4;
  const int64_t Mtot = a.IR, Ktot = a.IL;
  const int mtile = WM * 16 * MC;
  const int64_t mbeg = (int64_t)blockIdx.x * mtile;
  const int64_t cw = mbeg + wm * 16 * MC;
  const int64_t kbeg = (int64_t)blockIdx.y * a.kchunk;
  int64_t kend = kbeg + a.kchunk;
  if (kend > Ktot) kend = Ktot;
  const int ntiles = (int)((kend - kbeg + BK - 1) / BK);
  const float* X = (const float*)a.X;

  for (int c = threadIdx.x; c < RP; c += NT) cs[c] = (c < a.R) ? krp_colscale(a.krp, a.col0 + c) : 0.0;
  __syncthreads();

  f4 acc[NACC];
#pragma unroll
  for (int v = 0; v < NACC; ++v) acc[v] = f4{0.f, 0.f, 0.f, 0.f};

  auto load_step = [&](int s, f4 (&A)[MC][2]) {
    const int t = s / SPT, w = s % SPT;
    const int64_t kb = kbeg + (int64_t)t * BK + wk * (BK / WK) + w * KS + 4 * lq;
#pragma unroll
    for (int g = 0; g < MC; ++g) {
      const int64_t c = cw + 16 * g + li;
      const bool cv = c < Mtot;
      const float* col = X + Ktot * (cv ? c : 0);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int64_t k = kb + 16 * h;
        if (VEC) {
          if (cv && k < kend) A[g][h] = __builtin_nontemporal_load((const f4*)(col + k));
          else A[g][h] = f4{0.f, 0.f, 0.f, 0.f};
        } else {
          f4 v;
#pragma unroll
          for (int e = 0; e < 4; ++e) v[e] = (cv && k + e < kend) ? col[k + e] : 0.f;
          A[g][h] = v;
        }
      }
    }
  };

  build_tile<NB>(kt0, a.krp, cs, kbeg, kend, a.R, a.col0);
  __syncthreads();

  const int nsteps = ntiles * SPT;
  f4 Acur[MC][2], Anxt[MC][2];
  if (nsteps > 0) load_step(0, Acur);
  for (int t = 0; t < ntiles; ++t) {
    const float* kt = (t & 1) ? kt1 : kt0;
#pragma unroll
    for (int w = 0; w < SPT; ++w) {
      const int s = t * SPT + w;
      if (s + 1 < nsteps) load_step(s + 1, Anxt);
      const int kk = wk * (BK / WK) + w * KS + 4 * lq;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        f4 B[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) B[nb] = *(const f4*)&kt[(16 * nb + li) * PITCH + kk + 16 * h];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int g = 0; g < MC; ++g)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
              acc[g * NB + nb] = mfma4(Acur[g][h][u], B[nb][u], acc[g * NB + nb]);
      }
      if (s + 1 < nsteps) {
#pragma unroll
        for (int g = 0; g < MC; ++g)
#pragma unroll
          for (int h = 0; h < 2; ++h) Acur[g][h] = Anxt[g][h];
      }
    }
    if (t + 1 < ntiles)
      build_tile<NB>((t & 1) ? kt0 : kt1, a.krp, cs, kbeg + (int64_t)(t + 1) * BK, kend, a.R, a.col0);
    __syncthreads();
  }

  wave_reduce_k<NACC>(acc, lds, wk, wm, WK, WM);
  if (wk != 0 && a.nsplit == 1) return;

  // acc[g*NB+nb][v]: column c = cw + 16g + 4*lq + v, rank column 16nb + li.
  const bool direct = (a.nsplit == 1);
  const int64_t Mpad = (int64_t)gridDim.x * mtile;
  if (wk == 0) {
#pragma unroll
    for (int g = 0; g < MC; ++g)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        const int r = 16 * nb + li;
        const int64_t c = cw + 16 * g + 4 * lq;
        f4 o = acc[g * NB + nb];
        if (direct) {
          if (r < a.R) {
            float* dst = a.T + Mtot * (int64_t)(a.col0 + r);
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (c + e < Mtot) dst[c + e] = o[e];
          }
        } else {
          *(f4*)&a.partial[((size_t)blockIdx.y * RP + r) * Mpad + c] = o;
        }
      }
  }
  if (!direct) splitk_finish(a, Mtot, mtile, mbeg, RP, Mpad);
}

// Row groups (64 rows each) per wave on the left side: the accumulators of four
// column blocks leave no room for a second group without spilling.
constexpr int left_mr(int nb) { return nb >= 4 ? 1 : 2; }

template <int NB>
size_t pm_lds_bytes() {
  return (size_t)2 * NB * 16 * PITCH * sizeof(float) + NB * 16 * sizeof(double);
}

template <int NB, int WM>
hipError_t launch_f32(const PmLaunch& L, const PmArgs& a, bool vec, hipStream_t st) {
  dim3 grid(L.mtiles, L.nsplit), block(NT);
  size_t lds = pm_lds_bytes<NB>();
  // The cross-wave reduction reuses the tile buffers; they hold WM * NACC * 64 f4.
  if (L.side == 0) {
    constexpr int MR = left_mr(NB);
    constexpr int NACC = MR * 4 * NB;
    size_t need = (size_t)WM * NACC * 64 * 16;
    if (WM < 4 && need > lds) lds = need;
    if (vec) hipLaunchKernelGGL((pm_left_f32<NB, MR, WM, true>), grid, block, lds, st, a);
    else hipLaunchKernelGGL((pm_left_f32<NB, MR, WM, false>), grid, block, lds, st, a);
  } else {
    constexpr int NACC = 4 * NB;
    size_t need = (size_t)WM * NACC * 64 * 16;
    if (WM < 4 && need > lds) lds = need;
    if (vec) hipLaunchKernelGGL((pm_right_f32<NB, 4, WM, true>), grid, block, lds, st, a);
    else hipLaunchKernelGGL((pm_right_f32<NB, 4, WM, false>), grid, block, lds, st, a);
  }
  return hipGetLastError();
}

}  // namespace

// Tile/split heuristic: aim for >= ~4 work-groups per CU across the chip, keep each
// split at least two tiles deep, and prefer the narrower M tile (one wave along
// M, four along K) when the output has few rows.
PmLaunch pm_plan(int side, int dtype, int64_t IL, int64_t IR, int R) {
  PmLaunch L{};
  L.side = side;
  L.dtype = dtype;
  const int Rc = R < kPmMaxCols ? R : kPmMaxCols;
  L.nb = Rc <= 16 ? 1 : (Rc <= 32 ? 2 : 4);
  const int64_t Mtot = side == 0 ? IL : IR;
  const int64_t Ktot = side == 0 ? IR : IL;
  const int wave_rows = side == 0 ? 64 * left_mr(L.nb) : 64;
  const int64_t target = 1024;
  int wm = 4;
  if ((Mtot + 4 * wave_rows - 1) / (4 * wave_rows) < 64) wm = 1;
  L.mtile = wm * wave_rows;
  L.mtiles = (int)((Mtot + L.mtile - 1) / L.mtile);
  const int64_t ktiles = (Ktot + BK - 1) / BK;
  int64_t ns = (target + L.mtiles - 1) / L.mtiles;
  int64_t maxs = ktiles / 2 > 0 ? ktiles / 2 : 1;
  if (ns > maxs) ns = maxs;
  if (ns > 256) ns = 256;
  if (ns < 1) ns = 1;
  int64_t tiles_per = (ktiles + ns - 1) / ns;
  L.kchunk = tiles_per * BK;
  L.nsplit = (int)((Ktot + L.kchunk - 1) / L.kchunk);
  if (L.nsplit < 1) L.nsplit = 1;
  L.partial_floats = L.nsplit > 1 ? (size_t)L.nsplit * L.nb * 16 * (size_t)L.mtiles * L.mtile : 0;
  L.ncounters = L.mtiles;
  return L;
}

hipError_t pm_launch(const PmLaunch& L, const PmArgs& a, hipStream_t st) {
  const int64_t Mtot = L.side == 0 ? a.IL : a.IR;
  const int64_t Ktot = L.side == 0 ? a.IR : a.IL;
  (void)Ktot;
  bool vec = ((uintptr_t)a.X % 16 == 0) && ((L.side == 0 ? a.IL : a.IL) % 4 == 0);
  (void)Mtot;
  if (L.dtype != NNCP_F32) return hipErrorInvalidValue;
  const int wm = L.mtile / (L.side == 0 ? 64 * left_mr(L.nb) : 64);
  switch (L.nb * 10 + (wm == 4 ? 4 : 1)) {
    case 14: return launch_f32<1, 4>(L, a, vec, st);
    case 11: return launch_f32<1, 1>(L, a, vec, st);
    case 24: return launch_f32<2, 4>(L, a, vec, st);
    case 21: return launch_f32<2, 1>(L, a, vec, st);
    case 44: return launch_f32<4, 4>(L, a, vec, st);
    case 41: return launch_f32<4, 1>(L, a, vec, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace nncpk
