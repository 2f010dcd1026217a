// Partial MTTKRP on MFMA for FP32 tensors (the root edges of the dimension
// tree, Section IV-A, Figure 2a): T = X_[L] * K (left node) or
// T = X_[L]^T * K (right node), where X_[L] is the tensor viewed as the
// column-major I_L x I_R matrix (modes 1..s on the rows) and K is the
// Khatri-Rao product of the other side's factors.
//
// Design (gfx950, wave64):
//  * The reduction index k runs over X's columns (left) or rows (right). The
//    Khatri-Rao operand is never materialised in HBM: each work-group forms a
//    BK x R tile of it in LDS from factor rows (double-buffered), and every wave
//    of the group reads its MFMA B operand from that tile.
//  * X is streamed straight from HBM into VGPRs with 8- or 16-byte loads, one
//    k-step ahead of the MFMAs (v_mfma_f32_16x16x4_f32). The k order inside a
//    16- or 32-wide k-step is permuted so that one wide load per lane feeds
//    several MFMAs while A and B agree on which k sits in which slot.
//  * Precision: each MFMA chain covers one k-step only (4 or 8 MFMAs, 16 or 32
//    products per output) and is then added into FP64 accumulators, so the FP32
//    rounding of a running sum never spans more than 32 terms; split-K
//    partials, the cross-wave reduction and the output are FP64.
//  * Split-K over work-groups; the last work-group to finish an output tile
//    (device-scope counter) sums the partials in split order, so results do
//    not depend on scheduling.
#include "pm_common.hpp"

namespace nncpk {
namespace {

// ----------------------------------------------------------------------------
// Left side: T(m, r) = sum_k X[m + IL*k] * K(k, r); m is contiguous in X.
// A wave covers 16*TR rows. Lane (i, q) loads rows TR*i .. TR*i+TR-1 of column
// k = base + 4q + u (u = 0..3); MFMA t uses row TR*i + t of that load.
// ----------------------------------------------------------------------------
template <int NB, int TR, int WM, bool VEC>
__global__ __launch_bounds__(NT, 2) void pm_left_f32(PmArgs a) {
  constexpr int RP = NB * 16;
  constexpr int WK = 4 / WM;
  constexpr int KS = 16;                  // k per k-step
  constexpr int SPT = BK / WK / KS;       // k-steps per tile per wave
  constexpr int NACC = TR * NB;           // 4-element accumulators per lane
  constexpr int WROWS = 16 * TR;
  static_assert(SPT >= 1, "tile too shallow");
  typedef float vT __attribute__((ext_vector_type(TR)));
  extern __shared__ float lds[];
  float* kt0 = lds;
  float* kt1 = lds + RP * PITCH;
  double* cs = (double*)(lds + 2 * RP * PITCH);

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % WM, wk = wave / WM;
  const int li = lane & 15, lq = lane >> 4;
  const int64_t Mtot = a.IL, Ktot = a.IR;
  const int mtile = WM * WROWS;
  const int64_t mbeg = (int64_t)blockIdx.x * mtile;
  const int64_t mw = mbeg + wm * WROWS;
  const int64_t kbeg = (int64_t)blockIdx.y * a.kchunk;
  int64_t kend = kbeg + a.kchunk;
  if (kend > Ktot) kend = Ktot;
  const int ntiles = (int)((kend - kbeg + BK - 1) / BK);
  const float* X = (const float*)a.X;

  for (int c = threadIdx.x; c < RP; c += NT) cs[c] = (c < a.R) ? krp_colscale(a.krp, a.col0 + c) : 0.0;
  __syncthreads();

  double acc[NACC][4];
#pragma unroll
  for (int v = 0; v < NACC; ++v)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[v][e] = 0.0;

  const int64_t m = mw + TR * li;
  const bool mfull = m + TR <= Mtot;
  auto load_step = [&](int s, vT (&A)[4]) {
    const int t = s / SPT, w = s % SPT;
    const int64_t kb = kbeg + (int64_t)t * BK + wk * (BK / WK) + w * KS + 4 * lq;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t k = kb + u;
      const bool kv = k < kend;
      const float* col = X + Mtot * (kv ? k : 0);
      if (VEC) {
        if (kv && mfull) A[u] = __builtin_nontemporal_load((const vT*)(col + m));
        else A[u] = vT{};
      } else {
        vT v;
#pragma unroll
        for (int e = 0; e < TR; ++e) v[e] = (kv && m + e < Mtot) ? col[m + e] : 0.f;
        A[u] = v;
      }
    }
  };

  build_tile<NB>(kt0, a.krp, cs, kbeg, kend, a.R, a.col0);
  __syncthreads();

  const int nsteps = ntiles * SPT;
  vT Acur[4], Anxt[4];
  if (nsteps > 0) load_step(0, Acur);
  for (int t = 0; t < ntiles; ++t) {
    const float* kt = (t & 1) ? kt1 : kt0;
#pragma unroll 1
    for (int w = 0; w < SPT; ++w) {
      const int s = t * SPT + w;
      if (s + 1 < nsteps) load_step(s + 1, Anxt);
      const int kk = wk * (BK / WK) + w * KS + 4 * lq;
      f4 B[NB];
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) B[nb] = *(const f4*)&kt[(16 * nb + li) * PITCH + kk];
#pragma unroll
      for (int tt = 0; tt < TR; ++tt)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          f4 c = mfma4(Acur[0][tt], B[nb][0], f4{0.f, 0.f, 0.f, 0.f});
          c = mfma4(Acur[1][tt], B[nb][1], c);
          c = mfma4(Acur[2][tt], B[nb][2], c);
          c = mfma4(Acur[3][tt], B[nb][3], c);
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[tt * NB + nb][e] += (double)c[e];
        }
      if (s + 1 < nsteps) {
#pragma unroll
        for (int u = 0; u < 4; ++u) Acur[u] = Anxt[u];
      }
    }
    if (t + 1 < ntiles)
      build_tile<NB>((t & 1) ? kt0 : kt1, a.krp, cs, kbeg + (int64_t)(t + 1) * BK, kend, a.R, a.col0);
    __syncthreads();
  }

  wave_reduce_k<NACC>(acc, (double*)lds, wk, wm, WK);
  if (wk != 0 && a.nsplit == 1) return;

  // acc[tt*NB+nb][v]: row mw + TR*(4*lq + v) + tt, rank column 16nb + li.
  const bool direct = (a.nsplit == 1);
  const int64_t Mpad = (int64_t)gridDim.x * mtile;
  if (wk == 0) {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int tt = 0; tt < TR; ++tt)
          pm_store(a, direct, Mtot, Mpad, RP, 16 * nb + li, mw + TR * (4 * lq + v) + tt, acc[tt * NB + nb][v]);
  }
  if (!direct) splitk_finish(a, Mtot, mtile, mbeg, RP, Mpad);
}

// ----------------------------------------------------------------------------
// Right side: T(c, r) = sum_k X[k + IL*c] * K(k, r); k is contiguous in X.
// A wave covers MC groups of 16 columns c. Lane (i, q) loads k = base + 16h +
// 4q + u (u = 0..3 in one 16-byte load, h = 0..1) of column c = group + i.
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

  double acc[NACC][4];
#pragma unroll
  for (int v = 0; v < NACC; ++v)
#pragma unroll
    for (int e = 0; e < 4; ++e) acc[v][e] = 0.0;

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
#pragma unroll 1
    for (int w = 0; w < SPT; ++w) {
      const int s = t * SPT + w;
      if (s + 1 < nsteps) load_step(s + 1, Anxt);
      const int kk = wk * (BK / WK) + w * KS + 4 * lq;
      f4 B[2][NB];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) B[h][nb] = *(const f4*)&kt[(16 * nb + li) * PITCH + kk + 16 * h];
#pragma unroll
      for (int g = 0; g < MC; ++g)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
          f4 c = mfma4(Acur[g][0][0], B[0][nb][0], f4{0.f, 0.f, 0.f, 0.f});
          c = mfma4(Acur[g][0][1], B[0][nb][1], c);
          c = mfma4(Acur[g][0][2], B[0][nb][2], c);
          c = mfma4(Acur[g][0][3], B[0][nb][3], c);
          c = mfma4(Acur[g][1][0], B[1][nb][0], c);
          c = mfma4(Acur[g][1][1], B[1][nb][1], c);
          c = mfma4(Acur[g][1][2], B[1][nb][2], c);
          c = mfma4(Acur[g][1][3], B[1][nb][3], c);
#pragma unroll
          for (int e = 0; e < 4; ++e) acc[g * NB + nb][e] += (double)c[e];
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

  wave_reduce_k<NACC>(acc, (double*)lds, wk, wm, WK);
  if (wk != 0 && a.nsplit == 1) return;

  // acc[g*NB+nb][v]: column c = cw + 16g + 4*lq + v, rank column 16nb + li.
  const bool direct = (a.nsplit == 1);
  const int64_t Mpad = (int64_t)gridDim.x * mtile;
  if (wk == 0) {
#pragma unroll
    for (int g = 0; g < MC; ++g)
#pragma unroll
      for (int nb = 0; nb < NB; ++nb)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          pm_store(a, direct, Mtot, Mpad, RP, 16 * nb + li, cw + 16 * g + 4 * lq + v, acc[g * NB + nb][v]);
  }
  if (!direct) splitk_finish(a, Mtot, mtile, mbeg, RP, Mpad);
}

// Rows per left wave = 16 * left_tr(NB); columns per right wave = 16 * right_mc(NB).
// Chosen so that the FP64 accumulators (2 VGPRs per output) leave room for a
// double-buffered k-step of X without spilling.
constexpr int left_tr(int nb) { return nb >= 4 ? 2 : 4; }
constexpr int right_mc(int nb) { return nb >= 4 ? 2 : 4; }

template <int NB, int WM>
hipError_t launch_f32(const PmLaunch& L, const PmArgs& a, bool vec, hipStream_t st) {
  dim3 grid(L.mtiles, L.nsplit), block(NT);
  size_t lds = pm_lds_bytes(NB);
  if (L.side == 0) {
    constexpr int TR = left_tr(NB);
    const size_t need = (size_t)WM * TR * NB * 4 * 64 * sizeof(double);
    if (WM < 4 && need > lds) lds = need;
    if (vec) hipLaunchKernelGGL((pm_left_f32<NB, TR, WM, true>), grid, block, lds, st, a);
    else hipLaunchKernelGGL((pm_left_f32<NB, TR, WM, false>), grid, block, lds, st, a);
  } else {
    constexpr int MC = right_mc(NB);
    const size_t need = (size_t)WM * MC * NB * 4 * 64 * sizeof(double);
    if (WM < 4 && need > lds) lds = need;
    if (vec) hipLaunchKernelGGL((pm_right_f32<NB, MC, WM, true>), grid, block, lds, st, a);
    else hipLaunchKernelGGL((pm_right_f32<NB, MC, WM, false>), grid, block, lds, st, a);
  }
  return hipGetLastError();
}

}  // namespace

int pm_f32_wave_rows(int side, int nb) { return side == 0 ? 16 * left_tr(nb) : 16 * right_mc(nb); }

hipError_t pm_launch_f32(const PmLaunch& L, const PmArgs& a, hipStream_t st) {
  // vector loads need a 16-byte aligned base and I_L % 4 == 0 (every column aligned)
  const bool vec = ((uintptr_t)a.X % 16 == 0) && (a.IL % 4 == 0);
  const int wm = L.mtile / pm_f32_wave_rows(L.side, L.nb);
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
