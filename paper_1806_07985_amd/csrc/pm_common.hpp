// Device helpers shared by the partial-MTTKRP kernels (FP32 and 16-bit tensors).
#pragma once

#include "nncp_internal.hpp"

namespace nncpk {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int BK = 128;          // Khatri-Rao tile depth (operand rows per LDS tile)
constexpr int PITCH = BK + 4;    // floats per tile column in LDS (FP32 tiles)
constexpr int NT = 256;          // threads per work-group (4 waves)

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Operand-row digits: row k of a Khatri-Rao operand over nm modes (first mode
// fastest) picks row d_j of factor j.
__device__ __forceinline__ void krp_digits(const KrpDesc& krp, uint32_t k, int* d) {
#pragma unroll
  for (int j = 0; j < kMaxModes; ++j) {
    if (j < krp.nm) {
      const uint32_t dj = (uint32_t)krp.dim[j];
      const uint32_t q = k / dj;
      d[j] = (int)(k - q * dj);
      k = q;
    }
  }
}

// Value of the (scaled) operand at digits d, column col (computed in FP64).
__device__ __forceinline__ double krp_value(const KrpDesc& krp, const int* d, int col, double scale) {
  double p = scale;
#pragma unroll
  for (int j = 0; j < kMaxModes; ++j)
    if (j < krp.nm) p *= (double)krp.f[j][(int64_t)d[j] + (int64_t)krp.dim[j] * col];
  return p;
}

// Build rows [k0, k0+BK) of the Khatri-Rao operand into the FP32 LDS tile `kt`
// (layout kt[col * PITCH + k]). Rows at or beyond kend and columns >= R are zero.
template <int NB>
__device__ __forceinline__ void build_tile(float* kt, const KrpDesc& krp, const double* cs,
                                           int64_t k0, int64_t kend, int R, int col0) {
  constexpr int RP = NB * 16;
  const int kl = threadIdx.x % BK;
  const int c0 = threadIdx.x / BK;
  const int64_t k = k0 + kl;
  int d[kMaxModes];
  const bool valid = k < kend;
  if (valid) krp_digits(krp, (uint32_t)k, d);
  for (int c = c0; c < RP; c += NT / BK) {
    float v = 0.f;
    if (valid && c < R) v = (float)krp_value(krp, d, col0 + c, cs[c]);
    kt[c * PITCH + kl] = v;
  }
}

// Deterministic split-K epilogue: the group has written its FP64 partial; the
// last group of the M tile to arrive sums all splits in split order into T.
template <typename TO>
__device__ void splitk_finish_t(const PmArgs& a, int64_t Mtot, int mtile, int64_t mbeg, int RP,
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
  TO* T = (TO*)a.T;
  for (int64_t e = threadIdx.x; e < total; e += NT) {
    const int r = (int)(e / rows);
    const int64_t m = mbeg + (e - (int64_t)r * rows);
    const double* p = a.partial + (size_t)r * Mpad + m;
    double s = 0.0;
    for (int sp = 0; sp < a.nsplit; ++sp) s += __builtin_nontemporal_load(p + sp * sstride);
    T[m + Mtot * (int64_t)(a.col0 + r)] = (TO)s;
  }
  if (threadIdx.x == 0)
    __hip_atomic_store(&a.counters[blockIdx.x], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void splitk_finish(const PmArgs& a, int64_t Mtot, int mtile, int64_t mbeg, int RP,
                                              int64_t Mpad) {
  if (a.t_f64) splitk_finish_t<double>(a, Mtot, mtile, mbeg, RP, Mpad);
  else splitk_finish_t<float>(a, Mtot, mtile, mbeg, RP, Mpad);
}

// Sum the FP64 accumulators of the WK waves that share an M range through LDS;
// wave wk == 0 ends with the total.
template <int NACC>
__device__ __forceinline__ void wave_reduce_k(double (&acc)[NACC][4], double* lds, int wk, int wm, int WK) {
  if (WK == 1) return;
  const int lane = threadIdx.x & 63;
  for (int src = 1; src < WK; ++src) {
    __syncthreads();
    if (wk == src) {
#pragma unroll
      for (int v = 0; v < NACC; ++v)
#pragma unroll
        for (int e = 0; e < 4; ++e) lds[((wm * NACC + v) * 4 + e) * 64 + lane] = acc[v][e];
    }
    __syncthreads();
    if (wk == 0) {
#pragma unroll
      for (int v = 0; v < NACC; ++v)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[v][e] += lds[((wm * NACC + v) * 4 + e) * 64 + lane];
    }
  }
}

// Store one output element: directly into T (FP64 or FP32) or into the split partials.
__device__ __forceinline__ void pm_store(const PmArgs& a, bool direct, int64_t Mtot, int64_t Mpad, int RP,
                                         int r, int64_t mm, double o) {
  if (direct) {
    if (r < a.R && mm < Mtot) {
      const int64_t idx = mm + Mtot * (int64_t)(a.col0 + r);
      if (a.t_f64) ((double*)a.T)[idx] = o;
      else ((float*)a.T)[idx] = (float)o;
    }
  } else {
    a.partial[((size_t)blockIdx.y * RP + r) * Mpad + mm] = o;
  }
}

inline size_t pm_lds_bytes(int nb) {
  return (size_t)2 * nb * 16 * PITCH * sizeof(float) + nb * 16 * sizeof(double);
}

}  // namespace nncpk
