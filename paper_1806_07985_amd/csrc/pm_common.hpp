// Device helpers shared by the partial-MTTKRP kernels (FP32 and 16-bit tensors).
#pragma once

#include "nncp_internal.hpp"

namespace nncpk {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));

constexpr int NT = 256;          // threads per work-group (4 waves)

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Digits of index j over the contracted modes 1..nm-1 (mode 1 fastest) and the
// product of those factors' entries in column `col`, in FP64.
__device__ __forceinline__ double krest_value(const KrpDesc& krp, uint32_t j, int col) {
  double p = 1.0;
  for (int m = 1; m < krp.nm; ++m) {
    const uint32_t d = (uint32_t)krp.dim[m];
    const uint32_t q = j / d;
    p *= (double)krp.f[m][(int64_t)(j - q * d) + (int64_t)krp.dim[m] * col];
    j = q;
  }
  return p;
}

// LDS prologue shared by the FP32 kernels: the block's rows of the first
// contracted factor, hs[r * hp + i] = H_1(i1_0 + i, col0 + r) (zero padded), and
// the per-(j, column) scales sc[jj * RP + r] = Krest(j0 + jj, col0 + r) times the
// column's 1/lambda product.
__device__ __forceinline__ void pm_prologue(const PmArgs& a, float* hs, int hp, double* sc, int RP, int i1_0,
                                            int i1n, int64_t j0, int jn) {
  const float* f0 = a.krp.f[0];
  for (int e = threadIdx.x; e < RP * i1n; e += NT) {
    const int r = e / i1n, i = e - r * i1n;
    const int i1 = i1_0 + i;
    hs[r * hp + i] = (r < a.R && i1 < a.I1) ? f0[(int64_t)i1 + (int64_t)a.I1 * (a.col0 + r)] : 0.f;
  }
  for (int e = threadIdx.x; e < jn * RP; e += NT) {
    const int jj = e / RP, r = e - jj * RP;
    double v = 0.0;
    if (r < a.R) v = krp_colscale(a.krp, a.col0 + r) * krest_value(a.krp, (uint32_t)(j0 + jj), a.col0 + r);
    sc[e] = v;
  }
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

// Store one output element: directly into T (FP64 or FP32) or into the split
// partials of split `by`.
__device__ __forceinline__ void pm_store(const PmArgs& a, bool direct, int64_t Mtot, int64_t Mpad, int RP, int by,
                                         int r, int64_t mm, double o) {
  if (direct) {
    if (r < a.R && mm < Mtot) {
      const int64_t idx = mm + Mtot * (int64_t)(a.col0 + r);
      if (a.t_f64) ((double*)a.T)[idx] = o;
      else ((float*)a.T)[idx] = (float)o;
    }
  } else {
    a.partial[((size_t)by * RP + r) * Mpad + mm] = o;
  }
}

// Split of a flat step range [0, n) into WK contiguous parts.
__device__ __forceinline__ void wave_range(int n, int wk, int WK, int* b, int* e) {
  const int per = (n + WK - 1) / WK;
  *b = wk * per < n ? wk * per : n;
  *e = (wk + 1) * per < n ? (wk + 1) * per : n;
}

}  // namespace nncpk
