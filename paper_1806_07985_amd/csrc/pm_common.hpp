// Device helpers shared by the partial-MTTKRP kernels (FP32 and 16-bit tensors).
#pragma once

#include "nncp_internal.hpp"

namespace nncpk {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f2 __attribute__((ext_vector_type(2)));

constexpr int NT = 256;          // threads per work-group (4 waves)

// Vector types of tensor loads, aligned to the element only. A column of a
// tensor view starts at a multiple of its extent, so for most shapes vector
// loads are only element-aligned; gfx950 executes unaligned multi-dword global
// loads, and these types let the compiler emit them.
template <int L>
using f32v = float __attribute__((ext_vector_type(L), aligned(4)));
template <int L>
using u16v = unsigned short __attribute__((ext_vector_type(L), aligned(2)));

// A tensor load, with the nontemporal (streaming) hint when NT.
template <bool NT, typename V>
__device__ __forceinline__ V tload(const V* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Per-(j, column) factor of the Khatri-Rao row: Krest(j, col) = product over the
// contracted modes 1..nm-1 (mode 1 fastest in j) of their factor entries, times
// the column's 1/lambda product over all nm contracted modes (0 where a norm is
// 0), in FP64. All of the entry's loads are issued unconditionally from valid
// addresses before any is used (a load guarded by a branch would be waited for
// at the join), so a batch of entries costs one memory round trip.
__device__ __forceinline__ double krp_scale_entry(const KrpDesc& krp, uint32_t j, int col) {
  float fv[kMaxModes];
  double lv[kMaxModes];
  const int nm = krp.nm;
#pragma unroll
  for (int m = 0; m < kMaxModes; ++m) {
    const int mm = m < nm ? m : 0;
    const uint32_t d = (uint32_t)krp.dim[mm];
    const uint32_t q = j / d;
    const uint32_t dig = (m >= 1 && m < nm) ? j - q * d : 0u;
    if (m >= 1 && m < nm) j = q;
    fv[m] = krp.f[mm][(int64_t)dig + (int64_t)krp.dim[mm] * col];
    lv[m] = krp.lam ? krp.lam[(int64_t)krp.mode[mm] * krp.lam_ld + col] : 1.0;
  }
  double p = 1.0;
#pragma unroll
  for (int m = 0; m < kMaxModes; ++m) {
    if (m < nm) {
      if (m >= 1) p *= (double)fv[m];
      p = lv[m] > 0.0 ? p / lv[m] : 0.0;
    }
  }
  return p;
}

// Fill sc[jj * RP + r] (jj < jn, r < RP) with the Khatri-Rao scales of columns
// col0 + r (times extra[r] when given); 0 for r >= R. Four entries per thread
// per round trip.
template <typename T>
__device__ __forceinline__ void pm_fill_scales(const PmArgs& a, T* sc, int RP, int64_t j0, int jn,
                                               const float* extra) {
  const int total = jn * RP;
  constexpr int CH = 4;
  for (int e0 = threadIdx.x; e0 < total; e0 += NT * CH) {
    double v[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int e = e0 + NT * c;
      const int ec = e < total ? e : 0;
      const int jj = ec / RP, r = ec - jj * RP;
      const int rc = r < a.R ? r : 0;
      v[c] = krp_scale_entry(a.krp, (uint32_t)(j0 + jj), a.col0 + rc);
      if (extra) v[c] *= (double)extra[rc];
      if (r >= a.R) v[c] = 0.0;
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int e = e0 + NT * c;
      if (e < total) sc[e] = (T)v[c];
    }
  }
}

// The FP32 kernels' LDS copy of an i1 block of the first contracted factor:
// hs[r * hp + i] = H_1(i1_0 + i, col0 + r), zero for i1 >= I1 and r >= R. A work
// item is four consecutive rows of one column (one element-aligned 16-byte
// load, element loads where the four straddle I1; hp, i1n and i1_0 are
// multiples of four, so the LDS store is one aligned 16-byte write); eight
// items per thread per round trip, all loads issued before any is stored.
__device__ __forceinline__ void pm_stage_h1(const PmArgs& a, float* hs, int hp, int RP, int i1_0, int i1n) {
  const float* f0 = a.krp.f[0];
  const int q = i1n >> 2;  // items per column
  const int total = RP * q;
  constexpr int CH = 8;
  for (int e0 = threadIdx.x; e0 < total; e0 += NT * CH) {
    f4 v[CH];
    int dst[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int e = e0 + NT * c;
      const int r = e / q, i = 4 * (e - r * q);
      const int i1 = i1_0 + i;
      const bool colok = e < total && r < a.R;
      const float* src = f0 + (int64_t)a.I1 * (a.col0 + (colok ? r : 0));
      f4 x = {0.f, 0.f, 0.f, 0.f};
      if (colok && i1 + 4 <= a.I1) {
        x = *(const f32v<4>*)(src + i1);
      } else if (colok) {
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = (i1 + u < a.I1) ? src[i1 + u] : 0.f;
      }
      v[c] = x;
      dst[c] = e < total ? r * hp + i : -1;
    }
#pragma unroll
    for (int c = 0; c < CH; ++c)
      if (dst[c] >= 0) *(f4*)&hs[dst[c]] = v[c];
  }
}

// LDS prologue of the FP32 kernels: the first i1 block of H_1 and the
// per-(j, column) Khatri-Rao scales sc[jj * RP + r] of the group's j block,
// copied from the launch's scale table when there is one (a contiguous run of
// jn * RP doubles; 16-byte loads, all issued before any is stored), else
// computed here.
__device__ __forceinline__ void pm_prologue(const PmArgs& a, float* hs, int hp, double* sc, int RP, int i1_0,
                                            int i1n, int64_t j0, int jn) {
  pm_stage_h1(a, hs, hp, RP, i1_0, i1n);
  if (a.sctab) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2* src = (const d2*)(a.sctab + j0 * RP);
    const int total = jn * RP / 2;  // RP is a multiple of 16
    constexpr int CH = 4;
    for (int e0 = threadIdx.x; e0 < total; e0 += NT * CH) {
      d2 v[CH];
#pragma unroll
      for (int c = 0; c < CH; ++c) v[c] = src[e0 + NT * c < total ? e0 + NT * c : 0];
#pragma unroll
      for (int c = 0; c < CH; ++c)
        if (e0 + NT * c < total) ((d2*)sc)[e0 + NT * c] = v[c];
    }
  } else {
    pm_fill_scales<double>(a, sc, RP, j0, jn, nullptr);
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

// Store L consecutive output rows m0 .. m0+L-1 of rank column r (values o[]):
// 16-byte stores when the run is in range and aligned (rows are contiguous in
// T and in the partials), element stores otherwise.
template <int L>
__device__ __forceinline__ void pm_store_rows(const PmArgs& a, bool direct, int64_t Mtot, int64_t Mpad, int RP,
                                              int by, int r, int64_t m0, const double (&o)[L]) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  typedef float fv2 __attribute__((ext_vector_type(2)));
  if (direct) {
    if (r >= a.R) return;
    const int64_t base = m0 + Mtot * (int64_t)(a.col0 + r);
    if (m0 + L <= Mtot && (base % L) == 0) {
      if (a.t_f64) {
        d2* p = (d2*)((double*)a.T + base);
#pragma unroll
        for (int i = 0; i < L / 2; ++i) p[i] = d2{o[2 * i], o[2 * i + 1]};
      } else if (L >= 4) {
        f4* p = (f4*)((float*)a.T + base);
#pragma unroll
        for (int i = 0; i < L / 4; ++i)
          p[i] = f4{(float)o[4 * i], (float)o[4 * i + 1], (float)o[4 * i + 2], (float)o[4 * i + 3]};
      } else {
        *(fv2*)((float*)a.T + base) = fv2{(float)o[0], (float)o[1]};
      }
    } else {
#pragma unroll
      for (int i = 0; i < L; ++i)
        if (m0 + i < Mtot) {
          if (a.t_f64) ((double*)a.T)[base + i] = o[i];
          else ((float*)a.T)[base + i] = (float)o[i];
        }
    }
  } else {
    // Mpad is a multiple of the M tile and m0 of L: aligned
    d2* p = (d2*)(a.partial + ((size_t)by * RP + r) * Mpad + m0);
#pragma unroll
    for (int i = 0; i < L / 2; ++i) p[i] = d2{o[2 * i], o[2 * i + 1]};
  }
}

// Split of a flat step range [0, n) into WK contiguous parts.
__device__ __forceinline__ void wave_range(int n, int wk, int WK, int* b, int* e) {
  const int per = (n + WK - 1) / WK;
  *b = wk * per < n ? wk * per : n;
  *e = (wk + 1) * per < n ? (wk + 1) * per : n;
}

}  // namespace nncpk
