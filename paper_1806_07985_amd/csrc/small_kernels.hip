// Bandwidth- and latency-bound kernels of the NNCP iteration:
//  * multi-TTV (Section IV-A, Figure 2b): R independent matrix-vector products
//    over the contiguous blocks of a tree-node temporary, FP64 accumulation;
//  * the NLS-Update of one factor (Section II-B): HALS column sweep or the
//    multiplicative rule, one lane group per row, FP64 arithmetic;
//  * Gram matrix, column norms (lambda), the Hadamard product S of the other
//    modes' Grams, and the relative error from ||X||^2 - 2<X,M> + ||M||^2
//    (Section IV-B, appendix algorithm), all accumulated in FP64 with a
//    deterministic two-stage reduction;
//  * ||X||^2 and FP32 -> BF16/FP16 quantisation of the stored tensor.
#include <cstring>
#include <vector>

#include "nncp_internal.hpp"

namespace nncpk {
namespace {

constexpr int NT = 256;

template <typename T>
__device__ __forceinline__ double to_f64(T v);
template <>
__device__ __forceinline__ double to_f64<float>(float v) { return (double)v; }
template <>
__device__ __forceinline__ double to_f64<__bf16>(__bf16 v) { return (double)(float)v; }
template <>
__device__ __forceinline__ double to_f64<_Float16>(_Float16 v) { return (double)(float)v; }

// Element i of a buffer that holds doubles (f64 != 0) or floats.
__device__ __forceinline__ double ldv(const void* p, int64_t i, int f64) {
  return f64 ? ((const double*)p)[i] : (double)((const float*)p)[i];
}
__device__ __forceinline__ void stv(void* p, int64_t i, int f64, double v) {
  if (f64) ((double*)p)[i] = v;
  else ((float*)p)[i] = (float)v;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
  return t;  // valid in thread 0
}

// Returns true in every thread of the last block to arrive (device-scope counter,
// reset to zero by that block).
__device__ __forceinline__ bool last_block(unsigned* counter, unsigned total) {
  __shared__ int s_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    s_last = (prev == total - 1);
    if (s_last) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  if (s_last) __threadfence();
  return s_last;
}

// --------------------------------------------------------------------------
// ||X||^2 in FP64
// --------------------------------------------------------------------------
// Each thread reads 16-byte vectors (4 FP32 or 8 16-bit values), eight of them
// issued before any is used; the vector type is aligned to the element only, so
// any element-aligned base works. The n % VEC tail is read by block 0. Squares
// are exact in FP64 (a 24-bit significand squared fits 53 bits) and summed in
// FP64; the block sums are added by the last block in block order, so the
// result does not depend on scheduling.
template <typename T>
__global__ __launch_bounds__(NT) void norm_sq_kernel(const T* X, int64_t n, double* out,
                                                     double* partial, unsigned* counter) {
  constexpr int VEC = 16 / sizeof(T);
  constexpr int U = 8;
  typedef T vT __attribute__((ext_vector_type(VEC), aligned(sizeof(T))));
  __shared__ double sh[NT / 64];
  const vT* V = (const vT*)X;
  const int64_t nv = n / VEC;
  const int64_t stride = (int64_t)gridDim.x * NT;
  // four independent FP64 sums (vector lane e adds into e % 4), added in a fixed
  // order at the end, so the FMA chains do not serialise the stream
  double s4[4] = {0.0, 0.0, 0.0, 0.0};
  int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x;
  for (; i + (U - 1) * stride < nv; i += U * stride) {
    vT v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(V + i + u * stride);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const double x = to_f64<T>(v[u][e]);
        s4[e % 4] = __builtin_fma(x, x, s4[e % 4]);
      }
  }
  double s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
  for (; i < nv; i += stride) {
    const vT v = __builtin_nontemporal_load(V + i);
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const double x = to_f64<T>(v[e]);
      s = __builtin_fma(x, x, s);
    }
  }
  if (blockIdx.x == 0)
    for (int64_t e = nv * VEC + threadIdx.x; e < n; e += NT) {
      const double x = to_f64<T>(X[e]);
      s = __builtin_fma(x, x, s);
    }
  double t = block_sum(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
  if (!last_block(counter, gridDim.x)) return;
  double u = 0.0;
  if (threadIdx.x == 0) {
    for (unsigned b = 0; b < gridDim.x; ++b) u += partial[b];
    out[0] = u;
  }
}

// --------------------------------------------------------------------------
// FP32 -> BF16 / FP16 (round to nearest even)
// --------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NT) void quantize_kernel(const float* src, T* dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * NT;
  for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += stride) dst[i] = (T)src[i];
}

__global__ void fill_u32_kernel(unsigned* p, int64_t n, unsigned v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void fill_f64_kernel(double* p, int64_t n, double v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void copy_f64_kernel(double* d, const double* s, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = s[i];
}
__global__ void widen_f32_kernel(double* d, const float* s, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = (double)s[i];
}
__global__ void unit_lambda_kernel(double* lam, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) lam[i] = lam[i] > 0.0 ? 1.0 : 0.0;
}

// --------------------------------------------------------------------------
// Multi-TTV, trailing modes: out(i, r) = sum_j T(i, j, r) K(j, r).
// Block: 64 rows i x 4 interleaved phases of j; K(:, r) formed in LDS chunks.
// --------------------------------------------------------------------------
constexpr int TRAIL_KCH = 1024;

template <typename TN>
__device__ __forceinline__ void mttv_trail_body(const MttvArgs& a, int bx, int r) {
  __shared__ double kv[TRAIL_KCH];
  __shared__ double red[4][64];
  const int ti = threadIdx.x & 63, ph = threadIdx.x >> 6;
  const int64_t i = (int64_t)bx * 64 + ti;
  const double scale = krp_colscale(a.krp, r);
  const TN* Tr = (const TN*)a.T + (int64_t)r * a.Ia * a.J;
  double acc = 0.0;
  for (int64_t j0 = 0; j0 < a.J; j0 += TRAIL_KCH) {
    const int cnt = (int)((a.J - j0) < TRAIL_KCH ? (a.J - j0) : TRAIL_KCH);
    __syncthreads();
    // the Khatri-Rao column chunk: every factor load is issued (from a valid
    // address) before any product is formed
    for (int e = threadIdx.x; e < cnt; e += NT) {
      uint32_t rem = (uint32_t)(j0 + e);
      float fv[kMaxModes];
#pragma unroll
      for (int m = 0; m < kMaxModes; ++m) {
        const int mm = m < a.krp.nm ? m : 0;
        const uint32_t d = (uint32_t)a.krp.dim[mm];
        const uint32_t q = rem / d;
        const uint32_t dig = m < a.krp.nm ? rem - q * d : 0u;
        if (m < a.krp.nm) rem = q;
        fv[m] = a.krp.f[mm][(int64_t)dig + (int64_t)a.krp.dim[mm] * r];
      }
      double p = scale;
#pragma unroll
      for (int m = 0; m < kMaxModes; ++m)
        if (m < a.krp.nm) p *= (double)fv[m];
      kv[e] = p;
    }
    __syncthreads();
    // sixteen rows j of this phase in flight per step (each thread still adds
    // its rows j = ph, ph + 4, ... in increasing order); rows past the chunk
    // (or past I_a) read a valid element and are weighted by zero
    const int64_t ic = i < a.Ia ? i : 0;
    const TN* base = Tr + ic + a.Ia * j0;
    for (int e = ph; e < cnt; e += 64) {
      TN t[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int ej = e + 4 * u;
        t[u] = base[a.Ia * (int64_t)(ej < cnt ? ej : e)];
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int ej = e + 4 * u;
        if (ej < cnt) acc += (double)t[u] * kv[ej];
      }
    }
  }
  red[ph][ti] = acc;
  __syncthreads();
  if (ph == 0 && i < a.Ia) {
    double s = red[0][ti] + red[1][ti] + red[2][ti] + red[3][ti];
    stv(a.out, i + a.Ia * r, a.out_f64, s);
  }
}
template <typename TN>
__global__ __launch_bounds__(NT) void mttv_trail_kernel(MttvArgs a) {
  mttv_trail_body<TN>(a, blockIdx.x, blockIdx.y);
}

// --------------------------------------------------------------------------
// Multi-TTV, leading modes: out(j, r) = sum_i T(i, j, r) K(i, r), i over the
// leading mode(s) of the node (K = their Khatri-Rao product, the first
// fastest; one mode: K = H), one lane group of GS lanes per output
// (contiguous dot product, shuffle reduction).
// --------------------------------------------------------------------------
template <int GS, typename TN>
__device__ __forceinline__ void mttv_lead_body(const MttvArgs& a, int bx) {
  constexpr int OPB = NT / GS;
  const int g = threadIdx.x / GS, p = threadIdx.x % GS;
  const int64_t o = (int64_t)bx * OPB + g;  // output index j + J*r
  const int64_t total = a.J * a.R;
  double acc = 0.0;
  int r = 0;
  if (o < total) {
    r = (int)(o / a.J);
    const int64_t j = o - (int64_t)r * a.J;
    const TN* Tc = (const TN*)a.T + a.Ia * (j + a.J * (int64_t)r);
    if (a.krp.nm == 1) {
      // eight products of the lane in flight, added in increasing i
      const float* Hc = a.krp.f[0] + a.Ia * (int64_t)r;
      int64_t i = p;
      for (; i + 7 * GS < a.Ia; i += 8 * GS) {
        TN t[8];
        float h[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          t[u] = Tc[i + u * GS];
          h[u] = Hc[i + u * GS];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += (double)t[u] * (double)h[u];
      }
      for (; i < a.Ia; i += GS) acc += (double)Tc[i] * (double)Hc[i];
    } else {
      const bool narrow = a.Ia <= (int64_t)UINT32_MAX;  // 32-bit index arithmetic suffices
      for (int64_t i = p; i < a.Ia; i += GS) {
        double k = 1.0;
        if (narrow) {
          uint32_t rem = (uint32_t)i;
          for (int m = 0; m < a.krp.nm; ++m) {
            const uint32_t d = (uint32_t)a.krp.dim[m];
            const uint32_t q = rem / d;
            k *= (double)a.krp.f[m][(int64_t)(rem - q * d) + (int64_t)d * r];
            rem = q;
          }
        } else {
          int64_t rem = i;
          for (int m = 0; m < a.krp.nm; ++m) {
            const int64_t d = a.krp.dim[m];
            const int64_t q = rem / d;
            k *= (double)a.krp.f[m][(rem - q * d) + d * r];
            rem = q;
          }
        }
        acc += (double)Tc[i] * k;
      }
    }
  }
#pragma unroll
  for (int off = GS / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, GS);
  if (p == 0 && o < total) stv(a.out, o, a.out_f64, acc * krp_colscale(a.krp, r));
}
template <int GS, typename TN>
__global__ __launch_bounds__(NT) void mttv_lead_kernel(MttvArgs a) {
  mttv_lead_body<GS, TN>(a, blockIdx.x);
}

// --------------------------------------------------------------------------
// NLS update (Section II-B), one wave per row. Lane p holds columns
// k = p + 64*v (v < VPL) of the warm start w, the MTTKRP row m and the running
// product g = w S. HALS visits r = 0..R-1 in order (Gauss-Seidel): every lane
// forms its candidate change, the owner's one is broadcast with readlane, and
// every lane updates g += d S(r, :). S and 1/S(r,r) live in LDS; all FP64.
// --------------------------------------------------------------------------
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, lane);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), lane);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

template <int VPL>
__device__ __forceinline__ void update_body(const UpdateArgs& a, int bx) {
  extern __shared__ double Sl[];  // R*R, then R inverse diagonals
  const int R = a.R;
  double* invd = Sl + R * R;
  const int p = threadIdx.x & 63;
  const int64_t row = (int64_t)bx * (NT / 64) + (threadIdx.x >> 6);
  const bool live = row < a.I;  // wave-uniform
  // this row's loads are issued before S is staged, so their latency overlaps it
  double w[VPL], m[VPL], g[VPL];
#pragma unroll
  for (int v = 0; v < VPL; ++v) {
    const int k = p + 64 * v;
    w[v] = 0.0;
    m[v] = 0.0;
    g[v] = 0.0;
    if (live && k < R) {
      const double ls = a.lam_self[k];
      const double f = ls > 0.0 ? a.lam_model[k] / ls : 0.0;
      w[v] = (double)a.W[row + a.I * k] * f;
      m[v] = ldv(a.M, row + a.I * k, a.m_f64);
    }
  }
  for (int e = threadIdx.x; e < R * R; e += NT) Sl[e] = a.S[e];
  for (int k = threadIdx.x; k < R; k += NT) {
    const double d = a.S[k * R + k];
    invd[k] = d > 0.0 ? 1.0 / d : 0.0;
  }
  __syncthreads();
  if (!live) return;  // whole wave leaves together

  // g = w S with the starting w
  auto wS = [&]() {
#pragma unroll
    for (int q = 0; q < VPL; ++q) g[q] = 0.0;
    for (int r = 0; r < R; ++r) {
      const int v = r >> 6;
      double wv = w[0];
#pragma unroll
      for (int q = 1; q < VPL; ++q)
        if (v == q) wv = w[q];
      const double wr = readlane_f64(wv, r & 63);
#pragma unroll
      for (int q = 0; q < VPL; ++q) {
        const int k = p + 64 * q;
        if (k < R) g[q] += wr * Sl[r * R + k];
      }
    }
  };
  wS();
  const int sweeps = a.sweeps > 1 ? a.sweeps : 1;
  const double tol = a.tol;
  // the row's largest |w| (all lanes), for the relative change of a sweep
  auto wave_absmax = [&]() {
    double m = 0.0;
#pragma unroll
    for (int q = 0; q < VPL; ++q) m = fmax(m, fabs(w[q]));
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    return m;
  };
  if (a.update == NNCP_HALS) {
    // g stays equal to w S across sweeps: every column change is added to it
    for (int sw = 0; sw < sweeps; ++sw) {
      double dmax = 0.0;  // the sweep's largest |change| (uniform: every change is broadcast)
      for (int r = 0; r < R; ++r) {
        const int v = r >> 6;
        double wv = w[0], mv = m[0], gv = g[0];
  #pragma unroll
        for (int q = 1; q < VPL; ++q)
          if (v == q) {
            wv = w[q];
            mv = m[q];
            gv = g[q];
          }
        // column r: W(:,r) <- max(0, W(:,r) + (M(:,r) - (W S)(:,r)) / S(r,r)); a zero
        // diagonal (all-zero column elsewhere) sets the column to zero
        const double id = invd[r];
        double wn = id > 0.0 ? wv + (mv - gv) * id : 0.0;
        wn = wn > 0.0 ? wn : 0.0;
        const double d = readlane_f64(wn - wv, r & 63);
        dmax = fmax(dmax, fabs(d));
        if (p == (r & 63)) {
  #pragma unroll
          for (int q = 0; q < VPL; ++q)
            if (v == q) w[q] += d;
        }
  #pragma unroll
        for (int q = 0; q < VPL; ++q) {
          const int k = p + 64 * q;
          if (k < R) g[q] += d * Sl[r * R + k];
        }
      }
      if (tol > 0.0 && dmax <= tol * wave_absmax()) break;  // uniform
    }
  } else {
    for (int sw = 0; sw < sweeps; ++sw) {
      if (sw > 0) wS();
      double dloc = 0.0;
#pragma unroll
      for (int v = 0; v < VPL; ++v) {
        const double den = g[v] > 1e-16 ? g[v] : 1e-16;
        const double wn = w[v] * m[v] / den;
        dloc = fmax(dloc, fabs(wn - w[v]));
        w[v] = wn;
      }
      if (tol > 0.0) {
        for (int o = 32; o > 0; o >>= 1) dloc = fmax(dloc, __shfl_xor(dloc, o, 64));
        if (dloc <= tol * wave_absmax()) break;  // uniform
      }
    }
  }
#pragma unroll
  for (int v = 0; v < VPL; ++v) {
    const int k = p + 64 * v;
    if (k < R) {
      a.W[row + a.I * k] = (float)w[v];
      if (a.W64) a.W64[row + a.I * k] = w[v];
    }
  }
}
template <int VPL>
__global__ __launch_bounds__(NT) void update_kernel(UpdateArgs a) {
  update_body<VPL>(a, blockIdx.x);
}

// One row's update with lane k's column of S in registers (R <= RB <= 64): w =
// W(row, k) scaled to the model, m = M(row, k), srow[r] = S(r, k) (zero for r >= R
// or k >= R), invd = 1 / S(k, k) (zero unless positive). The column sweeps are
// unrolled over RB, so every broadcast uses a constant lane and the Gauss-Seidel
// chain touches no memory. Returns the new w.
// With tol > 0 the sweeps stop early, once a sweep changes no entry of the row
// by more than tol times the row's largest entry (the row is one NNLS
// subproblem of the block; the rows are independent).
__device__ __forceinline__ double wave_max_f64(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
template <int RB>
__device__ __forceinline__ double update_row_reg(double w, const double m, const double (&srow)[RB],
                                                 const double invd, const int k, const int R, const int update,
                                                 const int sweeps, const double tol) {
  double g = 0.0;
#pragma unroll
  for (int r = 0; r < RB; ++r) g += readlane_f64(w, r) * srow[r];
  if (update == NNCP_HALS) {
    double dmax = 0.0;  // a sweep's largest |change| (uniform: every change is broadcast)
    auto sweep = [&]() {
      // fresh copies of the lane index and the rank per sweep: the per-column
      // compares below then stay inside the sweep instead of being hoisted out of
      // the sweep loop into 64 live lane masks
      int kv, Rv;
      asm volatile("v_mov_b32 %0, %1" : "=v"(kv) : "v"(k));
      asm volatile("s_mov_b32 %0, %1" : "=s"(Rv) : "s"(R));
#pragma unroll
      for (int r = 0; r < RB; ++r) {
        if (r < Rv) {  // uniform
          // column r: W(:,r) <- max(0, W(:,r) + (M(:,r) - (W S)(:,r)) / S(r,r)); a zero
          // diagonal sets the column to zero (lane r owns column r)
          double wn = invd > 0.0 ? w + (m - g) * invd : 0.0;
          wn = wn > 0.0 ? wn : 0.0;
          const double dlt = readlane_f64(wn - w, r);
          dmax = fmax(dmax, fabs(dlt));
          if (kv == r) w += dlt;
          g += dlt * srow[r];
        }
      }
    };
    // g stays equal to w S across sweeps: every column change is added to it
    if (tol > 0.0) {
      for (int sw = 0; sw < sweeps; ++sw) {
        dmax = 0.0;
        sweep();
        if (dmax <= tol * wave_max_f64(fabs(w))) break;  // uniform
      }
    } else {
      for (int sw = 0; sw < sweeps; ++sw) sweep();
    }
  } else {
    for (int sw = 0; sw < sweeps; ++sw) {
      if (sw > 0) {
        g = 0.0;
#pragma unroll
        for (int r = 0; r < RB; ++r) g += readlane_f64(w, r) * srow[r];
      }
      const double den = g > 1e-16 ? g : 1e-16;
      const double wn = w * m / den;
      const double d = fabs(wn - w);
      w = wn;
      if (tol > 0.0 && wave_max_f64(d) <= tol * wave_max_f64(fabs(w))) break;  // uniform
    }
  }
  return w;
}

// Lane k's column of S (zero outside R x R) and 1 / S(k, k), loaded unconditionally.
template <int RB>
__device__ __forceinline__ void load_s_column(const UpdateArgs& a, int k, double (&srow)[RB], double& invd) {
  const int R = a.R;
  const bool col = k < R;
  const int kc = col ? k : 0;
#pragma unroll
  for (int r = 0; r < RB; ++r) srow[r] = a.S[(int64_t)(r < R ? r : 0) * R + kc];  // S symmetric
  const double dg = a.S[(int64_t)kc * R + kc];
  invd = (col && dg > 0.0) ? 1.0 / dg : 0.0;
#pragma unroll
  for (int r = 0; r < RB; ++r)
    if (!(col && r < R)) srow[r] = 0.0;
}

// The update for R <= RB <= 64: one wave per row.
template <int RB>
__device__ __forceinline__ void update_reg_body(const UpdateArgs& a, int bx) {
  const int R = a.R;
  const int k = threadIdx.x & 63;
  const int64_t row = (int64_t)bx * (NT / 64) + (threadIdx.x >> 6);
  if (row >= a.I) return;  // wave-uniform; no barrier in this kernel
  const bool col = k < R;
  const int kc = col ? k : 0;  // every load is unconditional (from a valid index), masked after
  const double ls = a.lam_self[kc], lm = a.lam_model[kc];
  const double w0 = (double)a.W[row + a.I * kc];
  const double m0 = ldv(a.M, row + a.I * kc, a.m_f64);
  double srow[RB], invd;
  load_s_column<RB>(a, k, srow, invd);
  const double f = ls > 0.0 ? lm / ls : 0.0;
  const double w = update_row_reg<RB>(col ? w0 * f : 0.0, col ? m0 : 0.0, srow, invd, k, R, a.update,
                                      a.sweeps > 1 ? a.sweeps : 1, a.tol);
  if (col) {
    a.W[row + a.I * k] = (float)w;
    if (a.W64) a.W64[row + a.I * k] = w;
  }
}
template <int RB>
__global__ __launch_bounds__(NT) void update_reg_kernel(UpdateArgs a) {
  update_reg_body<RB>(a, blockIdx.x);
}

// Rows of W staged in LDS at a time (FP64): about 32 KB.
__host__ __device__ inline int fin_sub_rows(int R) {
  int r = 4096 / (R > 0 ? R : 1);
  return r < 1 ? 1 : (r > 256 ? 256 : r);
}

// Stage 1: W^T W (and <M, W> when the fit is due) over this block's row chunk,
// written to partial[chunk] (R*R + 1 doubles).
__device__ void gram_chunk(const FinalizeArgs& a, double* fl, double* sh, int bx) {
  const int R = a.R, RR = R * R;
  const int sub = fin_sub_rows(R);
  const int64_t r0 = (int64_t)bx * a.rows_per_chunk;
  int64_t r1 = r0 + a.rows_per_chunk;
  if (r1 > a.I) r1 = a.I;
  double* part = a.partial + (size_t)bx * (RR + 1);
  // Each thread owns entries e = tid, tid + NT, ...; the running sums live in
  // this block's partial slot (only this thread touches them).
  double bsum = 0.0;
  bool first = true;
  for (int64_t s0 = r0; s0 < r1 || first; s0 += sub) {
    const int cnt = (int)((r1 - s0) < sub ? (r1 - s0) : sub);
    __syncthreads();
    for (int e = threadIdx.x; e < cnt * R; e += NT) {
      const int k = e / cnt, rw = e - k * cnt;
      const double wv = (double)a.W[s0 + rw + a.I * k];
      fl[rw * R + k] = wv;
      if (a.do_fit && a.M) bsum += wv * ldv(a.M, s0 + rw + a.I * k, a.m_f64);
    }
    __syncthreads();
    // four entries per thread at a time (independent FMA chains), rows unrolled
    for (int eg = threadIdx.x; eg < RR; eg += 4 * NT) {
      int ex[4], ey[4];
      double sacc[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = eg + q * NT < RR ? eg + q * NT : eg;
        ex[q] = e / R;
        ey[q] = e - ex[q] * R;
        sacc[q] = 0.0;
      }
#pragma unroll 4
      for (int rw = 0; rw < cnt; ++rw) {
        const double* row = fl + rw * R;
#pragma unroll
        for (int q = 0; q < 4; ++q) sacc[q] += row[ex[q]] * row[ey[q]];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = eg + q * NT;
        if (e < RR) part[e] = first ? sacc[q] : part[e] + sacc[q];
      }
    }
    first = false;
  }
  double bt = block_sum(bsum, sh);
  if (threadIdx.x == 0) part[RR] = bt;
}

// Stage 2 (one block): reduce the chunk partials in chunk order, then lambda =
// sqrt(diag G_hat), the normalised Gram, the model weights, S for the next mode
// and, after the last mode, the fit.
__device__ void finalize_tail(const FinalizeArgs& a, double* fl, double* sh) {
  const int R = a.R, RR = R * R;
  double* Gh = fl;  // R*R + 1 scratch
  for (int e = threadIdx.x; e < RR + 1; e += NT) {
    double s = 0.0;
    for (int c = 0; c < a.nchunks; ++c) s += a.partial[(size_t)c * (RR + 1) + e];
    Gh[e] = s;
  }
  __syncthreads();
  if (a.gram_raw)
    for (int e = threadIdx.x; e < RR; e += NT) a.gram_raw[e] = Gh[e];
  double* lamm = a.lam + (int64_t)a.mode * R;
  for (int k = threadIdx.x; k < R; k += NT) {
    const double l = sqrt(Gh[k * R + k]);
    lamm[k] = l;
    if (a.set_model) a.lam_model[k] = l;
  }
  double* Gm = a.G + (int64_t)a.mode * RR;
  for (int e = threadIdx.x; e < RR; e += NT) {
    const int x = e / R, y = e - x * R;
    const double lx = sqrt(Gh[x * R + x]), ly = sqrt(Gh[y * R + y]);
    Gm[e] = (lx > 0.0 && ly > 0.0) ? Gh[e] / (lx * ly) : 0.0;
  }
  __syncthreads();
  if (a.do_fit) {
    // gamma = 1^T (S^(mode) * G_hat) 1, S^(mode) the Hadamard of the other Grams
    const double* Sm = a.S + (int64_t)a.mode * RR;
    double gp = 0.0;
    for (int e = threadIdx.x; e < RR; e += NT) gp += Sm[e] * Gh[e];
    double gamma = block_sum(gp, sh);
    if (threadIdx.x == 0) {
      const double alpha = a.alpha[0];
      const double beta = Gh[RR];
      double num = alpha - 2.0 * beta + gamma;
      num = num > 0.0 ? num : 0.0;
      const double eps = alpha > 0.0 ? sqrt(num / alpha) : 0.0;
      const int it = *a.iter_counter;
      if (it < a.fit_capacity) a.fit_out[it] = 1.0 - eps;
      *a.iter_counter = it + 1;
    }
    __syncthreads();
  }
  if (a.next_mode >= 0) {
    // this block wrote G[mode] above; the other modes' Grams are from earlier kernels
    double* Sn = a.S + (int64_t)a.next_mode * RR;
    for (int e = threadIdx.x; e < RR; e += NT) {
      double s = 1.0;
      for (int k = 0; k < a.N; ++k)
        if (k != a.next_mode) s *= a.G[(int64_t)k * RR + e];
      Sn[e] = s;
    }
  }
}

// Ranks up to this use the 1024-thread Gram kernels below (4 x 4 register blocks of W^T W).
constexpr int kSmallMaxR = 64;

__host__ __device__ inline int gram_r4(int R) { return (R + 3) & ~3; }

// One block does both stages (a single row chunk).
__device__ __forceinline__ void finalize_fused_body(const FinalizeArgs& a) {
  extern __shared__ double fl[];
  __shared__ double sh[NT / 64];
  gram_chunk(a, fl, sh, 0);
  __syncthreads();
  finalize_tail(a, fl, sh);
}
__device__ __forceinline__ void gram_chunks_body(const FinalizeArgs& a, int bx) {
  extern __shared__ double fl[];
  __shared__ double sh[NT / 64];
  gram_chunk(a, fl, sh, bx);
}
__device__ __forceinline__ void finalize_tail_body(const FinalizeArgs& a) {
  extern __shared__ double fl[];
  __shared__ double sh[NT / 64];
  finalize_tail(a, fl, sh);
}
__global__ __launch_bounds__(NT) void finalize_fused_kernel(FinalizeArgs a) { finalize_fused_body(a); }
__global__ __launch_bounds__(NT) void gram_chunks_kernel(FinalizeArgs a) { gram_chunks_body(a, blockIdx.x); }
__global__ __launch_bounds__(NT) void finalize_tail_kernel(FinalizeArgs a) { finalize_tail_body(a); }

// ---------------------------------------------------------------------------
// Gram, lambda, next S and the fit for R <= 64 with 1024-thread work-groups.
// Sixteen waves per group (four per SIMD) hide one another's latencies where a
// 4-wave group left every latency exposed; only the upper triangle of 4x4
// blocks of W^T W is computed (the lower one is its mirror, bit for bit); and
// every global value the group needs is requested before the first is used.
// The staged rows have an odd stride in doubles, so a wave's column writes
// spread over the LDS banks. Entry e of an R x R matrix belongs to thread
// e mod 1024, slot e / 1024 (at most four slots).
constexpr int NTF = 1024;
constexpr int kFinStage = 8192;           // staged elements (rows x R4) per round
constexpr int kFinQS = kFinStage / NTF;   // staged elements per thread
constexpr int kFinMaxPh = 32;             // at most this many row phases per block

__host__ __device__ inline int fin_nb4(int R) { return gram_r4(R) >> 2; }
__host__ __device__ inline int fin_nblk(int R) { return fin_nb4(R) * (fin_nb4(R) + 1) / 2; }
__host__ __device__ inline int fin_nph(int R) {
  const int p = NTF / fin_nblk(R);
  return p < kFinMaxPh ? p : kFinMaxPh;
}
__host__ __device__ inline int fin_rows(int R) { return kFinStage / gram_r4(R); }
__host__ __device__ inline int fin_stride(int R) { return gram_r4(R) + 1; }
// dynamic LDS doubles: the staged rows, reused for the phase partials (<= 128 KB)
__host__ __device__ inline int fin_work_doubles(int R) {
  const int st = fin_rows(R) * fin_stride(R), ph = 16 * fin_nph(R) * fin_nblk(R);
  return st > ph ? st : ph;
}
// R x R entries per thread: 1, 2 or 4
__host__ __device__ inline int fin_ep(int R) { return R * R <= NTF ? 1 : (R * R <= 2 * NTF ? 2 : 4); }

// block (bx, by), bx <= by, of upper-triangle index b (row-major over the triangle)
__device__ __forceinline__ void tri_block(int b, int nb4, int& bx, int& by) {
  int x = 0;
  while (b >= nb4 - x) {
    b -= nb4 - x;
    ++x;
  }
  bx = x;
  by = x + b;
}
__device__ __forceinline__ int tri_index(int bx, int by, int nb4) { return bx * nb4 - bx * (bx - 1) / 2 + (by - bx); }

// Stage-load of rows [s0, s0 + cnt): element e = tid + NTF*q is (row s0 + e mod cnt,
// column e / cnt); columns R..R4-1 are zero. Loads are unconditional (clamped index).
__device__ __forceinline__ void fin_load(const FinalizeArgs& a, int64_t s0, int cnt, bool fit, float (&wf)[kFinQS],
                                         double (&mv)[kFinQS]) {
  const int R4 = gram_r4(a.R), tid = threadIdx.x;
  const int dk = NTF / cnt, drw = NTF - dk * cnt;
  int k = tid / cnt, rw = tid - (tid / cnt) * cnt;
#pragma unroll
  for (int q = 0; q < kFinQS; ++q) {
    const bool ok = tid + NTF * q < cnt * R4 && k < a.R;
    const int64_t idx = ok ? s0 + rw + a.I * (int64_t)k : 0;
    const float w = a.W[idx];
    wf[q] = ok ? w : 0.f;
    if (fit) {
      const double m = ldv(a.M, idx, a.m_f64);
      mv[q] = ok ? m : 0.0;
    }
    k += dk;
    rw += drw;
    if (rw >= cnt) {
      rw -= cnt;
      ++k;
    }
  }
}
__device__ __forceinline__ void fin_store(const FinalizeArgs& a, int cnt, const float (&wf)[kFinQS], double* work) {
  const int R4 = gram_r4(a.R), str = R4 + 1, tid = threadIdx.x;
  const int dk = NTF / cnt, drw = NTF - dk * cnt;
  int k = tid / cnt, rw = tid - (tid / cnt) * cnt;
#pragma unroll
  for (int q = 0; q < kFinQS; ++q) {
    if (tid + NTF * q < cnt * R4) work[rw * str + k] = (double)wf[q];
    k += dk;
    rw += drw;
    if (rw >= cnt) {
      rw -= cnt;
      ++k;
    }
  }
}

// W^T W over rows [r0, r1) into g[q] (entry tid + NTF*q; raw, unnormalised) and
// beta = sum of M o W over those rows (thread 0, when the fit is due). Block-wide;
// work: fin_work_doubles. The code is kept short on purpose: these kernels run
// once per mode on one group, and their time follows the instruction bytes that
// must be fetched more than the arithmetic.
template <int EP>
__device__ __forceinline__ void gram1k_rows(const FinalizeArgs& a, int64_t r0, int64_t r1, double* work, double* sh,
                                            double (&g)[EP], double& beta) {
  const int R = a.R, RR = R * R, tid = threadIdx.x;
  const int nb4 = fin_nb4(R), nblk = fin_nblk(R), nph = fin_nph(R), str = fin_stride(R), sub = fin_rows(R);
  const bool active = tid < nblk * nph;
  const int blk = tid % nblk, ph = tid / nblk;
  int bx, by;
  tri_block(active ? blk : 0, nb4, bx, by);
  const bool fit = a.do_fit && a.M;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  double bsum = 0.0;
  for (int64_t s0 = r0; s0 < r1; s0 += sub) {
    const int cnt = (int)(r1 - s0 < sub ? r1 - s0 : sub);
    float wf[kFinQS];
    double mv[kFinQS];
    fin_load(a, s0, cnt, fit, wf, mv);
    if (fit) {
#pragma unroll
      for (int q = 0; q < kFinQS; ++q) bsum += (double)wf[q] * mv[q];
    }
    __syncthreads();  // the previous round's rows are no longer read
    fin_store(a, cnt, wf, work);
    __syncthreads();
    if (active) {
      for (int r = ph; r < cnt; r += nph) {
        const double* row = work + r * str;
        double x[4], y[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          x[i] = row[4 * bx + i];
          y[i] = row[4 * by + i];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] += x[i] * y[j];
      }
    }
  }
  beta = fit ? block_sum(bsum, sh) : 0.0;
  // phases summed in phase order through LDS: [block entry][phase][block]
  __syncthreads();
  if (active) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) work[((i * 4 + j) * nph + ph) * nblk + blk] = acc[i][j];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < EP; ++q) {
    const int e = tid + NTF * q;
    const int ec = e < RR ? e : 0;
    const int x = ec / R, y = ec - (ec / R) * R;
    const int X = x >> 2, Y = y >> 2;
    const int b = X <= Y ? tri_index(X, Y, nb4) : tri_index(Y, X, nb4);
    const int qv = X <= Y ? (x & 3) * 4 + (y & 3) : (y & 3) * 4 + (x & 3);
    const double* src = work + (size_t)qv * nph * nblk + b;
    double s = 0.0;
    for (int p0 = 0; p0 < nph; p0 += 8) {  // eight loads in flight, added in order
      double t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) t[u] = src[(size_t)(p0 + u < nph ? p0 + u : 0) * nblk];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += p0 + u < nph ? t[u] : 0.0;
    }
    g[q] = s;
  }
}

// What the tail needs from global memory, requested up front: the product P of
// the Grams of the modes other than `mode` and `next_mode` (for S of the next
// mode), S of this mode (for gamma), alpha and the iteration counter.
template <int EP>
struct FinPre {
  double P[EP], Sm[EP];
  double alpha;
  int it;
};
template <int EP>
__device__ __forceinline__ void fin_preload(const FinalizeArgs& a, FinPre<EP>& p) {
  const int RR = a.R * a.R, tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < EP; ++q) p.P[q] = 1.0;
  if (a.next_mode >= 0) {
    const int lo = a.mode < a.next_mode ? a.mode : a.next_mode;
    const int hi = a.mode < a.next_mode ? a.next_mode : a.mode;
#pragma unroll
    for (int j = 0; j < kMaxModes - 2; ++j) {
      int k = j;
      if (k >= lo) ++k;
      if (k >= hi) ++k;
      const bool use = k < a.N;
      const int kc = use ? k : 0;
      double t[EP];
#pragma unroll
      for (int q = 0; q < EP; ++q) {
        const int e = tid + NTF * q;
        t[q] = a.G[(int64_t)kc * RR + (e < RR ? e : 0)];
      }
#pragma unroll
      for (int q = 0; q < EP; ++q) p.P[q] *= use ? t[q] : 1.0;
    }
  }
#pragma unroll
  for (int q = 0; q < EP; ++q) p.Sm[q] = 0.0;
  p.alpha = 0.0;
  p.it = 0;
  if (a.do_fit) {  // S, alpha and the counter are only there when the fit is due
#pragma unroll
    for (int q = 0; q < EP; ++q) {
      const int e = tid + NTF * q;
      p.Sm[q] = a.S[(int64_t)a.mode * RR + (e < RR ? e : 0)];
    }
    p.alpha = a.alpha[0];
    p.it = *a.iter_counter;
  }
}

// lambda, normalised Gram, S of the next mode, the raw Gram if asked, and the fit.
template <int EP>
__device__ __forceinline__ void fin1k_tail(const FinalizeArgs& a, const double (&g)[EP], double beta, const FinPre<EP>& p,
                           double* sh) {
  __shared__ double dg[kSmallMaxR], il[kSmallMaxR];
  const int R = a.R, RR = R * R, tid = threadIdx.x;
  int xs[EP], ys[EP];
#pragma unroll
  for (int q = 0; q < EP; ++q) {
    const int e = tid + NTF * q;
    const int ec = e < RR ? e : 0;
    xs[q] = ec / R;
    ys[q] = ec - xs[q] * R;
    if (e < RR && xs[q] == ys[q]) dg[xs[q]] = g[q];
  }
  __syncthreads();
  double* lamm = a.lam + (int64_t)a.mode * R;
  if (tid < R) {
    const double l = sqrt(dg[tid]);
    lamm[tid] = l;
    if (a.set_model) a.lam_model[tid] = l;
    il[tid] = l > 0.0 ? 1.0 / l : 0.0;
  }
  __syncthreads();
  double* Gm = a.G + (int64_t)a.mode * RR;
  double* Sn = a.next_mode >= 0 ? a.S + (int64_t)a.next_mode * RR : nullptr;
  double gp = 0.0;
#pragma unroll
  for (int q = 0; q < EP; ++q) {
    const int e = tid + NTF * q;
    if (e < RR) {
      const double gn = g[q] * il[xs[q]] * il[ys[q]];
      Gm[e] = gn;
      if (Sn) Sn[e] = p.P[q] * gn;
      if (a.gram_raw) a.gram_raw[e] = g[q];
      gp += p.Sm[q] * g[q];
    }
  }
  if (a.do_fit) {
    // gamma = 1^T (S^(mode) * G_hat) 1 with G_hat the Gram of the unnormalised factor
    const double gamma = block_sum(gp, sh);
    if (tid == 0) {
      double num = p.alpha - 2.0 * beta + gamma;
      num = num > 0.0 ? num : 0.0;
      const double eps = p.alpha > 0.0 ? sqrt(num / p.alpha) : 0.0;
      if (p.it < a.fit_capacity) a.fit_out[p.it] = 1.0 - eps;
      *a.iter_counter = p.it + 1;
    }
  }
}

// One row chunk: everything in one group.
template <int EP>
__device__ __forceinline__ void fin1k_body(const FinalizeArgs& a) {
  extern __shared__ double lds[];
  __shared__ double sh[NTF / 64];
  FinPre<EP> p;
  fin_preload(a, p);
  double g[EP], beta;
  gram1k_rows<EP>(a, 0, a.I, lds, sh, g, beta);
  fin1k_tail<EP>(a, g, beta, p, sh);
}
// Several row chunks: chunk bx's Gram and beta into partial[bx] ...
template <int EP>
__device__ __forceinline__ void gram1k_chunk_body(const FinalizeArgs& a, int bx) {
  extern __shared__ double lds[];
  __shared__ double sh[NTF / 64];
  const int RR = a.R * a.R;
  const int64_t r0 = (int64_t)bx * a.rows_per_chunk;
  const int64_t r1 = r0 + a.rows_per_chunk < a.I ? r0 + a.rows_per_chunk : a.I;
  double g[EP], beta;
  gram1k_rows<EP>(a, r0, r1, lds, sh, g, beta);
  double* out = a.partial + (size_t)bx * (RR + 1);
#pragma unroll
  for (int q = 0; q < EP; ++q) {
    const int e = threadIdx.x + NTF * q;
    if (e < RR) out[e] = g[q];
  }
  if (threadIdx.x == 0) out[RR] = beta;
}
// ... then one group sums the partials in chunk order and finishes.
template <int EP>
__device__ __forceinline__ void tail1k_body(const FinalizeArgs& a) {
  __shared__ double sh[NTF / 64];
  const int RR = a.R * a.R, tid = threadIdx.x;
  FinPre<EP> p;
  fin_preload(a, p);
  double g[EP];
#pragma unroll
  for (int q = 0; q < EP; ++q) g[q] = 0.0;
  double beta = 0.0;
  constexpr int CB = EP == 1 ? 16 : (EP == 2 ? 8 : 4);  // chunks whose loads fly together
  for (int c0 = 0; c0 < a.nchunks; c0 += CB) {
    double t[CB][EP], tb[CB];
#pragma unroll
    for (int u = 0; u < CB; ++u) {
      const int c = c0 + u < a.nchunks ? c0 + u : 0;
      const double* pc = a.partial + (size_t)c * (RR + 1);
#pragma unroll
      for (int q = 0; q < EP; ++q) {
        const int e = tid + NTF * q;
        t[u][q] = pc[e < RR ? e : 0];
      }
      tb[u] = pc[RR];
    }
#pragma unroll
    for (int u = 0; u < CB; ++u) {
      if (c0 + u < a.nchunks) {
#pragma unroll
        for (int q = 0; q < EP; ++q) g[q] += t[u][q];
        beta += tb[u];
      }
    }
  }
  fin1k_tail<EP>(a, g, beta, p, sh);
}

template <int EP>
__global__ __launch_bounds__(NTF) void fin1k_kernel(FinalizeArgs a) { fin1k_body<EP>(a); }
template <int EP>
__global__ __launch_bounds__(NTF) void gram1k_chunk_kernel(FinalizeArgs a) { gram1k_chunk_body<EP>(a, blockIdx.x); }
template <int EP>
__global__ __launch_bounds__(NTF) void tail1k_kernel(FinalizeArgs a) { tail1k_body<EP>(a); }

__device__ __forceinline__ void fin_op(const KOp& op, int bx) {
  switch (op.kind) {
    case K_FIN1K:
      if (op.variant == 1) fin1k_body<1>(op.u.fin);
      else if (op.variant == 2) fin1k_body<2>(op.u.fin);
      else fin1k_body<4>(op.u.fin);
      break;
    case K_GRAM1K:
      if (op.variant == 1) gram1k_chunk_body<1>(op.u.fin, bx);
      else if (op.variant == 2) gram1k_chunk_body<2>(op.u.fin, bx);
      else gram1k_chunk_body<4>(op.u.fin, bx);
      break;
    case K_TAIL1K:
      if (op.variant == 1) tail1k_body<1>(op.u.fin);
      else if (op.variant == 2) tail1k_body<2>(op.u.fin);
      else tail1k_body<4>(op.u.fin);
      break;
    default: break;
  }
}
// Persistent batched form of the 1024-thread finalize kernels.
__global__ __launch_bounds__(NTF) void fin_batch_kernel(const BItem* __restrict__ items, const int* __restrict__ grp,
                                                        const KOp* __restrict__ ops) {
  const int off = grp[0], n = grp[1];
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const BItem it = items[off + i];
    fin_op(ops[it.op], it.bx);
    __syncthreads();
  }
}

// Split-K sum of partial-MTTKRP partials: T(m, col0 + r) = sum over splits (in
// split order) of part[(sp*RP + r)*Mpad + m], one thread per output (coalesced along m).
template <typename TO>
__device__ __forceinline__ void pm_reduce_body(const ReduceArgs& ra, int bx) {
  const int64_t e = (int64_t)bx * NT + threadIdx.x;
  const int64_t total = ra.Mtot * ra.R;
  if (e >= total) return;
  const int r = (int)(e / ra.Mtot);
  const int64_t m = e - (int64_t)r * ra.Mtot;
  const double* p = ra.part + (size_t)r * ra.Mpad + m;
  const size_t st = (size_t)ra.RP * ra.Mpad;
  double s = 0.0;
  int sp = 0;
  for (; sp + 4 <= ra.nsplit; sp += 4) {
    const double v0 = p[(sp + 0) * st], v1 = p[(sp + 1) * st], v2 = p[(sp + 2) * st], v3 = p[(sp + 3) * st];
    s += v0;
    s += v1;
    s += v2;
    s += v3;
  }
  for (; sp < ra.nsplit; ++sp) s += p[sp * st];
  ((TO*)ra.T)[m + ra.Mtot * (int64_t)(ra.col0 + r)] = (TO)s;
}
template <typename TO>
__global__ __launch_bounds__(NT) void pm_reduce_kernel(ReduceArgs ra) {
  pm_reduce_body<TO>(ra, blockIdx.x);
}

// Persistent batched forms of the small kernels of the iteration: one kernel
// per kind (and per register variant of the update), so that each runs at its
// own occupancy rather than at that of the most register-hungry one.
template <int KIND, int VAR>
__device__ __forceinline__ void small_op(const KOp& op, int bx, int by) {
  if constexpr (KIND == K_PM_REDUCE) {
    if (op.variant) pm_reduce_body<double>(op.u.red, bx);
    else pm_reduce_body<float>(op.u.red, bx);
  } else if constexpr (KIND == K_MTTV_TRAIL) {
    if (op.variant) mttv_trail_body<double>(op.u.mt, bx, by);
    else mttv_trail_body<float>(op.u.mt, bx, by);
  } else if constexpr (KIND == K_MTTV_LEAD) {
    switch (op.variant) {
      case 41: mttv_lead_body<4, double>(op.u.mt, bx); break;
      case 40: mttv_lead_body<4, float>(op.u.mt, bx); break;
      case 81: mttv_lead_body<8, double>(op.u.mt, bx); break;
      case 80: mttv_lead_body<8, float>(op.u.mt, bx); break;
      case 161: mttv_lead_body<16, double>(op.u.mt, bx); break;
      case 160: mttv_lead_body<16, float>(op.u.mt, bx); break;
      case 321: mttv_lead_body<32, double>(op.u.mt, bx); break;
      case 320: mttv_lead_body<32, float>(op.u.mt, bx); break;
      case 641: mttv_lead_body<64, double>(op.u.mt, bx); break;
      default: mttv_lead_body<64, float>(op.u.mt, bx); break;
    }
  } else if constexpr (KIND == K_UPDATE) {
    if constexpr (VAR <= 2) update_body<VAR>(op.u.up, bx);
    else update_reg_body<VAR>(op.u.up, bx);
  } else if constexpr (KIND == K_FIN_FUSED) {
    finalize_fused_body(op.u.fin);
  } else if constexpr (KIND == K_GRAM_CHUNKS) {
    gram_chunks_body(op.u.fin, bx);
  } else if constexpr (KIND == K_FIN_TAIL) {
    finalize_tail_body(op.u.fin);
  }
}

template <int KIND, int VAR>
__global__ __launch_bounds__(NT) void small_items_kernel(const BItem* __restrict__ items, const int* __restrict__ grp,
                                                         const KOp* __restrict__ ops) {
  const int off = grp[0], n = grp[1];
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const BItem it = items[off + i];
    const KOp& op = ops[it.op];
    const unsigned b0 = (unsigned)it.bx * op.coarse, b1 = min(b0 + op.coarse, op.gx);
    for (unsigned b = b0; b < b1; ++b) {
      small_op<KIND, VAR>(op, (int)b, it.by);
      __syncthreads();  // LDS is reused by the next work-group's share
    }
  }
}

__global__ void init_model_kernel(const double* lam_in, const double* lam, double* lam_model,
                                  const double* G, double* S, int N, int R) {
  for (int k = threadIdx.x; k < R; k += blockDim.x) {
    double l = lam_in ? lam_in[k] : 1.0;
    for (int n = 0; n < N; ++n) l *= lam[(int64_t)n * R + k];
    lam_model[k] = l;
  }
  const int RR = R * R;
  for (int e = threadIdx.x; e < RR; e += blockDim.x) {
    double s = 1.0;
    for (int n = 1; n < N; ++n) s *= G[(int64_t)n * RR + e];
    S[e] = s;
  }
}

__global__ void normalize_out_kernel(float* W, int64_t I, int R, const double* lam) {
  const int64_t n = I * R;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(e / I);
    const double l = lam[k];
    W[e] = l > 0.0 ? (float)((double)W[e] / l) : 0.f;
  }
}

inline unsigned grid_for(int64_t n, int threads, unsigned cap = 65535u * 32u) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > (int64_t)cap) g = cap;
  return (unsigned)g;
}

}  // namespace

int norm_sq_blocks(int64_t n) {
  // 64 values per thread at least; at most 256 groups, one per CU of this chip:
  // measured on a 1 GiB FP32 tensor, 256 groups stream ||X||^2 in about half
  // the time of 1024 (more groups per CU interleave more distant addresses).
  // A fixed count keeps the summation order, and so the result, the same on
  // every device.
  int64_t b = (n + NT * 64 - 1) / (NT * 64);
  if (b < 1) b = 1;
  if (b > 256) b = 256;
  return (int)b;
}

hipError_t norm_sq_launch(const void* X, int dtype, int64_t n, double* out, double* partial,
                          unsigned* counter, int nblocks, hipStream_t st) {
  dim3 g(nblocks), b(NT);
  switch (dtype) {
    case NNCP_F32: hipLaunchKernelGGL(norm_sq_kernel<float>, g, b, 0, st, (const float*)X, n, out, partial, counter); break;
    case NNCP_BF16: hipLaunchKernelGGL(norm_sq_kernel<__bf16>, g, b, 0, st, (const __bf16*)X, n, out, partial, counter); break;
    case NNCP_F16: hipLaunchKernelGGL(norm_sq_kernel<_Float16>, g, b, 0, st, (const _Float16*)X, n, out, partial, counter); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t quantize_launch(const float* src, void* dst, int dtype, int64_t n, hipStream_t st) {
  dim3 g(grid_for(n, NT * 4, 8192)), b(NT);
  if (dtype == NNCP_BF16) hipLaunchKernelGGL(quantize_kernel<__bf16>, g, b, 0, st, src, (__bf16*)dst, n);
  else if (dtype == NNCP_F16) hipLaunchKernelGGL(quantize_kernel<_Float16>, g, b, 0, st, src, (_Float16*)dst, n);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t fill_u32_launch(unsigned* p, int64_t n, unsigned v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n, NT)), dim3(NT), 0, st, p, n, v);
  return hipGetLastError();
}
hipError_t fill_f64_launch(double* p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_f64_kernel, dim3(grid_for(n, NT)), dim3(NT), 0, st, p, n, v);
  return hipGetLastError();
}
hipError_t widen_f32_launch(double* d, const float* s, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(widen_f32_kernel, dim3(grid_for(n, NT)), dim3(NT), 0, st, d, s, n);
  return hipGetLastError();
}
hipError_t copy_f64_launch(double* d, const double* s, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_f64_kernel, dim3(grid_for(n, NT)), dim3(NT), 0, st, d, s, n);
  return hipGetLastError();
}
hipError_t unit_lambda_launch(double* lam, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(unit_lambda_kernel, dim3(grid_for(n, NT)), dim3(NT), 0, st, lam, n);
  return hipGetLastError();
}

static hipError_t record_or_launch(const Sink& sk, int kind, int variant, unsigned gx, unsigned gy, size_t lds,
                                   const void* kernel, const void* arg_struct, size_t arg_bytes, int threads = NT) {
  if (sk.rec) {
    KOp op{};
    op.kind = kind;
    op.variant = variant;
    op.gx = gx;
    op.gy = gy;
    op.lds = (unsigned)lds;
    std::memcpy(&op.u, arg_struct, arg_bytes);
    return sink_record(sk, op);
  }
  void* args[] = {const_cast<void*>(arg_struct)};
  return hipLaunchKernel(kernel, dim3(gx, gy), dim3(threads), args, lds, sk.st);
}

hipError_t mttv_trail_launch(const MttvArgs& a, const Sink& sk) {
  if (a.Ia <= 0 || a.R <= 0) return hipSuccess;
  const void* k = a.t_f64 ? (const void*)mttv_trail_kernel<double> : (const void*)mttv_trail_kernel<float>;
  return record_or_launch(sk, K_MTTV_TRAIL, a.t_f64 ? 1 : 0, (unsigned)((a.Ia + 63) / 64), (unsigned)a.R, 0, k, &a,
                          sizeof(a));
}

hipError_t mttv_lead_launch(const MttvArgs& a, const Sink& sk) {
  const int64_t outputs = a.J * a.R;
  if (outputs <= 0) return hipSuccess;
  // lanes per output: about 8 elements of the contracted range per lane (at
  // least 4 lanes, at most a wave), so that short ranges still give each
  // work-group many outputs and each lane several independent loads
  int gs = 4;
  while (gs < 64 && gs * 8 < a.Ia) gs <<= 1;
  const unsigned blocks = (unsigned)((outputs * gs + NT - 1) / NT);
  const void* k = nullptr;
#define NNCP_LEAD(GSV) \
  k = a.t_f64 ? (const void*)mttv_lead_kernel<GSV, double> : (const void*)mttv_lead_kernel<GSV, float>;
  switch (gs) {
    case 4: NNCP_LEAD(4) break;
    case 8: NNCP_LEAD(8) break;
    case 16: NNCP_LEAD(16) break;
    case 32: NNCP_LEAD(32) break;
    default: NNCP_LEAD(64) break;
  }
#undef NNCP_LEAD
  return record_or_launch(sk, K_MTTV_LEAD, gs * 10 + (a.t_f64 ? 1 : 0), blocks, 1, 0, k, &a, sizeof(a));
}

hipError_t update_launch(const UpdateArgs& a, const Sink& sk) {
  if (a.I <= 0) return hipSuccess;
  const int rpb = NT / 64;
  const unsigned g = (unsigned)((a.I + rpb - 1) / rpb);
  if (a.R <= 64) {
    const int rb = a.R <= 16 ? 16 : (a.R <= 32 ? 32 : 64);
    const void* k = rb == 16 ? (const void*)update_reg_kernel<16>
                             : (rb == 32 ? (const void*)update_reg_kernel<32> : (const void*)update_reg_kernel<64>);
    return record_or_launch(sk, K_UPDATE, rb, g, 1, 0, k, &a, sizeof(a));
  }
  const size_t lds = ((size_t)a.R * a.R + a.R) * sizeof(double);
  const int vpl = a.R <= 64 ? 1 : 2;
  const void* k = vpl == 1 ? (const void*)update_kernel<1> : (const void*)update_kernel<2>;
  return record_or_launch(sk, K_UPDATE, vpl, g, 1, lds, k, &a, sizeof(a));
}

hipError_t pm_reduce_launch(const ReduceArgs& r, const Sink& sk) {
  const int64_t total = r.Mtot * r.R;
  if (total <= 0) return hipSuccess;
  const void* k = r.t_f64 ? (const void*)pm_reduce_kernel<double> : (const void*)pm_reduce_kernel<float>;
  return record_or_launch(sk, K_PM_REDUCE, r.t_f64 ? 1 : 0, (unsigned)((total + NT - 1) / NT), 1, 0, k, &r,
                          sizeof(r));
}

hipError_t mttv_trail_launch(const MttvArgs& a, hipStream_t st) {
  Sink sk;
  sk.st = st;
  return mttv_trail_launch(a, sk);
}
hipError_t mttv_lead_launch(const MttvArgs& a, hipStream_t st) {
  Sink sk;
  sk.st = st;
  return mttv_lead_launch(a, sk);
}
hipError_t update_launch(const UpdateArgs& a, hipStream_t st) {
  Sink sk;
  sk.st = st;
  return update_launch(a, sk);
}

hipError_t sink_record(const Sink& s, const KOp& op) {
  if (!s.rec) return hipErrorInvalidValue;
  try {
    KOp o = op;
    o.stage = 64 * s.mode + 4 * s.step + kslot(op.kind);
    static_cast<std::vector<KOp>*>(s.rec)->push_back(o);
  } catch (...) {
    return hipErrorOutOfMemory;
  }
  return hipSuccess;
}

const void* small_batch_kernel_ptr(int kind, int variant) {
  switch (kind) {
    case K_PM_REDUCE: return (const void*)small_items_kernel<K_PM_REDUCE, 0>;
    case K_MTTV_TRAIL: return (const void*)small_items_kernel<K_MTTV_TRAIL, 0>;
    case K_MTTV_LEAD: return (const void*)small_items_kernel<K_MTTV_LEAD, 0>;
    case K_UPDATE:
      switch (variant) {
        case 1: return (const void*)small_items_kernel<K_UPDATE, 1>;
        case 2: return (const void*)small_items_kernel<K_UPDATE, 2>;
        case 16: return (const void*)small_items_kernel<K_UPDATE, 16>;
        case 32: return (const void*)small_items_kernel<K_UPDATE, 32>;
        case 64: return (const void*)small_items_kernel<K_UPDATE, 64>;
        default: return nullptr;
      }
    case K_FIN_FUSED: return (const void*)small_items_kernel<K_FIN_FUSED, 0>;
    case K_GRAM_CHUNKS: return (const void*)small_items_kernel<K_GRAM_CHUNKS, 0>;
    case K_FIN_TAIL: return (const void*)small_items_kernel<K_FIN_TAIL, 0>;
    default: return nullptr;
  }
}
const void* fin_batch_kernel_ptr() {
  static bool attr = [] {
    (void)hipFuncSetAttribute((const void*)fin_batch_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)fin_batch_max_lds());
    (void)hipGetLastError();
    return true;
  }();
  (void)attr;
  return (const void*)fin_batch_kernel;
}
// The most dynamic LDS a 1024-thread Gram/finalize op of rank <= 64 uses.
size_t fin_batch_max_lds() {
  size_t m = 0;
  for (int R = 1; R <= kSmallMaxR; ++R) {
    const size_t b = (size_t)fin_work_doubles(R) * sizeof(double);
    if (b > m) m = b;
  }
  return m;
}

// Row chunks for the Gram: one group when the work is small (no second launch),
// otherwise chunks of about I_chunk x R4^2 = 2^20 (R <= 64: 1024-thread groups
// that compute only the upper triangle) or 2^19 (R > 64) products each, at most 64.
int finalize_chunks(int64_t I, int R, int* rows_per_chunk) {
  const int shift = R <= kSmallMaxR ? 20 : 19;
  const int64_t R4 = R <= kSmallMaxR ? gram_r4(R) : R;
  const int64_t work = I * R4 * R4;
  int64_t chunks = (work + (1ll << shift) - 1) >> shift;
  if (chunks > 64) chunks = 64;
  if (chunks > I) chunks = I;
  if (chunks < 1) chunks = 1;
  int64_t rpc = (I + chunks - 1) / chunks;
  if (rpc < 1) rpc = 1;
  chunks = (I + rpc - 1) / rpc;
  *rows_per_chunk = (int)rpc;
  return (int)chunks;
}

hipError_t finalize_launch(const FinalizeArgs& a, const Sink& sk) {
  const size_t RR = (size_t)a.R * a.R;
  if (a.R <= kSmallMaxR) {
    static bool attr = [] {
      const void* ks[] = {(const void*)fin1k_kernel<1>,        (const void*)fin1k_kernel<2>,
                          (const void*)fin1k_kernel<4>,        (const void*)gram1k_chunk_kernel<1>,
                          (const void*)gram1k_chunk_kernel<2>, (const void*)gram1k_chunk_kernel<4>};
      for (const void* k : ks)
        if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024) != hipSuccess)
          (void)hipGetLastError();
      return true;
    }();
    (void)attr;
    const int ep = fin_ep(a.R);
    const size_t lds = (size_t)fin_work_doubles(a.R) * sizeof(double);
    if (a.nchunks <= 1) {
      const void* k = ep == 1 ? (const void*)fin1k_kernel<1>
                              : (ep == 2 ? (const void*)fin1k_kernel<2> : (const void*)fin1k_kernel<4>);
      return record_or_launch(sk, K_FIN1K, ep, 1, 1, lds, k, &a, sizeof(a), NTF);
    }
    const void* kc = ep == 1 ? (const void*)gram1k_chunk_kernel<1>
                             : (ep == 2 ? (const void*)gram1k_chunk_kernel<2> : (const void*)gram1k_chunk_kernel<4>);
    hipError_t e = record_or_launch(sk, K_GRAM1K, ep, (unsigned)a.nchunks, 1, lds, kc, &a, sizeof(a), NTF);
    if (e != hipSuccess) return e;
    const void* kt = ep == 1 ? (const void*)tail1k_kernel<1>
                             : (ep == 2 ? (const void*)tail1k_kernel<2> : (const void*)tail1k_kernel<4>);
    return record_or_launch(sk, K_TAIL1K, ep, 1, 1, 0, kt, &a, sizeof(a), NTF);
  }
  size_t lds = (size_t)fin_sub_rows(a.R) * a.R * sizeof(double);
  const size_t need = (RR + 1) * sizeof(double);
  if (need > lds) lds = need;
  if (a.nchunks <= 1)
    return record_or_launch(sk, K_FIN_FUSED, 0, 1, 1, lds, (const void*)finalize_fused_kernel, &a, sizeof(a));
  hipError_t e = record_or_launch(sk, K_GRAM_CHUNKS, 0, (unsigned)a.nchunks, 1, lds,
                                  (const void*)gram_chunks_kernel, &a, sizeof(a));
  if (e != hipSuccess) return e;
  return record_or_launch(sk, K_FIN_TAIL, 0, 1, 1, lds, (const void*)finalize_tail_kernel, &a, sizeof(a));
}

hipError_t finalize_launch(const FinalizeArgs& a, hipStream_t st) {
  Sink sk;
  sk.st = st;
  return finalize_launch(a, sk);
}


hipError_t init_model_launch(const double* lam_in, double* lam, double* lam_model, const double* G,
                             double* S, int N, int R, hipStream_t st) {
  hipLaunchKernelGGL(init_model_kernel, dim3(1), dim3(NT), 0, st, lam_in, lam, lam_model, G, S, N, R);
  return hipGetLastError();
}

hipError_t normalize_out_launch(float* W, int64_t I, int R, double* lam_self, hipStream_t st) {
  const int64_t n = I * R;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(normalize_out_kernel, dim3(grid_for(n, NT, 4096)), dim3(NT), 0, st, W, I, R,
                     (const double*)lam_self);
  return hipGetLastError();
}

}  // namespace nncpk
