// Gram-Schmidt building blocks for the Arnoldi process on the preconditioned
// operator (Algorithm 1: h_ij = <w, v_i>, w <- w - v_i h_ij, h_{j+1,j} = ||w||,
// v_{j+1} = w / h_{j+1,j}), written as tall-skinny matrix-vector products over
// the device-resident basis V (column-major, leading dimension ldv):
//   project : h = V^H w          (GEMV with V^H; two-stage deterministic sum)
//   update  : w <- w - V h       (GEMV with V), optionally ||w||^2 on the fly
//   combine : x = V z            (the final f_m = V_m z_m)
//   normalize: v = w / ||w||
// Classical Gram-Schmidt applied twice is project + update, twice.
//
// Reductions never use floating-point atomics: every block writes its partial
// sums to a scratch array and a second kernel adds them in a fixed order, so
// results are bitwise reproducible from run to run.
#include <hip/hip_runtime.h>

#include "devmath.hpp"
#include "fa_internal.hpp"

namespace fa {

constexpr int kThreads = 256;
// rows per thread and columns per reduction round: from a sweep at n = 128^3
// over 1..64 columns (8 rows x 4 columns led for projections, 8 rows for
// updates, 5.5-6.8 TB/s once the basis has 8 or more columns)
constexpr int kRpt = 8;  // rows per thread in the GEMV sweeps
constexpr int kCb = 4;   // columns per reduction round in project

RedPlan red_plan(int64_t n) {
  RedPlan p;
  p.rows = kThreads * kRpt;
  p.nblk = (int)((n + p.rows - 1) / p.rows);
  return p;
}

template <typename T>
__device__ __forceinline__ T block_sum(T v, T* sh /* [4] */) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  T r = sh[0];
  r += sh[1];
  r += sh[2];
  r += sh[3];
  __syncthreads();
  return r;
}

// part[c * nblk + blk] = sum over the block's rows of conj(V[r, c]) w[r]
template <typename T>
__global__ __launch_bounds__(kThreads) void project_k(int64_t n, int ncols, const T* __restrict__ V,
                                                      int64_t ldv, const T* __restrict__ w,
                                                      T* __restrict__ part, int nblk) {
  __shared__ T red[kThreads / 64][kCb];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * (kThreads * kRpt) + tid;
  T wr[kRpt];
#pragma unroll
  for (int q = 0; q < kRpt; ++q) {
    const int64_t r = r0 + (int64_t)q * kThreads;
    wr[q] = (r < n) ? w[r] : zero(T{});
  }
  const bool full = r0 + (int64_t)(kRpt - 1) * kThreads < n;
  for (int c0 = 0; c0 < ncols; c0 += kCb) {
    T acc[kCb];
#pragma unroll
    for (int cc = 0; cc < kCb; ++cc) {
      acc[cc] = zero(T{});
      if (c0 + cc < ncols) {
        const T* col = V + (int64_t)(c0 + cc) * ldv + r0;
        if (full) {
#pragma unroll
          for (int q = 0; q < kRpt; ++q) acc[cc] = cmad(col[q * kThreads], wr[q], acc[cc]);
        } else {
#pragma unroll
          for (int q = 0; q < kRpt; ++q)
            if (r0 + (int64_t)q * kThreads < n) acc[cc] = cmad(col[q * kThreads], wr[q], acc[cc]);
        }
      }
    }
#pragma unroll
    for (int cc = 0; cc < kCb; ++cc) acc[cc] = wave_sum(acc[cc]);
    if (lane == 0) {
#pragma unroll
      for (int cc = 0; cc < kCb; ++cc) red[wv][cc] = acc[cc];
    }
    __syncthreads();
    if (tid < kCb && c0 + tid < ncols) {
      T s = red[0][tid];
      s += red[1][tid];
      s += red[2][tid];
      s += red[3][tid];
      part[(int64_t)(c0 + tid) * nblk + blockIdx.x] = s;
    }
    __syncthreads();
  }
}

// second stage: h[c] = sum_b part[c * nblk + b] in a fixed order; mode 1 also
// stores hsum[c] = h[c], mode 2 adds it (CGS2: H(:, j) = h1 + h2)
template <typename T>
__global__ __launch_bounds__(kThreads) void reduce_cols_k(int nblk, const T* __restrict__ part,
                                                          T* h, T* hsum, int mode) {
  __shared__ T sh[kThreads / 64];
  const int c = blockIdx.x;
  T s = zero(T{});
  for (int b = threadIdx.x; b < nblk; b += kThreads) s += part[(int64_t)c * nblk + b];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) {
    if (h) h[c] = s;
    if (mode == 1) hsum[c] = s;
    if (mode == 2) hsum[c] += s;
  }
}

// w[r] = ASSIGN ? sum_c V[r, c] h[c] : w[r] - sum_c V[r, c] h[c]; optional ||w||^2 partials
template <typename T, bool ASSIGN, bool NORM>
__global__ __launch_bounds__(kThreads) void update_k(int64_t n, int ncols, const T* __restrict__ V,
                                                     int64_t ldv, const T* __restrict__ h,
                                                     T* __restrict__ w,
                                                     double* __restrict__ part) {
  __shared__ double sh[kThreads / 64];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * (kThreads * kRpt) + tid;
  T acc[kRpt];
#pragma unroll
  for (int q = 0; q < kRpt; ++q) acc[q] = zero(T{});
  if (r0 + (int64_t)(kRpt - 1) * kThreads < n) {  // full block of rows
#pragma unroll 4
    for (int c = 0; c < ncols; ++c) {
      const T hc = h[c];
      const T* col = V + (int64_t)c * ldv + r0;
#pragma unroll
      for (int q = 0; q < kRpt; ++q) acc[q] = mad(col[q * kThreads], hc, acc[q]);
    }
  } else {
    for (int c = 0; c < ncols; ++c) {
      const T hc = h[c];
      const T* col = V + (int64_t)c * ldv;
#pragma unroll
      for (int q = 0; q < kRpt; ++q) {
        const int64_t r = r0 + (int64_t)q * kThreads;
        if (r < n) acc[q] = mad(col[r], hc, acc[q]);
      }
    }
  }
  double s2 = 0.0;
#pragma unroll
  for (int q = 0; q < kRpt; ++q) {
    const int64_t r = r0 + (int64_t)q * kThreads;
    if (r < n) {
      const T nw = ASSIGN ? acc[q] : w[r] - acc[q];
      w[r] = nw;
      if (NORM) s2 += abs2(nw);
    }
  }
  if (NORM) {
    s2 = block_sum(s2, sh);
    if (tid == 0) part[blockIdx.x] = s2;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void normalize_k(int64_t n, const T* w,
                                                        const double* __restrict__ nrm2,
                                                        T* out, T* hout) {
  const double nr = sqrt(nrm2[0]);
  const double inv = nr > 0.0 ? 1.0 / nr : 0.0;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i == 0 && hout) {
    T hv = zero(T{});
    *reinterpret_cast<double*>(&hv) = nr;
    *hout = hv;
  }
  if (i < n) out[i] = inv * w[i];
}

__device__ __forceinline__ double scale_val(double a_re, double, double x) { return a_re * x; }
__device__ __forceinline__ cplx scale_val(double a_re, double a_im, cplx x) {
  return cplx{a_re * x.x - a_im * x.y, a_re * x.y + a_im * x.x};
}
template <typename T>
__global__ __launch_bounds__(kThreads) void scale_k(int64_t n, double a_re, double a_im,
                                                    const T* x, T* y) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) y[i] = scale_val(a_re, a_im, x[i]);
}

// One step of the recurrence of the least-squares polynomial (Sec. 5.3),
// after the chain launch has formed t = (A w_{k-1} - h_{k-1,k-1} w_{k-1}) / h_{k,k-1}
// in column k of W:
//   w_k = t + sum_{i < k-1} g_i w_i        (g_i = -h_{i,k-1} / h_{k,k-1})
//   out = (k == 1 ? a_0 w_0 : out) + a_k w_k
// w_k is stored back only if a later step reads it.
__device__ __forceinline__ double coef_of(const LsCoef& g, int i, double) { return g.re[i]; }
__device__ __forceinline__ cplx coef_of(const LsCoef& g, int i, cplx) { return cplx{g.re[i], g.im[i]}; }
__device__ __forceinline__ double cval(double re, double, double) { return re; }
__device__ __forceinline__ cplx cval(double re, double im, cplx) { return cplx{re, im}; }

template <typename T, bool FIRST, bool KEEP>
__global__ __launch_bounds__(kThreads) void ls_step_k(int64_t n, int k, T* __restrict__ W,
                                                      int64_t ldv, LsCoef g, T* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (r >= n) return;
  T w = W[(int64_t)k * ldv + r];
  for (int i = 0; i + 1 < k; ++i) w = mad(coef_of(g, i, T{}), W[(int64_t)i * ldv + r], w);
  if (KEEP) W[(int64_t)k * ldv + r] = w;
  const T o = FIRST ? cval(g.a0_re, g.a0_im, T{}) * W[r] : out[r];
  out[r] = mad(cval(g.ak_re, g.ak_im, T{}), w, o);
}

hipError_t launch_ls_step(int dtype, int64_t n, int k, void* W, int64_t ldv, const LsCoef& g,
                          bool keep, void* out, hipStream_t s) {
  const int grid = (int)((n + kThreads - 1) / kThreads);
  const bool first = k == 1;
#define FA_LS(T, F, K)                                                                      \
  ls_step_k<T, F, K><<<grid, kThreads, 0, s>>>(n, k, (T*)W, ldv, g, (T*)out)
  if (dtype == FA_C128) {
    if (first) { if (keep) FA_LS(cplx, true, true); else FA_LS(cplx, true, false); }
    else { if (keep) FA_LS(cplx, false, true); else FA_LS(cplx, false, false); }
  } else {
    if (first) { if (keep) FA_LS(double, true, true); else FA_LS(double, true, false); }
    else { if (keep) FA_LS(double, false, true); else FA_LS(double, false, false); }
  }
#undef FA_LS
  return hipGetLastError();
}

// --------------------------------------------------------------------------
template <typename T>
static hipError_t project_t(int64_t n, int ncols, const T* V, int64_t ldv, const T* w, T* part,
                            T* h, T* hsum, int mode, hipStream_t s) {
  const RedPlan p = red_plan(n);
  project_k<T><<<p.nblk, kThreads, 0, s>>>(n, ncols, V, ldv, w, part, p.nblk);
  reduce_cols_k<T><<<ncols, kThreads, 0, s>>>(p.nblk, part, h, hsum, mode);
  return hipGetLastError();
}

hipError_t launch_project(int dtype, int64_t n, int ncols, const void* V, int64_t ldv,
                          const void* w, void* part, void* h, void* hsum, int hsum_mode,
                          hipStream_t s) {
  if (ncols <= 0) return hipSuccess;
  if (dtype == FA_C128)
    return project_t<cplx>(n, ncols, (const cplx*)V, ldv, (const cplx*)w, (cplx*)part,
                           (cplx*)h, (cplx*)hsum, hsum_mode, s);
  return project_t<double>(n, ncols, (const double*)V, ldv, (const double*)w, (double*)part,
                           (double*)h, (double*)hsum, hsum_mode, s);
}

template <typename T>
static hipError_t update_t(int64_t n, int ncols, const T* V, int64_t ldv, const T* h, T* w,
                           void* part, double* nrm2, hipStream_t s) {
  const RedPlan p = red_plan(n);
  if (nrm2) {
    update_k<T, false, true><<<p.nblk, kThreads, 0, s>>>(n, ncols, V, ldv, h, w, (double*)part);
    reduce_cols_k<double><<<1, kThreads, 0, s>>>(p.nblk, (const double*)part, nrm2, nullptr, 0);
  } else {
    update_k<T, false, false><<<p.nblk, kThreads, 0, s>>>(n, ncols, V, ldv, h, w, nullptr);
  }
  return hipGetLastError();
}

hipError_t launch_update(int dtype, int64_t n, int ncols, const void* V, int64_t ldv,
                         const void* h, void* w, void* part, double* nrm2, hipStream_t s) {
  if (dtype == FA_C128)
    return update_t<cplx>(n, ncols, (const cplx*)V, ldv, (const cplx*)h, (cplx*)w, part, nrm2, s);
  return update_t<double>(n, ncols, (const double*)V, ldv, (const double*)h, (double*)w, part,
                          nrm2, s);
}

hipError_t launch_combine(int dtype, int64_t n, int ncols, const void* V, int64_t ldv,
                          const void* z, void* x, hipStream_t s) {
  const RedPlan p = red_plan(n);
  if (dtype == FA_C128)
    update_k<cplx, true, false><<<p.nblk, kThreads, 0, s>>>(n, ncols, (const cplx*)V, ldv,
                                                            (const cplx*)z, (cplx*)x, nullptr);
  else
    update_k<double, true, false><<<p.nblk, kThreads, 0, s>>>(n, ncols, (const double*)V, ldv,
                                                              (const double*)z, (double*)x,
                                                              nullptr);
  return hipGetLastError();
}

hipError_t launch_normalize(int dtype, int64_t n, const void* w, const double* nrm2, void* out,
                            void* hout, hipStream_t s) {
  const int grid = (int)((n + kThreads - 1) / kThreads);
  if (dtype == FA_C128)
    normalize_k<cplx><<<grid, kThreads, 0, s>>>(n, (const cplx*)w, nrm2, (cplx*)out, (cplx*)hout);
  else
    normalize_k<double><<<grid, kThreads, 0, s>>>(n, (const double*)w, nrm2, (double*)out,
                                                  (double*)hout);
  return hipGetLastError();
}

__global__ __launch_bounds__(kThreads) void to_f32_k(int64_t n, const double* __restrict__ x,
                                                     float* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}

hipError_t launch_to_f32(int64_t n, const double* x, float* y, hipStream_t s) {
  const int grid = (int)((n + kThreads - 1) / kThreads);
  to_f32_k<<<grid, kThreads, 0, s>>>(n, x, y);
  return hipGetLastError();
}

hipError_t launch_scale(int dtype, int64_t n, cd a, const void* x, void* y, hipStream_t s) {
  const int grid = (int)((n + kThreads - 1) / kThreads);
  if (dtype == FA_C128)
    scale_k<cplx><<<grid, kThreads, 0, s>>>(n, a.real(), a.imag(), (const cplx*)x, (cplx*)y);
  else
    scale_k<double><<<grid, kThreads, 0, s>>>(n, a.real(), a.imag(), (const double*)x, (double*)y);
  return hipGetLastError();
}

}  // namespace fa
