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

// The projections on complex vectors reduce 2 columns per round instead of
// 4: with 4 columns of two complex vectors the round's loads and sums held
// 146 registers (three waves per SIMD) and the two-vector sweep ran at
// 3.45 TB/s on the 16^4 lattice; measured over rows per thread {2, 4, 8}
// x columns per round {1, 2, 3, 4} (2048 rows per workgroup), 8 rows and 2
// columns reach 4.7 TB/s at bases of 64 to 191 vectors.  Their workgroups
// are one wave (512 rows): 2048-row workgroups left a 16^4 vector (786,432
// entries) 384 workgroups, one and a half per CU, and the plain 16^4 solve
// (m = 192) takes 4.5 % less time with 1,536 (1,024-row workgroups: 3 %).
#ifndef FA_PROJ_CPLX_RPT
#define FA_PROJ_CPLX_RPT 8
#endif
#ifndef FA_PROJ_CPLX_CB
#define FA_PROJ_CPLX_CB 2
#endif
#ifndef FA_PROJ_CPLX_NTH
#define FA_PROJ_CPLX_NTH 64
#endif
template <typename T>
constexpr int proj_rpt() {
  return sizeof(T) == 16 ? FA_PROJ_CPLX_RPT : kRpt;
}
// columns per reduction round of the projections
template <typename T>
constexpr int proj_cb() {
  return sizeof(T) == 16 ? FA_PROJ_CPLX_CB : kCb;
}
// threads per workgroup of the projections (the kernels' default)
template <typename T>
constexpr int proj_threads() {
  return sizeof(T) == 16 ? FA_PROJ_CPLX_NTH : kThreads * kRpt / proj_rpt<T>();
}
// Real projections of vectors of at least 512 x 4096 entries run 512-thread
// workgroups (4096 rows), still two per CU: half the partial sums for the
// one-workgroup finish of the delayed CGS2 to read (128^3: 2 (j + 1) x 512);
// the plain 128^3 solve (m = 448) took 2 % less time, the degree-16 one
// 0.6 %.  Smaller vectors keep 256 threads: at n = 281,903 the wider
// workgroups left 69 of them and the solves ran 8-11 % slower.
constexpr int kProjWide = 2 * kThreads;
template <typename T>
static int proj_nth(int64_t n) {
  if (sizeof(T) == 16) return FA_PROJ_CPLX_NTH;
  return n >= (int64_t)512 * kProjWide * kRpt ? kProjWide : proj_threads<T>();
}

RedPlan red_plan(int64_t n) {
  RedPlan p;
  p.threads = kThreads;
  p.rows = kThreads * kRpt;
  p.nblk = (int)((n + p.rows - 1) / p.rows);
  return p;
}
// the projections' first stage (rows per workgroup of project_k / project2_k)
template <typename T>
static RedPlan proj_plan(int64_t n) {
  RedPlan p;
  p.threads = proj_nth<T>(n);
  p.rows = p.threads * proj_rpt<T>();
  p.nblk = (int)((n + p.rows - 1) / p.rows);
  return p;
}
int proj_nblk(int64_t n, int dtype) {
  return dtype == FA_C128 ? proj_plan<cplx>(n).nblk : proj_plan<double>(n).nblk;
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
template <typename T, int RPT = proj_rpt<T>(), int NTH = proj_threads<T>(), int CB = proj_cb<T>()>
__global__ __launch_bounds__(NTH) void project_k(int64_t n, int ncols, const T* __restrict__ V,
                                                      int64_t ldv, const T* __restrict__ w,
                                                      T* __restrict__ part, int nblk) {
  __shared__ T red[NTH / 64][CB];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * (NTH * RPT) + tid;
  T wr[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t r = r0 + (int64_t)q * NTH;
    wr[q] = (r < n) ? w[r] : zero(T{});
  }
  const bool full = r0 + (int64_t)(RPT - 1) * NTH < n;
  for (int c0 = 0; c0 < ncols; c0 += CB) {
    T acc[CB];
#pragma unroll
    for (int cc = 0; cc < CB; ++cc) {
      acc[cc] = zero(T{});
      if (c0 + cc < ncols) {
        const T* col = V + (int64_t)(c0 + cc) * ldv + r0;
        if (full) {
#pragma unroll
          for (int q = 0; q < RPT; ++q) acc[cc] = cmad(col[q * NTH], wr[q], acc[cc]);
        } else {
#pragma unroll
          for (int q = 0; q < RPT; ++q)
            if (r0 + (int64_t)q * NTH < n) acc[cc] = cmad(col[q * NTH], wr[q], acc[cc]);
        }
      }
    }
#pragma unroll
    for (int cc = 0; cc < CB; ++cc) acc[cc] = wave_sum(acc[cc]);
    if (lane == 0) {
#pragma unroll
      for (int cc = 0; cc < CB; ++cc) red[wv][cc] = acc[cc];
    }
    __syncthreads();
    if (tid < CB && c0 + tid < ncols) {
      T s = red[0][tid];
#pragma unroll
      for (int w = 1; w < NTH / 64; ++w) s += red[w][tid];
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
// CGS2 with the reorthogonalization delayed by one step (one sweep of
// projections and one sweep of updates per Arnoldi step):
//   project2 : S[2c + r] = V_c^H w_r for c < ncols and the two vectors
//              w_0 = u_j (the once-orthogonalized vector, also column j of V)
//              and w_1 = z = Op u_j
//   dcgs2_coef : finishes column j - 1 of H with the second-pass
//              coefficients s = Q_j^H u_j and nu = ||u_j - Q_j s||, and forms
//              the first-pass column j from p = Q_j^H z (one workgroup)
//   update2  : q_j = (u_j - Q_j s) / nu (in place of u_j) and
//              u_{j+1} = (z - Q_j p - q_j gamma) / nu (in place of z)
// --------------------------------------------------------------------------
template <typename T, int RPT = proj_rpt<T>(), int NTH = proj_threads<T>(), int CB = proj_cb<T>()>
__global__ __launch_bounds__(NTH) void project2_k(int64_t n, int ncols,
                                                       const T* __restrict__ V, int64_t ldv,
                                                       const T* __restrict__ w0,
                                                       const T* __restrict__ w1,
                                                       T* __restrict__ part, int nblk) {
  __shared__ T red[NTH / 64][2 * CB];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * (NTH * RPT) + tid;
  T a0[RPT], a1[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int64_t r = r0 + (int64_t)q * NTH;
    a0[q] = (r < n) ? w0[r] : zero(T{});
    a1[q] = (r < n) ? w1[r] : zero(T{});
  }
  const bool full = r0 + (int64_t)(RPT - 1) * NTH < n;
  for (int c0 = 0; c0 < ncols; c0 += CB) {
    T acc[2 * CB];
#pragma unroll
    for (int cc = 0; cc < CB; ++cc) {
      acc[2 * cc] = acc[2 * cc + 1] = zero(T{});
      if (c0 + cc < ncols) {
        const T* col = V + (int64_t)(c0 + cc) * ldv + r0;
        if (full) {  // no row checks: all loads of the round issue together
#pragma unroll
          for (int q = 0; q < RPT; ++q) {
            const T v = col[q * NTH];
            acc[2 * cc] = cmad(v, a0[q], acc[2 * cc]);
            acc[2 * cc + 1] = cmad(v, a1[q], acc[2 * cc + 1]);
          }
        } else {
#pragma unroll
          for (int q = 0; q < RPT; ++q) {
            if (r0 + (int64_t)q * NTH < n) {
              const T v = col[q * NTH];
              acc[2 * cc] = cmad(v, a0[q], acc[2 * cc]);
              acc[2 * cc + 1] = cmad(v, a1[q], acc[2 * cc + 1]);
            }
          }
        }
      }
    }
#pragma unroll
    for (int e = 0; e < 2 * CB; ++e) acc[e] = wave_sum(acc[e]);
    if (lane == 0) {
#pragma unroll
      for (int e = 0; e < 2 * CB; ++e) red[wv][e] = acc[e];
    }
    __syncthreads();
    if (tid < 2 * CB && c0 + tid / 2 < ncols) {
      T t = red[0][tid];
#pragma unroll
      for (int w = 1; w < NTH / 64; ++w) t += red[w][tid];
      part[(int64_t)(2 * c0 + tid) * nblk + blockIdx.x] = t;
    }
    __syncthreads();
  }
}

__device__ __forceinline__ double re_of(double a) { return a; }
__device__ __forceinline__ double re_of(cplx a) { return a.x; }
__device__ __forceinline__ double mk_real(double a, double) { return a; }
__device__ __forceinline__ cplx mk_real(double a, cplx) { return cplx{a, 0.0}; }
__device__ __forceinline__ double div_real(double a, double d) { return a / d; }
__device__ __forceinline__ cplx div_real(cplx a, double d) { return cplx{a.x / d, a.y / d}; }

// S (2 (j + 1) entries, see project2), H column-major (ldh), j >= 1.
// Writes cs = s, cp = p (j entries each), sc[0] = 1 / nu, sc[1] = gamma.
template <typename T>
__global__ __launch_bounds__(kThreads) void dcgs2_coef_k(int j, const T* __restrict__ S, T* H,
                                                         int64_t ldh, T* __restrict__ cs,
                                                         T* __restrict__ cp,
                                                         T* __restrict__ sc) {
  __shared__ double shd[kThreads / 64];
  __shared__ T sht[kThreads / 64];
  __shared__ double s_nu;
  __shared__ T s_gam;
  const int tid = threadIdx.x;
  // ||s||^2 and s^H p
  double ss = 0.0;
  T sp = zero(T{});
  for (int i = tid; i < j; i += kThreads) {
    ss += abs2(S[2 * i]);
    sp = cmad(S[2 * i], S[2 * i + 1], sp);
  }
  ss = block_sum(ss, shd);
  sp = block_sum(sp, sht);
  if (tid == 0) {
    const double alpha = re_of(S[2 * j]);
    const double nu2 = alpha - ss;
    const double nu = nu2 > 0.0 ? sqrt(nu2) : 0.0;
    s_nu = nu;
    s_gam = div_real(S[2 * j + 1] - sp, nu);
    sc[0] = mk_real(nu > 0.0 ? 1.0 / nu : 0.0, T{});
    sc[1] = s_gam;
  }
  // finish column j - 1: H(0:j, j-1) += s, H(j, j-1) = nu
  for (int i = tid; i < j; i += kThreads) {
    H[(int64_t)(j - 1) * ldh + i] += S[2 * i];
    cs[i] = S[2 * i];
    cp[i] = S[2 * i + 1];
  }
  if (tid == 0) H[(int64_t)(j - 1) * ldh + j] = mk_real(s_nu, T{});
}

// first-pass column j of H: (Q_{j+1}^H z - Hbar s) / nu with Hbar = H(0:j,
// 0:j-1) (column j - 1 finished by dcgs2_coef_k).  64 rows per workgroup
// (one per lane); the four waves take every fourth column and their partial
// sums are added in LDS in a fixed order.
template <typename T>
__global__ __launch_bounds__(kThreads) void dcgs2_col_k(int j, const T* __restrict__ S, T* H,
                                                        int64_t ldh, const T* __restrict__ sc) {
  __shared__ T part[kThreads / 64][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  T t = zero(T{});
  if (i <= j) {
#pragma unroll 4
    for (int c = max(0, i - 1) + wv; c < j; c += 4) t = mad(H[(int64_t)c * ldh + i], S[2 * c], t);
  }
  part[wv][lane] = t;
  __syncthreads();
  if (wv == 0 && i <= j) {
    T tt = part[0][lane];
    tt += part[1][lane];
    tt += part[2][lane];
    tt += part[3][lane];
    const double inv = re_of(sc[0]);
    const T top = (i < j) ? S[2 * i + 1] : sc[1];
    H[(int64_t)j * ldh + i] = mk_real(inv, T{}) * (top - tt);
  }
}

// The three small steps between the two sweeps of a delayed-CGS2 step in
// one 1024-thread workgroup (one launch instead of three):
//   1. S[c] = sum_b part[c * nblk + b] for the 2 (j + 1) projections (wave w
//      takes columns w, w + 16, ..; lanes stride the partials, then a
//      fixed-order wave reduction), kept in LDS;
//   2. the coefficients: nu, gamma, cs = s, cp = p and the finished column
//      j - 1 of H (as dcgs2_coef_k);
//   3. the first-pass column j of H (as dcgs2_col_k): rows in blocks of 64
//      lanes, the 16 waves take every 16th column, partial sums added in
//      LDS in a fixed order.
// Every sum is in a fixed order: the result does not depend on timing.
constexpr int kFinThreads = 1024;
template <typename T>
__global__ __launch_bounds__(kFinThreads) void dcgs2_finish_k(int j, int nblk,
                                                              const T* __restrict__ part, T* H,
                                                              int64_t ldh, T* __restrict__ cs,
                                                              T* __restrict__ cp,
                                                              T* __restrict__ sc) {
  extern __shared__ unsigned char fin_lds[];
  T* S = reinterpret_cast<T*>(fin_lds);  // 2 (j + 1) entries
  __shared__ T colpart[kFinThreads / 64][64];
  __shared__ double s_nu;
  __shared__ T s_gam;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr int NW = kFinThreads / 64;
  // 1. the projections
  for (int c = wv; c < 2 * (j + 1); c += NW) {
    T a = zero(T{});
    // unrolled so that several loads are in flight before their adds (the
    // adds keep their order)
#pragma unroll 8
    for (int b = lane; b < nblk; b += 64) a += part[(int64_t)c * nblk + b];
    a = wave_sum(a);
    if (lane == 0) S[c] = a;
  }
  __syncthreads();
  // 2. the coefficients (one wave)
  if (wv == 0) {
    double ss = 0.0;
    T sp = zero(T{});
    for (int i = lane; i < j; i += 64) {
      ss += abs2(S[2 * i]);
      sp = cmad(S[2 * i], S[2 * i + 1], sp);
    }
    ss = wave_sum(ss);
    sp = wave_sum(sp);
    if (lane == 0) {
      const double alpha = re_of(S[2 * j]);
      const double nu2 = alpha - ss;
      const double nu = nu2 > 0.0 ? sqrt(nu2) : 0.0;
      s_nu = nu;
      s_gam = div_real(S[2 * j + 1] - sp, nu);
      sc[0] = mk_real(nu > 0.0 ? 1.0 / nu : 0.0, T{});
      sc[1] = s_gam;
      H[(int64_t)(j - 1) * ldh + j] = mk_real(nu, T{});
    }
  }
  for (int i = tid; i < j; i += kFinThreads) {
    H[(int64_t)(j - 1) * ldh + i] += S[2 * i];
    cs[i] = S[2 * i];
    cp[i] = S[2 * i + 1];
  }
  __syncthreads();  // column j - 1 of H and s_nu, s_gam visible to the block
  // 3. the first-pass column j: (Q_{j+1}^H z - Hbar s) / nu
  const double inv = s_nu > 0.0 ? 1.0 / s_nu : 0.0;
  for (int i0 = 0; i0 <= j; i0 += 64) {
    const int i = i0 + lane;
    T t = zero(T{});
    if (i <= j) {
#pragma unroll 4
      for (int c = max(0, i - 1) + wv; c < j; c += NW) t = mad(H[(int64_t)c * ldh + i], S[2 * c], t);
    }
    colpart[wv][lane] = t;
    __syncthreads();
    if (wv == 0 && i <= j) {
      T tt = colpart[0][lane];
#pragma unroll
      for (int w = 1; w < NW; ++w) tt += colpart[w][lane];
      const T top = (i < j) ? S[2 * i + 1] : s_gam;
      H[(int64_t)j * ldh + i] = mk_real(inv, T{}) * (top - tt);
    }
    __syncthreads();
  }
}

// The device side of a convergence check: copies na doubles a -> ha and nb
// doubles b -> hb, where ha and hb are page-locked, coherent host memory,
// then stores `seq` into the host flag once every copied value is visible
// to the host (each thread fences at system scope before the barrier that
// precedes the flag's release store).  One workgroup.
__global__ __launch_bounds__(1024) void check_export_k(const double* __restrict__ a, int64_t na,
                                                       double* ha, const double* __restrict__ b,
                                                       int64_t nb, double* hb, int* flag,
                                                       int seq) {
  for (int64_t i = threadIdx.x; i < na; i += 1024) ha[i] = a[i];
  for (int64_t i = threadIdx.x; i < nb; i += 1024) hb[i] = b[i];
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

hipError_t launch_check_export(const double* a, int64_t na, double* ha, const double* b,
                               int64_t nb, double* hb, int* flag, int seq, hipStream_t s) {
  check_export_k<<<1, 1024, 0, s>>>(a, na, ha, b, nb, hb, flag, seq);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(kThreads) void update2_k(int64_t n, int ncols, const T* __restrict__ V,
                                                      int64_t ldv, const T* __restrict__ cs,
                                                      const T* __restrict__ cp,
                                                      const T* __restrict__ sc, T* u, T* z) {
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * (kThreads * kRpt) + tid;
  T as[kRpt], ap[kRpt];
#pragma unroll
  for (int q = 0; q < kRpt; ++q) as[q] = ap[q] = zero(T{});
  if (r0 + (int64_t)(kRpt - 1) * kThreads < n) {  // full block of rows
#pragma unroll 4
    for (int c = 0; c < ncols; ++c) {
      const T hs = cs[c], hp = cp[c];
      const T* col = V + (int64_t)c * ldv + r0;
#pragma unroll
      for (int q = 0; q < kRpt; ++q) {
        const T v = col[q * kThreads];
        as[q] = mad(v, hs, as[q]);
        ap[q] = mad(v, hp, ap[q]);
      }
    }
  } else {
    for (int c = 0; c < ncols; ++c) {
      const T hs = cs[c], hp = cp[c];
      const T* col = V + (int64_t)c * ldv;
#pragma unroll
      for (int q = 0; q < kRpt; ++q) {
        const int64_t r = r0 + (int64_t)q * kThreads;
        if (r < n) {
          const T v = col[r];
          as[q] = mad(v, hs, as[q]);
          ap[q] = mad(v, hp, ap[q]);
        }
      }
    }
  }
  const double inv = re_of(sc[0]);
  const T gam = sc[1];
#pragma unroll
  for (int q = 0; q < kRpt; ++q) {
    const int64_t r = r0 + (int64_t)q * kThreads;
    if (r < n) {
      const T qv = mk_real(inv, T{}) * (u[r] - as[q]);
      u[r] = qv;
      z[r] = mk_real(inv, T{}) * (z[r] - ap[q] - qv * gam);
    }
  }
}

hipError_t launch_dcgs2(int dtype, int64_t n, int j, const void* V, int64_t ldv, void* part,
                        void* S, void* H, int64_t ldh, void* coef, hipStream_t s, int stage) {
  const bool proj = stage != kDcgs2Update, upd = stage != kDcgs2Project;
  const RedPlan p = red_plan(n);
  const RedPlan pp = dtype == FA_C128 ? proj_plan<cplx>(n) : proj_plan<double>(n);
  const size_t es = dtype == FA_C128 ? 16 : 8;
  void* u = (char*)V + (size_t)j * ldv * es;
  void* z = (char*)V + (size_t)(j + 1) * ldv * es;
  char* cs = (char*)coef;
  char* cp = cs + (size_t)j * es;
  char* sc = cp + (size_t)j * es;
  // one launch up to j = 32, else the three kernels: the one workgroup's
  // work grows linearly in j (8.8 us at j = 20, 14.4 at 32, 75 at 158 on the
  // 128^3 grid), the three kernels' stays near 15 us.  The one workgroup
  // also reads all 2 (j + 1) x nblk partial sums, so large vectors (many
  // first-stage blocks, e.g. 49,152 for a 64 x 32^3 lattice) take the three
  // kernels, whose partial sums are read by 2 (j + 1) workgroups
  const size_t lds = 2 * (size_t)(j + 1) * es;
  const bool fused = lds <= 32768 && j <= 32 && 2 * (int64_t)(j + 1) * pp.nblk <= (1 << 17);
  if (dtype == FA_C128) {
    if (proj)
      project2_k<cplx><<<pp.nblk, proj_threads<cplx>(), 0, s>>>(
          n, j + 1, (const cplx*)V, ldv, (const cplx*)u, (const cplx*)z, (cplx*)part, pp.nblk);
    if (proj && fused) {
      dcgs2_finish_k<cplx><<<1, kFinThreads, lds, s>>>(j, pp.nblk, (const cplx*)part, (cplx*)H,
                                                      ldh, (cplx*)cs, (cplx*)cp, (cplx*)sc);
    } else if (proj) {
      reduce_cols_k<cplx><<<2 * (j + 1), kThreads, 0, s>>>(pp.nblk, (const cplx*)part, (cplx*)S,
                                                           nullptr, 0);
      dcgs2_coef_k<cplx><<<1, kThreads, 0, s>>>(j, (const cplx*)S, (cplx*)H, ldh, (cplx*)cs,
                                                (cplx*)cp, (cplx*)sc);
      dcgs2_col_k<cplx><<<(j + 64) / 64, kThreads, 0, s>>>(j, (const cplx*)S, (cplx*)H, ldh,
                                                           (const cplx*)sc);
    }
    if (upd)
      update2_k<cplx><<<p.nblk, kThreads, 0, s>>>(n, j, (const cplx*)V, ldv, (const cplx*)cs,
                                                (const cplx*)cp, (const cplx*)sc, (cplx*)u,
                                                (cplx*)z);
  } else {
    if (proj && pp.threads == kProjWide)
      project2_k<double, kRpt, kProjWide><<<pp.nblk, kProjWide, 0, s>>>(
          n, j + 1, (const double*)V, ldv, (const double*)u, (const double*)z, (double*)part,
          pp.nblk);
    else if (proj)
      project2_k<double><<<pp.nblk, proj_threads<double>(), 0, s>>>(
          n, j + 1, (const double*)V, ldv, (const double*)u, (const double*)z, (double*)part,
          pp.nblk);
    if (proj && fused) {
      dcgs2_finish_k<double><<<1, kFinThreads, lds, s>>>(j, pp.nblk, (const double*)part,
                                                        (double*)H, ldh, (double*)cs,
                                                        (double*)cp, (double*)sc);
    } else if (proj) {
      reduce_cols_k<double><<<2 * (j + 1), kThreads, 0, s>>>(pp.nblk, (const double*)part,
                                                             (double*)S, nullptr, 0);
      dcgs2_coef_k<double><<<1, kThreads, 0, s>>>(j, (const double*)S, (double*)H, ldh,
                                                  (double*)cs, (double*)cp, (double*)sc);
      dcgs2_col_k<double><<<(j + 64) / 64, kThreads, 0, s>>>(j, (const double*)S, (double*)H,
                                                             ldh, (const double*)sc);
    }
    if (upd)
      update2_k<double><<<p.nblk, kThreads, 0, s>>>(n, j, (const double*)V, ldv,
                                                  (const double*)cs, (const double*)cp,
                                                  (const double*)sc, (double*)u, (double*)z);
  }
  return hipGetLastError();
}

// --------------------------------------------------------------------------
template <typename T>
static hipError_t project_t(int64_t n, int ncols, const T* V, int64_t ldv, const T* w, T* part,
                            T* h, T* hsum, int mode, hipStream_t s) {
  const RedPlan p = proj_plan<T>(n);
  if constexpr (sizeof(T) == 8) {
    if (p.threads == kProjWide) {
      project_k<T, kRpt, kProjWide><<<p.nblk, kProjWide, 0, s>>>(n, ncols, V, ldv, w, part,
                                                                 p.nblk);
      reduce_cols_k<T><<<ncols, kThreads, 0, s>>>(p.nblk, part, h, hsum, mode);
      return hipGetLastError();
    }
  }
  project_k<T><<<p.nblk, proj_threads<T>(), 0, s>>>(n, ncols, V, ldv, w, part, p.nblk);
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
