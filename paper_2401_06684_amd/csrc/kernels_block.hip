// Kernels of the block (several right-hand sides) form of the method.
//
// Blocks of s vectors are stored row-major: entry (point p, column c) of an
// n x s block at p * s + c, so the s values of one grid point are contiguous
// (one wavefront row of 64 lanes for s = 64).
//
//   st7_blk_k    : one recurrence term of q(A) on a block, 7-point stencil:
//                  out = alpha A X + beta X + g0 Y0 + g1 Y1
//   st7_blk_pair_k : two consecutive terms in one launch (the intermediate
//                  term kept on chip)
//   blk_proj_k   : split-K partial products V_i^T W (block Gram-Schmidt, Gram
//                  matrices), FP64 MFMA 16x16x4
//   gemm_k       : C = alpha A B + beta C, FP64 MFMA 16x16x4 (block updates
//                  W -= V P, W R^{-1}, x = V Z, the dense products of the
//                  Newton-Schulz iteration)
//   sum_parts_k  : deterministic sum of the split-K partials
//   chol_k       : Cholesky G = R^T R of an s x s Gram matrix and R^{-1}
//                  (one workgroup)
//
// FP64 MFMA lane layout (v_mfma_f64_16x16x4f64, checked on gfx950): lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16]; the four accumulator
// values of lane l are D[l / 16 + 4 r][l % 16], r = 0..3.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "devmath.hpp"
#include "fa_internal.hpp"

namespace fa {

typedef double dx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ dx4 mfma16(double a, double b, dx4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// --------------------------------------------------------------------------
// stencil term on a block
// --------------------------------------------------------------------------
struct BlkSt7 {
  int nx, ny, nz;
  int zc;  // planes per workgroup (z-march length)
  double c0, cxm, cxp, cym, cyp, czm, czp;
};

template <typename TX, typename TY, typename TO>
using blk_calc_t =
    typename std::conditional<std::is_same<TX, double>::value && std::is_same<TY, double>::value &&
                                  std::is_same<TO, double>::value,
                              double, float>::type;

// Workgroup tile: a segment of 1024 / S points of one x-line (fixed y) and
// all S columns, marching along z through zc planes.  Each thread owns four
// consecutive columns of one point (16- or 32-byte vector loads and stores)
// and keeps them at z - 1, z, z + 1 in registers, so the z-neighbours are
// read once.  x-neighbours come from the neighbouring threads' fresh loads
// (L1), the y-neighbour lines from the workgroups of the adjacent lines,
// which run alongside (tiles ordered segment, y, z-chunk, each XCD owning a
// contiguous range of tiles).
__device__ __forceinline__ void ld4(const float* p, float (&v)[4]) {
  const float4 t = *reinterpret_cast<const float4*>(p);
  v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
}
__device__ __forceinline__ void ld4(const double* p, double (&v)[4]) {
  const double2 a = *reinterpret_cast<const double2*>(p);
  const double2 b = *reinterpret_cast<const double2*>(p + 2);
  v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
__device__ __forceinline__ void st4(float* p, const float (&v)[4]) {
  *reinterpret_cast<float4*>(p) = float4{v[0], v[1], v[2], v[3]};
}
__device__ __forceinline__ void st4(double* p, const double (&v)[4]) {
  *reinterpret_cast<double2*>(p) = double2{v[0], v[1]};
  *reinterpret_cast<double2*>(p + 2) = double2{v[2], v[3]};
}
template <typename T, typename U>
__device__ __forceinline__ void ld4c(const U* p, T (&v)[4]) {
  U u[4];
  ld4(p, u);
#pragma unroll
  for (int q = 0; q < 4; ++q) v[q] = (T)u[q];
}

template <typename TX, typename TY, typename TO, int S, bool Y0, bool Y1>
__global__ __launch_bounds__(256) void st7_blk_k(BlkSt7 g, const TX* __restrict__ x,
                                                 const TY* __restrict__ y0, const TY* y1, TO* out,
                                                 double alpha, double beta, double g0, double g1) {
  using T = blk_calc_t<TX, TY, TO>;
  constexpr int CG = S / 4;      // column groups of 4
  constexpr int PPW = 256 / CG;  // points per segment
  const int nseg = (g.nx + PPW - 1) / PPW;
  const int lid = xcd_contiguous(blockIdx.x, gridDim.x);
  const int seg = lid % nseg;
  const int j = (lid / nseg) % g.ny;
  const int k0 = (lid / (nseg * g.ny)) * g.zc;
  const int k1 = min(k0 + g.zc, g.nz);
  const int i = seg * PPW + (int)threadIdx.x / CG;
  if (i >= g.nx) return;
  const int c = 4 * ((int)threadIdx.x % CG);
  const int64_t ls = (int64_t)g.nx * S;  // one line of the block
  const int64_t ps = ls * g.ny;          // one plane of the block
  const bool hx0 = i > 0, hx1 = i + 1 < g.nx, hy0 = j > 0, hy1 = j + 1 < g.ny;
  const T c0 = (T)g.c0, cxm = (T)g.cxm, cxp = (T)g.cxp, cym = (T)g.cym, cyp = (T)g.cyp,
          czm = (T)g.czm, czp = (T)g.czp;
  const T ta = (T)alpha, tb = (T)beta, t0 = (T)g0, t1 = (T)g1;
  int64_t e = (int64_t)k0 * ps + (int64_t)j * ls + (int64_t)i * S + c;
  T xm[4], xc[4], xp[4], v[4];
  if (k0 > 0) ld4c(x + e - ps, xm);
  else xm[0] = xm[1] = xm[2] = xm[3] = T(0);
  ld4c(x + e, xc);
  for (int k = k0; k < k1; ++k, e += ps) {
    if (k + 1 < g.nz) ld4c(x + e + ps, xp);
    else xp[0] = xp[1] = xp[2] = xp[3] = T(0);
    T ax[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) ax[q] = c0 * xc[q] + czm * xm[q] + czp * xp[q];
    if (hx0) {
      ld4c(x + e - S, v);
#pragma unroll
      for (int q = 0; q < 4; ++q) ax[q] += cxm * v[q];
    }
    if (hx1) {
      ld4c(x + e + S, v);
#pragma unroll
      for (int q = 0; q < 4; ++q) ax[q] += cxp * v[q];
    }
    if (hy0) {
      ld4c(x + e - ls, v);
#pragma unroll
      for (int q = 0; q < 4; ++q) ax[q] += cym * v[q];
    }
    if (hy1) {
      ld4c(x + e + ls, v);
#pragma unroll
      for (int q = 0; q < 4; ++q) ax[q] += cyp * v[q];
    }
    T r[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) r[q] = ta * ax[q] + tb * xc[q];
    if (Y0) {
      ld4c(y0 + e, v);
#pragma unroll
      for (int q = 0; q < 4; ++q) r[q] += t0 * v[q];
    }
    if (Y1) {  // y1 may alias out: read before the write
      ld4c(y1 + e, v);
#pragma unroll
      for (int q = 0; q < 4; ++q) r[q] += t1 * v[q];
    }
    TO o[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) o[q] = (TO)r[q];
    st4(out + e, o);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      xm[q] = xc[q];
      xc[q] = xp[q];
    }
  }
}

template <typename TX, typename TY, typename TO, int S>
static hipError_t st7_blk_s(const BlkSt7& g, const void* x, const void* y0, const void* y1,
                            void* out, double a, double b, double c0, double c1, hipStream_t st) {
  constexpr int PPW = 1024 / S;
  const int grid = ((g.nx + PPW - 1) / PPW) * g.ny * ((g.nz + g.zc - 1) / g.zc);
  const TX* X = (const TX*)x;
  const TY *A0 = (const TY*)y0, *A1 = (const TY*)y1;
  TO* O = (TO*)out;
  if (y0 && y1)
    st7_blk_k<TX, TY, TO, S, true, true><<<grid, 256, 0, st>>>(g, X, A0, A1, O, a, b, c0, c1);
  else if (y0)
    st7_blk_k<TX, TY, TO, S, true, false><<<grid, 256, 0, st>>>(g, X, A0, A1, O, a, b, c0, c1);
  else if (y1)
    st7_blk_k<TX, TY, TO, S, false, true><<<grid, 256, 0, st>>>(g, X, A0, A1, O, a, b, c0, c1);
  else
    st7_blk_k<TX, TY, TO, S, false, false><<<grid, 256, 0, st>>>(g, X, A0, A1, O, a, b, c0, c1);
  return hipGetLastError();
}

template <typename TX, typename TY, typename TO>
static hipError_t st7_blk_t(const BlkSt7& g, int lg_s, const void* x, const void* y0,
                            const void* y1, void* out, double a, double b, double c0, double c1,
                            hipStream_t st) {
  if (lg_s == 6) return st7_blk_s<TX, TY, TO, 64>(g, x, y0, y1, out, a, b, c0, c1, st);
  if (lg_s == 5) return st7_blk_s<TX, TY, TO, 32>(g, x, y0, y1, out, a, b, c0, c1, st);
  return st7_blk_s<TX, TY, TO, 16>(g, x, y0, y1, out, a, b, c0, c1, st);
}

hipError_t launch_blk_chain(const Op& op, int s, const void* x, const void* y0, const void* y1,
                            void* out, const ChainCoef& k, Prec px, Prec py, Prec po,
                            hipStream_t st, int zc) {
  if (zc < 1) return hipErrorInvalidValue;
  BlkSt7 g{op.dims[0], op.dims[1], op.dims[2], zc, op.coef[0], op.coef[1], op.coef[2],
           op.coef[3], op.coef[4], op.coef[5], op.coef[6]};
  const int lg_s = s == 16 ? 4 : s == 32 ? 5 : 6;
  const double a = k.alpha.real(), b = k.beta.real(), c0 = k.g0.real(), c1 = k.g1.real();
  if (px == P64 && py == P64 && po == P64)
    return st7_blk_t<double, double, double>(g, lg_s, x, y0, y1, out, a, b, c0, c1, st);
  if (px == P32 && py == P32 && po == P32)
    return st7_blk_t<float, float, float>(g, lg_s, x, y0, y1, out, a, b, c0, c1, st);
  if (px == P64 && po == P32 && !y0 && !y1)
    return st7_blk_t<double, float, float>(g, lg_s, x, y0, y1, out, a, b, c0, c1, st);
  if (px == P32 && py == P32 && po == P64)
    return st7_blk_t<float, float, double>(g, lg_s, x, y0, y1, out, a, b, c0, c1, st);
  return hipErrorInvalidValue;
}

// --------------------------------------------------------------------------
// two consecutive recurrence terms on a block (7-point stencil):
//   s = a1 A x + b1 x + e01 v + e11 y1,   out1 = s (if out1),
//   out2 = a2 A s + b2 s + e02 v + e12 x
// s never leaves the chip: 5 block passes for 2 terms instead of 8.
// --------------------------------------------------------------------------
// Workgroup tile: PX points along x, 4 lines along y, all S columns, marching
// along z; 1024 threads, each owning CW columns (16 bytes: 4 FP32 or 2 FP64
// values) of one tile point and of one point of the ring around the tile
// (the tile grown by one point, where s is needed for the second term's
// in-plane neighbours).  Step p computes s(p) on the tile and the ring (x's
// in-plane neighbours read from memory and cache, its z-neighbours kept in
// registers), then the second term at plane p - 1 on the tile (s's in-plane
// neighbours from an LDS plane buffer, its z-neighbours from registers), then
// stores s(p) into the other buffer: one barrier per plane.  Outputs must
// not alias inputs (neighbouring tiles read x around their own).
struct BlkPairCoef {
  double a1, b1, e01, e11, a2, b2, e02, e12;
};
template <int S, int CW>
struct BlkPairGeo {
  static constexpr int CG = S / CW;          // column groups, one per thread
  static constexpr int PY = 4;               // tile lines along y
  static constexpr int PX = 1024 / (PY * CG);  // tile points along x
  static constexpr int RW = PX + 2, RH = PY + 2;  // the grown tile
  static constexpr int RING = 2 * RW + 2 * PY;    // its points outside the tile
  static_assert(PX * PY * CG == 1024 && RING <= PX * PY, "one tile and one ring point per thread");
};

// CW consecutive values (16 bytes of U = T) or their conversion
template <int CW, typename U, typename T>
__device__ __forceinline__ void ldw(const U* p, T (&v)[CW]) {
  if constexpr (CW == 4) {
    U u[4];
    ld4(p, u);
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = (T)u[q];
  } else {
    static_assert(std::is_same<U, double>::value && CW == 2, "two doubles");
    const double2 a = *reinterpret_cast<const double2*>(p);
    v[0] = (T)a.x;
    v[1] = (T)a.y;
  }
}
template <int CW, typename U, typename T>
__device__ __forceinline__ void stw(U* p, const T (&v)[CW]) {
  if constexpr (CW == 4) {
    U u[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) u[q] = (U)v[q];
    st4(p, u);
  } else {
    static_assert(std::is_same<U, double>::value && CW == 2, "two doubles");
    *reinterpret_cast<double2*>(p) = double2{(double)v[0], (double)v[1]};
  }
}

template <typename TX, typename TO, int S, bool Y1G, bool W1>
__global__ __launch_bounds__(1024) void st7_blk_pair_k(BlkSt7 g, int gx, int gy,
                                                       const TX* __restrict__ x,
                                                       const TX* __restrict__ v,
                                                       const TX* __restrict__ y1,
                                                       TO* __restrict__ out1,
                                                       TO* __restrict__ out2, BlkPairCoef cf) {
  using T = blk_calc_t<TX, TX, TO>;
  constexpr int CW = 16 / (int)sizeof(T);
  using G = BlkPairGeo<S, CW>;
  __shared__ T sb[2][G::RW * G::RH * S];
  const int tid = threadIdx.x;
  const int cg = tid % G::CG, pt = tid / G::CG;
  const int c = CW * cg;
  const int lid = xcd_contiguous(blockIdx.x, gridDim.x);
  const int bx = lid % gx, by = (lid / gx) % gy, bz = lid / (gx * gy);
  const int i0 = bx * G::PX, j0 = by * G::PY;
  const int k0 = bz * g.zc, k1 = min(k0 + g.zc, g.nz);
  const int64_t ls = (int64_t)g.nx * S;  // one line of the block
  const int64_t ps = ls * g.ny;          // one plane of the block
  const T c0 = (T)g.c0, cxm = (T)g.cxm, cxp = (T)g.cxp, cym = (T)g.cym, cyp = (T)g.cyp,
          czm = (T)g.czm, czp = (T)g.czp;
  const T a1 = (T)cf.a1, b1 = (T)cf.b1, e01 = (T)cf.e01, e11 = (T)cf.e11;
  const T a2 = (T)cf.a2, b2 = (T)cf.b2, e02 = (T)cf.e02, e12 = (T)cf.e12;
  const bool has_ring = pt < G::RING;

  // u = 0: the tile point, u = 1: ring point pt (threads past the ring size
  // compute ring point 0 but store nothing: with no branch around the ring
  // work, the loads of both points issue together, 5 % faster in FP32)
  int ra[2], rb[2];  // coordinates in the grown tile
  ra[0] = pt % G::PX + 1;
  rb[0] = pt / G::PX + 1;
  {
    const int h = has_ring ? pt : 0;
    if (h < G::RW) {
      ra[1] = h;
      rb[1] = 0;
    } else if (h < 2 * G::RW) {
      ra[1] = h - G::RW;
      rb[1] = G::RH - 1;
    } else {
      const int r = h - 2 * G::RW;
      ra[1] = (r / G::PY) ? G::RW - 1 : 0;
      rb[1] = 1 + r % G::PY;
    }
  }
  bool ing[2];     // the point lies in the grid
  int64_t off[2];  // its in-plane offset (clamped into the grid)
  int nbm[2];      // bits 0..3: neighbour W, E, S, N inside the grid
  int li[2];       // LDS index of the point (grown-tile layout, column c)
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int i = i0 - 1 + ra[u], j = j0 - 1 + rb[u];
    ing[u] = i >= 0 && i < g.nx && j >= 0 && j < g.ny;
    off[u] = (int64_t)min(max(j, 0), g.ny - 1) * ls + (int64_t)min(max(i, 0), g.nx - 1) * S + c;
    // a neighbour of a point outside the grid is never used (that point's
    // value is zero); the bits then stay clear and the loads read `off`
    nbm[u] = ing[u] ? ((i > 0) | ((i + 1 < g.nx) << 1) | ((j > 0) << 2) | ((j + 1 < g.ny) << 3))
                    : 0;
    li[u] = (rb[u] * G::RW + ra[u]) * S + c;
  }
  auto pin = [&](int p) { return p >= 0 && p < g.nz; };
  auto poff = [&](int p) { return (int64_t)min(max(p, 0), g.nz - 1) * ps; };

  T xr[2][3][CW];  // x at planes p - 1, p, p + 1 of each point
  T sr[3][CW];     // s at planes p - 2, p - 1, p of the tile point
  T vk[CW];        // v at plane p - 1 of the tile point
#pragma unroll
  for (int q = 0; q < CW; ++q) sr[0][q] = sr[1][q] = sr[2][q] = vk[q] = T(0);
  auto load_pt = [&](const TX* base, int p, int u, T (&r)[CW]) {
    ldw<CW>(base + poff(p) + off[u], r);
    const bool z = pin(p) && ing[u];
#pragma unroll
    for (int q = 0; q < CW; ++q) r[q] = z ? r[q] : T(0);
  };
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    load_pt(x, k0 - 2, u, xr[u][1]);
    load_pt(x, k0 - 1, u, xr[u][2]);
  }
  for (int p = k0 - 1; p <= k1; ++p) {
    // x(p - 1), x(p) into place, x(p + 1) loaded
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
      for (int q = 0; q < CW; ++q) {
        xr[u][0][q] = xr[u][1][q];
        xr[u][1][q] = xr[u][2][q];
      }
      load_pt(x, p + 1, u, xr[u][2]);
    }
    // s(p) on the tile point and the ring point
    T sp[2][CW], vp[CW];
    const bool zp = pin(p);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const bool live = zp && ing[u];
      T as[CW], w[CW];
#pragma unroll
      for (int q = 0; q < CW; ++q) {
        as[q] = c0 * xr[u][1][q];
        as[q] = fma(czm, xr[u][0][q], as[q]);
        as[q] = fma(czp, xr[u][2][q], as[q]);
      }
      const TX* xb = x + poff(p) + off[u];
      const int64_t dn[4] = {-S, S, -ls, ls};
      const T cn[4] = {cxm, cxp, cym, cyp};
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        const bool in = (nbm[u] >> d) & 1;
        ldw<CW>(xb + (in ? dn[d] : 0), w);
#pragma unroll
        for (int q = 0; q < CW; ++q) as[q] = fma(cn[d], in ? w[q] : T(0), as[q]);
      }
      T vv[CW], yy[CW];
      ldw<CW>(v + poff(p) + off[u], vv);
      if (Y1G) ldw<CW>(y1 + poff(p) + off[u], yy);
#pragma unroll
      for (int q = 0; q < CW; ++q) {
        T val = fma(a1, as[q], b1 * xr[u][1][q]);
        val = fma(e01, live ? vv[q] : T(0), val);
        if (Y1G) val = fma(e11, live ? yy[q] : T(0), val);
        sp[u][q] = live ? val : T(0);
        if (u == 0) vp[q] = live ? vv[q] : T(0);
      }
    }
    // the second term at plane p - 1 on the tile point
    const int pm = p - 1;
    if (pm >= k0 && pm < k1) {
      const T* L = sb[pm & 1] + li[0];
      T nw[CW], ne[CW], ns[CW], nn[CW];
      ldw<CW>(L - S, nw);
      ldw<CW>(L + S, ne);
      ldw<CW>(L - G::RW * S, ns);
      ldw<CW>(L + G::RW * S, nn);
      T o2[CW], o1[CW];
#pragma unroll
      for (int q = 0; q < CW; ++q) {
        const T sc = sr[2][q];  // s(p - 1)
        T as = c0 * sc;
        as = fma(czm, sr[1][q], as);
        as = fma(czp, sp[0][q], as);
        as = fma(cxm, nw[q], as);
        as = fma(cxp, ne[q], as);
        as = fma(cym, ns[q], as);
        as = fma(cyp, nn[q], as);
        T val = fma(a2, as, b2 * sc);
        val = fma(e02, vk[q], val);
        val = fma(e12, xr[0][0][q], val);
        o2[q] = val;
        o1[q] = sc;
      }
      if (ing[0]) {
        stw<CW>(out2 + (int64_t)pm * ps + off[0], o2);
        if (W1) stw<CW>(out1 + (int64_t)pm * ps + off[0], o1);
      }
    }
    // s(p) into its plane buffer
    stw<CW>(&sb[p & 1][li[0]], sp[0]);
    if (has_ring) stw<CW>(&sb[p & 1][li[1]], sp[1]);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < CW; ++q) {
      sr[1][q] = sr[2][q];
      sr[2][q] = sp[0][q];
      vk[q] = vp[q];
    }
  }
}

template <typename TX, typename TO, int S>
static hipError_t st7_blk_pair_s(const BlkSt7& g, const void* x, const void* v, const void* y1,
                                 void* out1, void* out2, const BlkPairCoef& cf, hipStream_t st) {
  using G = BlkPairGeo<S, 16 / (int)sizeof(blk_calc_t<TX, TX, TO>)>;
  const int gx = (g.nx + G::PX - 1) / G::PX, gy = (g.ny + G::PY - 1) / G::PY;
  const int grid = gx * gy * ((g.nz + g.zc - 1) / g.zc);
  const TX *X = (const TX*)x, *Vp = (const TX*)v, *Y = (const TX*)y1;
  TO *O1 = (TO*)out1, *O2 = (TO*)out2;
#define FA_BLK_PAIR(A, B) \
  st7_blk_pair_k<TX, TO, S, A, B><<<grid, 1024, 0, st>>>(g, gx, gy, X, Vp, Y, O1, O2, cf)
  if (y1 && out1)
    FA_BLK_PAIR(true, true);
  else if (y1)
    FA_BLK_PAIR(true, false);
  else if (out1)
    FA_BLK_PAIR(false, true);
  else
    FA_BLK_PAIR(false, false);
#undef FA_BLK_PAIR
  return hipGetLastError();
}

template <typename TX, typename TO>
static hipError_t st7_blk_pair_t(const BlkSt7& g, int s, const void* x, const void* v,
                                 const void* y1, void* out1, void* out2, const BlkPairCoef& cf,
                                 hipStream_t st) {
  if (s == 64) return st7_blk_pair_s<TX, TO, 64>(g, x, v, y1, out1, out2, cf, st);
  if (s == 32) return st7_blk_pair_s<TX, TO, 32>(g, x, v, y1, out1, out2, cf, st);
  return st7_blk_pair_s<TX, TO, 16>(g, x, v, y1, out1, out2, cf, st);
}

hipError_t launch_blk_chain_pair(const Op& op, int s, const void* x, const void* v,
                                 const void* y1, void* out1, void* out2, const ChainCoef& k1,
                                 const ChainCoef& k2, Prec pin, Prec pout, hipStream_t st,
                                 int zc) {
  if (zc < 1 || !x || !v || !out2 || (s != 16 && s != 32 && s != 64))
    return hipErrorInvalidValue;
  BlkSt7 g{op.dims[0], op.dims[1], op.dims[2], zc, op.coef[0], op.coef[1], op.coef[2],
           op.coef[3], op.coef[4], op.coef[5], op.coef[6]};
  const BlkPairCoef cf{k1.alpha.real(), k1.beta.real(), k1.g0.real(), k1.g1.real(),
                       k2.alpha.real(), k2.beta.real(), k2.g0.real(), k2.g1.real()};
  if (pin == P64 && pout == P64)
    return st7_blk_pair_t<double, double>(g, s, x, v, y1, out1, out2, cf, st);
  if (pin == P32 && pout == P32)
    return st7_blk_pair_t<float, float>(g, s, x, v, y1, out1, out2, cf, st);
  if (pin == P32 && pout == P64 && !out1)
    return st7_blk_pair_t<float, double>(g, s, x, v, y1, out1, out2, cf, st);
  return hipErrorInvalidValue;
}

__global__ __launch_bounds__(256) void blk_to_f32_k(int64_t n, const double* __restrict__ x,
                                                    float* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}

hipError_t launch_blk_to_f32(int64_t count, const double* x, float* y, hipStream_t st) {
  blk_to_f32_k<<<(int)((count + 255) / 256), 256, 0, st>>>(count, x, y);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// split-K projections: part[sp][i][a][b] = sum_{r in chunk sp} V_i[r][a] W[r][b]
// --------------------------------------------------------------------------
// nsplit * nb workgroups of 256 threads; workgroup (sp, i) multiplies chunk
// sp of V_i and W.  The nb workgroups of one chunk are consecutive in a
// range that one XCD owns, so they run together there and read the chunk of
// W once from HBM (then from that XCD's L2).  Every wave takes every fourth
// group of 4 rows of the chunk and accumulates all (s/16)^2 output tiles; the
// four waves' tiles are added in LDS in a fixed order.
// Output index permutation: in tile (t, u) the MFMA row i and column j stand
// for a = T i + t and b = T j + u, so every lane reads its T values of a row
// of V_i (and of W) as one vector load.
template <int T> struct DVec;
template <> struct DVec<1> {
  double v[1];
  __device__ static DVec load(const double* p) { return DVec{{p[0]}}; }
};
template <> struct DVec<2> {
  double v[2];
  __device__ static DVec load(const double* p) {
    const double2 a = *reinterpret_cast<const double2*>(p);
    return DVec{{a.x, a.y}};
  }
};
template <> struct DVec<4> {
  double v[4];
  __device__ static DVec load(const double* p) {
    const dx4 a = *reinterpret_cast<const dx4*>(p);
    return DVec{{a[0], a[1], a[2], a[3]}};
  }
};

template <int T>
__global__ __launch_bounds__(256) void blk_proj_k(int64_t n, const double* __restrict__ V,
                                                  int64_t v_blk, const double* __restrict__ W,
                                                  double* __restrict__ part, int64_t chunk,
                                                  int nb) {
  constexpr int S = 16 * T;
  __shared__ double red[S * S];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int lid = xcd_contiguous(blockIdx.x, gridDim.x);
  const int sp = lid / nb, i = lid % nb;
  const double* Vi = V + (int64_t)i * v_blk;
  const int64_t r_beg = (int64_t)sp * chunk;
  const int64_t r_end = min(n, r_beg + chunk);
  dx4 acc[T][T];
#pragma unroll
  for (int a = 0; a < T; ++a)
#pragma unroll
    for (int b = 0; b < T; ++b) acc[a][b] = dx4{0.0, 0.0, 0.0, 0.0};
  const int rl = lane >> 4, cl = lane & 15;
  // Rows are loaded NS iterations ahead into NS register slots (one wave
  // per SIMD: the accumulators take the AGPRs, so the latency of HBM must be
  // hidden inside the wave); the loop is unrolled by NS so that each slot is
  // fixed at compile time, and a slot is refilled only after its MFMAs (a
  // load scheduled above them would need another register and a copy of an
  // unfinished load, i.e. a wait).  Rows past the chunk load a clamped row
  // and count as zero.
  constexpr int NS = 4;
  if (r_beg < r_end) {
    DVec<T> av[NS], bv[NS];
    auto fetch = [&](int64_t r0, auto slot) {
      constexpr int S2 = decltype(slot)::value;
      const int64_t r = min(r0 + rl, r_end - 1);
      av[S2] = DVec<T>::load(Vi + r * S + T * cl);
      bv[S2] = DVec<T>::load(W + r * S + T * cl);
    };
    auto use = [&](int64_t r0, auto slot) {
      constexpr int S2 = decltype(slot)::value;
      const bool ok = r0 + rl < r_end;
#pragma unroll
      for (int a = 0; a < T; ++a)
#pragma unroll
        for (int b = 0; b < T; ++b)
          acc[a][b] = mfma16(ok ? av[S2].v[a] : 0.0, bv[S2].v[b], acc[a][b]);
      __builtin_amdgcn_sched_barrier(0);
      fetch(r0 + 16 * NS, slot);
    };
    const int64_t first = r_beg + 4 * wv;
    fetch(first, std::integral_constant<int, 0>());
    fetch(first + 16, std::integral_constant<int, 1>());
    fetch(first + 32, std::integral_constant<int, 2>());
    fetch(first + 48, std::integral_constant<int, 3>());
    for (int64_t r0 = first; r0 < r_end; r0 += 16 * NS) {
      use(r0, std::integral_constant<int, 0>());
      use(r0 + 16, std::integral_constant<int, 1>());
      use(r0 + 32, std::integral_constant<int, 2>());
      use(r0 + 48, std::integral_constant<int, 3>());
    }
  }
  // wave w adds its tiles into red in turn (w = 0 stores)
  for (int w = 0; w < 4; ++w) {
    if (wv == w) {
#pragma unroll
      for (int a = 0; a < T; ++a)
#pragma unroll
        for (int b = 0; b < T; ++b)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int row = T * (rl + 4 * q) + a, col = T * cl + b;
            if (w == 0) red[row * S + col] = acc[a][b][q];
            else red[row * S + col] += acc[a][b][q];
          }
    }
    __syncthreads();
  }
  double* dst = part + ((int64_t)sp * nb + i) * S * S;
  for (int e = threadIdx.x; e < S * S; e += 256) dst[e] = red[e];
}

// P[i][a][b] (= or +=) sum_sp part[sp][i][a][b]; P (row i*s + a, column b)
// written into a row-major matrix with leading dimension ldp; with `acc`
// the sum is added to P instead of stored.
__global__ __launch_bounds__(256) void sum_parts_k(const double* __restrict__ part, int nsplit,
                                                   int nb, int s, double* P, int ldp, int acc) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t per = (int64_t)nb * s * s;
  if (e >= per) return;
  double t = 0.0;
  for (int sp = 0; sp < nsplit; ++sp) t += part[(int64_t)sp * per + e];
  const int i = (int)(e / ((int64_t)s * s));
  const int a = (int)((e / s) % s), b = (int)(e % s);
  double* d = P + (int64_t)(i * s + a) * ldp + b;
  *d = acc ? *d + t : t;
}

hipError_t launch_blk_proj(int64_t n, int s, int nb, const double* V, int64_t v_blk,
                           const double* W, double* part, int nsplit, double* P, int ldp, bool acc,
                           hipStream_t st) {
  const int64_t chunk = ((n + nsplit - 1) / nsplit + 15) / 16 * 16;
  const int grid = nsplit * nb;
  if (s == 64)
    blk_proj_k<4><<<grid, 256, 0, st>>>(n, V, v_blk, W, part, chunk, nb);
  else if (s == 32)
    blk_proj_k<2><<<grid, 256, 0, st>>>(n, V, v_blk, W, part, chunk, nb);
  else if (s == 16)
    blk_proj_k<1><<<grid, 256, 0, st>>>(n, V, v_blk, W, part, chunk, nb);
  else
    return hipErrorInvalidValue;
  const int64_t per = (int64_t)nb * s * s;
  sum_parts_k<<<(int)((per + 255) / 256), 256, 0, st>>>(part, nsplit, nb, s, P, ldp, acc ? 1 : 0);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// C = alpha A B + beta C (FP64 MFMA)
// --------------------------------------------------------------------------
// A (M x K): element (r, k) at A[(k / kb) * a_blk + r * lda + k % kb] (a
// matrix stored as column blocks of width kb, e.g. the basis blocks V_i, or a
// plain row-major matrix with kb = K); B (K x N) row-major ldb; C (M x N)
// row-major ldc.  Workgroup tile 64 rows x 16 T columns, one wave per 16
// rows.  K and kb multiples of 16, A 32-byte aligned with lda a multiple of
// 4, B and C 8 T-byte aligned with ldb, ldc multiples of T.
// Permutations that turn operand reads into vector loads: inside a group of
// 16 k, MFMA step q of lane group g takes k = 4 g + q (one 32-byte load of A
// per lane), and in column tile t the MFMA column j stands for column
// T j + t (one T-wide load of B per k, and T-wide stores of C).
template <int T>
__global__ __launch_bounds__(256) void gemm_k(int64_t M, int K, double alpha,
                                              const double* __restrict__ A, int64_t a_blk,
                                              int64_t lda, int kb, const double* __restrict__ B,
                                              int64_t ldb, double beta, double* C, int64_t ldc) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int rl = lane >> 4, cl = lane & 15;
  const int64_t r0 = (int64_t)blockIdx.x * 64 + wv * 16;
  const int c0 = blockIdx.y * 16 * T;
  if (r0 >= M) return;
  dx4 acc[T];
#pragma unroll
  for (int t = 0; t < T; ++t) acc[t] = dx4{0.0, 0.0, 0.0, 0.0};
  const int64_t ra = r0 + cl;  // the A row this lane supplies
  const bool arow = ra < M;
  const double* Ab = A + ra * lda + 4 * rl;
  const double* Bb = B + (int64_t)(4 * rl) * ldb + c0 + T * cl;
  const int per = kb / 16;  // groups of 16 k per column block of A
  const int ng = K / 16;
  // Groups are loaded two ahead into two register slots, the loop unrolled
  // by two so that the slots are fixed at compile time; a slot is refilled
  // only after its MFMAs (no copy of a register a load is still filling).
  // Groups past the end load the last group again and count as zero; rows
  // past M load row 0 and count as zero.
  const double* Abase = arow ? Ab : A + 4 * rl;
  dx4 a4[2];
  DVec<T> bq[2][4];
  auto fetch = [&](int g, auto slot) {
    constexpr int S = decltype(slot)::value;
    const int gc = min(g, ng - 1);
    const int blk = gc / per, kk = (gc - blk * per) * 16;
    a4[S] = *reinterpret_cast<const dx4*>(Abase + (int64_t)blk * a_blk + kk);
    const double* Bk = Bb + (int64_t)gc * 16 * ldb;
#pragma unroll
    for (int q = 0; q < 4; ++q) bq[S][q] = DVec<T>::load(Bk + (int64_t)q * ldb);
  };
  auto use = [&](int g, auto slot) {
    constexpr int S = decltype(slot)::value;
    const bool ok = arow && g < ng;
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int t = 0; t < T; ++t) acc[t] = mfma16(ok ? a4[S][q] : 0.0, bq[S][q].v[t], acc[t]);
    __builtin_amdgcn_sched_barrier(0);
    fetch(g + 2, slot);
  };
  fetch(0, std::integral_constant<int, 0>());
  fetch(1, std::integral_constant<int, 1>());
  for (int g = 0; g < ng; g += 2) {
    use(g, std::integral_constant<int, 0>());
    use(g + 1, std::integral_constant<int, 1>());
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t row = r0 + rl + 4 * q;
    if (row < M) {
      double* d = C + row * ldc + c0 + T * cl;
#pragma unroll
      for (int t = 0; t < T; ++t)
        d[t] = beta == 0.0 ? alpha * acc[t][q] : alpha * acc[t][q] + beta * d[t];
    }
  }
}

hipError_t launch_gemm(int64_t M, int N, int K, double alpha, const double* A, int64_t a_blk,
                       int64_t lda, int kb, const double* B, int64_t ldb, double beta, double* C,
                       int64_t ldc, hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (N % 16 || K % 16 || kb % 16 || K <= 0 || lda % 4 || ((uintptr_t)A & 31))
    return hipErrorInvalidValue;
  const int T = N % 64 == 0 ? 4 : N % 32 == 0 ? 2 : 1;
  if (ldb % T || ldc % T || ((uintptr_t)B & (8 * T - 1)) || ((uintptr_t)C & (8 * T - 1)))
    return hipErrorInvalidValue;
  const int gx = (int)((M + 63) / 64);
  if (N % 64 == 0) {
    gemm_k<4><<<dim3(gx, N / 64), 256, 0, st>>>(M, K, alpha, A, a_blk, lda, kb, B, ldb, beta, C, ldc);
  } else if (N % 32 == 0) {
    gemm_k<2><<<dim3(gx, N / 32), 256, 0, st>>>(M, K, alpha, A, a_blk, lda, kb, B, ldb, beta, C, ldc);
  } else {
    gemm_k<1><<<dim3(gx, N / 16), 256, 0, st>>>(M, K, alpha, A, a_blk, lda, kb, B, ldb, beta, C, ldc);
  }
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// small dense helpers (one workgroup or elementwise)
// --------------------------------------------------------------------------
// Cholesky G = R^T R (R upper triangular, s x s, row-major) and Rinv = R^{-1}.
// *flag = 1 when G is not (numerically) positive definite.
__global__ __launch_bounds__(256) void chol_k(int s, const double* __restrict__ G, double* R,
                                              double* Rinv, int* flag) {
  __shared__ double g[64 * 64];
  __shared__ double ri[64 * 64];
  __shared__ int bad;
  const int tid = threadIdx.x;
  for (int e = tid; e < s * s; e += 256) {
    g[e] = G[e];
    ri[e] = 0.0;
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  // right-looking: row k of R from the updated trailing matrix
  for (int k = 0; k < s; ++k) {
    if (tid == 0) {
      const double d = g[k * s + k];
      if (!(d > 0.0)) bad = 1;
      g[k * s + k] = d > 0.0 ? sqrt(d) : 1.0;
    }
    __syncthreads();
    const double rkk = g[k * s + k];
    for (int j = k + 1 + tid; j < s; j += 256) g[k * s + j] /= rkk;
    __syncthreads();
    for (int e = tid; e < (s - k - 1) * (s - k - 1); e += 256) {
      const int i = k + 1 + e / (s - k - 1), j = k + 1 + e % (s - k - 1);
      if (j >= i) g[i * s + j] -= g[k * s + i] * g[k * s + j];
    }
    __syncthreads();
  }
  // R^{-1} by back substitution, one column per thread
  for (int c = tid; c < s; c += 256) {
    for (int i = c; i >= 0; --i) {
      double t = (i == c) ? 1.0 : 0.0;
      for (int j = i + 1; j <= c; ++j) t -= g[i * s + j] * ri[j * s + c];
      ri[i * s + c] = t / g[i * s + i];
    }
  }
  __syncthreads();
  for (int e = tid; e < s * s; e += 256) {
    const int i = e / s, j = e % s;
    R[e] = j >= i ? g[e] : 0.0;
    Rinv[e] = j >= i ? ri[e] : 0.0;
  }
  if (tid == 0 && bad) *flag = 1;
}

hipError_t launch_chol(int s, const double* G, double* R, double* Rinv, int* flag,
                       hipStream_t st) {
  if (s > 64) return hipErrorInvalidValue;
  chol_k<<<1, 256, 0, st>>>(s, G, R, Rinv, flag);
  return hipGetLastError();
}

// C (M x N, ldc) = diag value d on the diagonal, 0 elsewhere
__global__ __launch_bounds__(256) void set_diag_k(int M, int N, double d, double* C, int64_t ldc) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)M * N) return;
  const int i = (int)(e / N), j = (int)(e % N);
  C[i * ldc + j] = (i == j) ? d : 0.0;
}

hipError_t launch_set_diag(int M, int N, double d, double* C, int64_t ldc, hipStream_t st) {
  set_diag_k<<<(int)(((int64_t)M * N + 255) / 256), 256, 0, st>>>(M, N, d, C, ldc);
  return hipGetLastError();
}

// Y (M x N, ldy) = a X (ldx)
__global__ __launch_bounds__(256) void scale_mat_k(int M, int N, double a, const double* X,
                                                   int64_t ldx, double* Y, int64_t ldy) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)M * N) return;
  const int i = (int)(e / N), j = (int)(e % N);
  Y[i * ldy + j] = a * X[i * ldx + j];
}

hipError_t launch_scale_mat(int M, int N, double a, const double* X, int64_t ldx, double* Y,
                            int64_t ldy, hipStream_t st) {
  scale_mat_k<<<(int)(((int64_t)M * N + 255) / 256), 256, 0, st>>>(M, N, a, X, ldx, Y, ldy);
  return hipGetLastError();
}

// Y (M x N, ldy) += X (ldx)
__global__ __launch_bounds__(256) void add_mat_k(int M, int N, const double* X, int64_t ldx,
                                                 double* Y, int64_t ldy) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)M * N) return;
  const int i = (int)(e / N), j = (int)(e % N);
  Y[i * ldy + j] += X[i * ldx + j];
}

hipError_t launch_add_mat(int M, int N, const double* X, int64_t ldx, double* Y, int64_t ldy,
                          hipStream_t st) {
  add_mat_k<<<(int)(((int64_t)M * N + 255) / 256), 256, 0, st>>>(M, N, X, ldx, Y, ldy);
  return hipGetLastError();
}

// row statistics, one wave per row: rs[i] = sum_j |X[i][j]|,
// dv[i] = max_j |X[i][j] - (i == j)|; then out[0] = max rs, out[1] = max dv
__global__ __launch_bounds__(256) void row_stats_k(int M, const double* __restrict__ X,
                                                   int64_t ldx, double* __restrict__ rs,
                                                   double* __restrict__ dv) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= M) return;
  double sum = 0.0, mx = 0.0;
  for (int j = lane; j < M; j += 64) {
    const double v = X[(int64_t)i * ldx + j];
    sum += fabs(v);
    mx = fmax(mx, fabs(v - (i == j ? 1.0 : 0.0)));
  }
  for (int m = 32; m >= 1; m >>= 1) {
    sum += __shfl_xor(sum, m, 64);
    mx = fmax(mx, __shfl_xor(mx, m, 64));
  }
  if (lane == 0) {
    rs[i] = sum;
    dv[i] = mx;
  }
}

__global__ __launch_bounds__(256) void max2_k(int M, const double* __restrict__ rs,
                                              const double* __restrict__ dv, double* out) {
  __shared__ double sh[2][4];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < M; i += 256) {
    a = fmax(a, rs[i]);
    b = fmax(b, dv[i]);
  }
  for (int m = 32; m >= 1; m >>= 1) {
    a = fmax(a, __shfl_xor(a, m, 64));
    b = fmax(b, __shfl_xor(b, m, 64));
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    sh[0][wv] = a;
    sh[1][wv] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = fmax(fmax(sh[0][0], sh[0][1]), fmax(sh[0][2], sh[0][3]));
    out[1] = fmax(fmax(sh[1][0], sh[1][1]), fmax(sh[1][2], sh[1][3]));
  }
}

// scratch: 2 M doubles
hipError_t launch_mat_norms(int M, const double* X, int64_t ldx, double* out, double* scratch,
                            hipStream_t st) {
  row_stats_k<<<(M + 3) / 4, 256, 0, st>>>(M, X, ldx, scratch, scratch + M);
  max2_k<<<1, 256, 0, st>>>(M, scratch, scratch + M, out);
  return hipGetLastError();
}

}  // namespace fa
