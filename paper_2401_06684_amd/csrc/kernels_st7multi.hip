// Temporal blocking of a polynomial recurrence on the 7-point stencil: NT
// consecutive terms of
//     s_t = a_t A s_{t-1} + b_t s_{t-1} + g0_t v + g1_t s_{t-2},   t = 1..NT,
// with s_0 = x and s_{-1} = y1, in one launch (the Clenshaw recurrence of a
// Chebyshev polynomial, Sec. 5.1: s_{t-2} is b_{k+2}, v the vector q(A) acts
// on).  Memory sees x, y1 and v read and s_{NT-1}, s_NT written: 5 vector
// passes for NT terms (NT = 3: 5/3 per term, against 5/2 for two terms and 4
// for one).  The intermediate terms never leave the chip.
//
// A workgroup owns a 64 x TY tile of the (x, y) plane and marches through its
// slab of kz planes in z.  Term t is needed on the tile grown by NT - t
// points on each side (its halo for the terms after it) and lags term t - 1
// by one plane: at step q, term t produces plane q - t + 1 (term 0, x itself,
// "produces" plane q + 1 by loading it).
//   * Every thread owns fixed points of the region of term 1 (the largest
//     computed one) and computes every term there, so the z-neighbours and
//     the centre of s_{t-1} (and s_{t-2}, the y1 of term t) are the thread's
//     own values of the last three steps, kept in registers.
//   * Only the in-plane neighbours go through LDS: each term has two plane
//     buffers; step q reads the planes written at step q - 1 and writes the
//     other buffer, so one barrier per step separates everything.
//   * Global loads are issued two steps before their use, into registers.
// Points outside the grid, and planes outside [0, nz), are zero (Dirichlet),
// so every s_t is zero there.
// The workgroup id is remapped so that each XCD gets a contiguous range of
// slabs (the halo planes of neighbouring slabs then meet in one L2).
// --------------------------------------------------------------------------
#include <hip/hip_runtime.h>

#include <type_traits>

#include "devmath.hpp"
#include "fa_internal.hpp"

#ifndef FA_MULTI_TY
#define FA_MULTI_TY 8
#endif
#ifndef FA_MULTI_BLOCKS
#define FA_MULTI_BLOCKS 512
#endif

namespace fa {

namespace {

struct St7M {
  int nx, ny, nz;
  double c0, cxm, cxp, cym, cyp, czm, czp;
};

template <int NT>
struct MultiCoef {
  double a[NT], b[NT], g0[NT], g1[NT];
};

template <int NT, int TY>
struct Geo {
  static constexpr int TX = 64, P = TX * TY;
  // region of term t: the tile grown by NT - t on each side
  static constexpr int W(int t) { return TX + 2 * (NT - t); }
  static constexpr int H(int t) { return TY + 2 * (NT - t); }
  static constexpr int N(int t) { return W(t) * H(t); }
  static constexpr int U = (N(1) + P - 1) / P;  // owned points per thread
  static constexpr int HALO = N(0) - N(1);      // x only: the ring around region 1
  // LDS (elements): two plane buffers per term 0 .. NT-1
  static constexpr int off(int t) {
    int o = 0;
    for (int u = 0; u < t; ++u) o += 2 * N(u);
    return o;
  }
  static constexpr int total() { return off(NT); }
};

template <typename T, typename TX, typename TO, int NT, int TY, bool Y1G, bool W1>
// at least 4 waves per SIMD: two 512-thread workgroups per CU
__global__ __launch_bounds__(64 * TY) __attribute__((amdgpu_waves_per_eu(4))) void st7_multi(St7M g, int kz, int gx, int gy, int nwg,
                                                     const TX* __restrict__ x,
                                                     const TX* __restrict__ v,
                                                     const TX* __restrict__ y1,
                                                     TO* __restrict__ out1,
                                                     TO* __restrict__ out2,
                                                     MultiCoef<NT> cd) {
  using G = Geo<NT, TY>;
  constexpr int U = G::U;
  __shared__ T lds[G::total()];
  const T c0 = (T)g.c0, cxm = (T)g.cxm, cxp = (T)g.cxp, cym = (T)g.cym, cyp = (T)g.cyp,
          czm = (T)g.czm, czp = (T)g.czp;
  const int lid = xcd_contiguous(blockIdx.x, nwg);
  const int bx = lid % gx, by = (lid / gx) % gy, bz = lid / (gx * gy);
  const int i0 = bx * G::TX, j0 = by * TY;
  const int k0 = bz * kz, k1 = min(k0 + kz, g.nz);
  const int tid = threadIdx.x;
  const int64_t plane = (int64_t)g.nx * g.ny;

  // owned points: region-1 coordinates (a, b), grid offset, in-grid flag
  int pa[U], pb[U];
  bool own[U], ing[U];
  int64_t poff[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int r = tid + u * G::P;
    own[u] = r < G::N(1);
    pa[u] = r % G::W(1);
    pb[u] = r / G::W(1);
    const int i = i0 - (NT - 1) + pa[u], j = j0 - (NT - 1) + pb[u];
    ing[u] = own[u] && i >= 0 && i < g.nx && j >= 0 && j < g.ny;
    poff[u] = (int64_t)j * g.nx + i;
  }
  // one point of the x ring around region 1 (threads tid < HALO)
  int hidx = 0;
  bool hing = false;
  int64_t hoff = 0;
  {
    const int h = tid;
    int xa = 0, ya = 0;
    if (h < G::W(0)) {
      xa = h;
      ya = 0;
    } else if (h < 2 * G::W(0)) {
      xa = h - G::W(0);
      ya = G::H(0) - 1;
    } else if (h < 2 * G::W(0) + G::H(1)) {
      xa = 0;
      ya = 1 + (h - 2 * G::W(0));
    } else {
      xa = G::W(0) - 1;
      ya = 1 + (h - 2 * G::W(0) - G::H(1));
    }
    hidx = ya * G::W(0) + xa;
    const int i = i0 - NT + xa, j = j0 - NT + ya;
    hing = tid < G::HALO && i >= 0 && i < g.nx && j >= 0 && j < g.ny;
    hoff = (int64_t)j * g.nx + i;
  }
  auto zin = [&](int p) { return p >= 0 && p < g.nz; };
  auto zoff = [&](int p) { return (int64_t)p * plane; };

  // rings: ring[s][k][u] = term s at the owned point u, produced two steps
  // ago (k = 0), one step ago (k = 1), this step (k = 2); s = 0 is x
  T ring[NT][3][U];
  T vr[NT][U];  // v at planes q, q - 1, .., q - NT + 1
#pragma unroll
  for (int s = 0; s < NT; ++s)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ring[s][0][u] = ring[s][1][u] = ring[s][2][u] = T(0);
      vr[s][u] = T(0);
    }

  // loads in flight, two steps ahead: slot 0 is consumed at step q (x at
  // plane q + 1, v and y1 at plane q), slot 1 at step q + 1
  T xn[2][U], xh[2] = {T(0), T(0)};
  T vn[2][U], yn[2][U];
  auto load_x = [&](int p, T* r, T& h) {
    const bool z = zin(p);
#pragma unroll
    for (int u = 0; u < U; ++u) r[u] = (z && ing[u]) ? (T)x[zoff(p) + poff[u]] : T(0);
    h = (z && hing) ? (T)x[zoff(p) + hoff] : T(0);
  };
  auto load_vy = [&](int p, T* rv, T* ry) {
    const bool z = zin(p);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      rv[u] = (z && ing[u]) ? (T)v[zoff(p) + poff[u]] : T(0);
      ry[u] = (Y1G && z && ing[u]) ? (T)y1[zoff(p) + poff[u]] : T(0);
    }
  };
  // x plane p into its LDS buffer (owned points and the halo point)
  auto put_x = [&](int p, const T* r, T h) {
    T* X = lds + G::off(0) + (p & 1) * G::N(0);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (own[u]) X[(pb[u] + 1) * G::W(0) + pa[u] + 1] = r[u];
    if (tid < G::HALO) X[hidx] = h;
  };

  const int q0 = k0 - NT + 1, qend = k1 + NT - 2;
  // prologue: x(q0 - 1) and x(q0) in the ring, x(q0) in LDS, x(q0 + 1) and
  // v, y1 at planes q0 and q0 + 1 in registers
  {
    T t0[U], t1[U], h1;
    load_x(q0 - 1, t0, h1);
    load_x(q0, t1, h1);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ring[0][0][u] = t0[u];
      ring[0][1][u] = t1[u];
    }
    put_x(q0, t1, h1);
  }
  load_x(q0 + 1, xn[0], xh[0]);
  load_vy(q0, vn[0], yn[0]);
  load_x(q0 + 2, xn[1], xh[1]);
  load_vy(q0 + 1, vn[1], yn[1]);
  __syncthreads();

  for (int q = q0; q <= qend; ++q) {
    // term 0: x(q + 1) into the ring and LDS; v, y1 at plane q into use
#pragma unroll
    for (int u = 0; u < U; ++u) ring[0][2][u] = xn[0][u];
    put_x(q + 1, xn[0], xh[0]);
    T ycur[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int s = NT - 1; s > 0; --s) vr[s][u] = vr[s - 1][u];
      vr[0][u] = vn[0][u];
      ycur[u] = yn[0][u];
      xn[0][u] = xn[1][u];
      vn[0][u] = vn[1][u];
      yn[0][u] = yn[1][u];
    }
    xh[0] = xh[1];
    // loads for step q + 2 (none past the last plane the slab needs)
    if (q + 3 <= k1 + NT - 1) load_x(q + 3, xn[1], xh[1]);
    if (q + 2 <= qend) load_vy(q + 2, vn[1], yn[1]);

    // terms 1 .. NT
#pragma unroll
    for (int t = 1; t <= NT; ++t) {
      const int p = q - t + 1;
      const bool need = p >= k0 - (NT - t) && p < k1 + (NT - t);
      const bool zp = zin(p);
      // in-plane neighbours of s_{t-1} at plane p (written at step q - 1)
      const int wl = G::W(t - 1);
      const T* L = lds + G::off(t - 1) + (p & 1) * G::N(t - 1);
      T* D = (t < NT) ? lds + G::off(t) + (p & 1) * G::N(t) : nullptr;
      const T a = (T)cd.a[t - 1], b = (T)cd.b[t - 1], e0 = (T)cd.g0[t - 1],
              e1 = (T)cd.g1[t - 1];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        // region-t coordinates of the owned point
        const int ra = pa[u] - (t - 1), rb = pb[u] - (t - 1);
        const bool inr = own[u] && ra >= 0 && ra < G::W(t) && rb >= 0 && rb < G::H(t);
        T val = T(0);
        if (inr && ing[u] && zp && need) {
          const int c = (rb + 1) * wl + (ra + 1);  // the point in region t - 1
          const T sv = ring[t - 1][1][u];
          T as = c0 * sv;
          as = fma(czm, ring[t - 1][0][u], as);
          as = fma(czp, ring[t - 1][2][u], as);
          as = fma(cxm, L[c - 1], as);
          as = fma(cxp, L[c + 1], as);
          as = fma(cym, L[c - wl], as);
          as = fma(cyp, L[c + wl], as);
          val = fma(a, as, b * sv);
          val = fma(e0, vr[t - 1][u], val);
          if (t == 1) {
            if (Y1G) val = fma(e1, ycur[u], val);
          } else {
            val = fma(e1, ring[t - 2][0][u], val);
          }
          const bool tile = ra >= NT - t && ra < NT - t + G::TX && rb >= NT - t &&
                            rb < NT - t + TY && p >= k0 && p < k1;
          if (t == NT && tile) out2[zoff(p) + poff[u]] = (TO)val;
          if (W1 && t == NT - 1 && tile) out1[zoff(p) + poff[u]] = (TO)val;
        }
        if (t < NT) {
          ring[t][2][u] = val;
          if (inr) D[rb * G::W(t) + ra] = val;
        }
      }
    }
    __syncthreads();  // this step's planes visible; last step's buffers free
#pragma unroll
    for (int s = 0; s < NT; ++s)
#pragma unroll
      for (int u = 0; u < U; ++u) {
        ring[s][0][u] = ring[s][1][u];
        ring[s][1][u] = ring[s][2][u];
      }
  }
}

template <typename T, typename TX, typename TO, int NT, int TY>
hipError_t launch_multi_t(const Op& op, const void* x, const void* v, const void* y1, void* out1,
                          void* out2, const MultiCoef<NT>& c, int blocks, hipStream_t st) {
  St7M g{op.dims[0], op.dims[1], op.dims[2], op.coef[0], op.coef[1], op.coef[2],
         op.coef[3], op.coef[4], op.coef[5], op.coef[6]};
  const int gx = (g.nx + 63) / 64, gy = (g.ny + TY - 1) / TY;
  int gz = (int)std::max<int64_t>(1, std::min<int64_t>(g.nz / 2, blocks / ((int64_t)gx * gy)));
  const int kz = (g.nz + gz - 1) / gz;
  gz = (g.nz + kz - 1) / kz;
  const int nwg = gx * gy * gz;
  const dim3 grid(nwg), block(64 * TY);
  const TX* xp = (const TX*)x;
  const TX* vp = (const TX*)v;
  const TX* yp = (const TX*)y1;
  TO* o1 = (TO*)out1;
  TO* o2 = (TO*)out2;
#define FA_MULTI(A, B)                                                                   \
  st7_multi<T, TX, TO, NT, TY, A, B><<<grid, block, 0, st>>>(g, kz, gx, gy, nwg, xp, vp, yp, \
                                                              o1, o2, c)
  if (y1 && out1)
    FA_MULTI(true, true);
  else if (y1)
    FA_MULTI(true, false);
  else if (out1)
    FA_MULTI(false, true);
  else
    FA_MULTI(false, false);
#undef FA_MULTI
  return hipGetLastError();
}

}  // namespace

hipError_t launch_chain_triple(const Op& op, const void* x, const void* v, const void* y1,
                               void* out1, void* out2, const ChainCoef k[3], hipStream_t s,
                               Prec pin, Prec pout, int blocks) {
  if (op.kind != OP_STENCIL7 || !x || !v || !out2) return hipErrorInvalidValue;
  MultiCoef<3> c;
  for (int t = 0; t < 3; ++t) {
    c.a[t] = k[t].alpha.real();
    c.b[t] = k[t].beta.real();
    c.g0[t] = k[t].g0.real();
    c.g1[t] = k[t].g1.real();
  }
  if (blocks <= 0) blocks = FA_MULTI_BLOCKS;
  constexpr int TY = FA_MULTI_TY;
  if (pin == P64 && pout == P64)
    return launch_multi_t<double, double, double, 3, TY>(op, x, v, y1, out1, out2, c, blocks, s);
  if (pin == P32 && pout == P32)
    return launch_multi_t<float, float, float, 3, TY>(op, x, v, y1, out1, out2, c, blocks, s);
  if (pin == P32 && pout == P64 && out1 == nullptr)
    return launch_multi_t<float, float, double, 3, TY>(op, x, v, y1, out1, out2, c, blocks, s);
  return hipErrorInvalidValue;
}

}  // namespace fa
