// Fused polynomial-chain step for every operator:
//     out = alpha * (A x) + beta * x + g0 * y0 + g1 * y1
// One launch evaluates one term of the Clenshaw recurrence of Sec. 5.1
// (b_k = c_k v + 2 Ahat b_{k+1} - b_{k+2}, Ahat = sigma A + tau I), one step of
// the Horner-type Newton recurrence of Sec. 5.2 (r <- (A - theta) r / rho + eta v)
// or a plain product with A: the operator application and the vector update
// of the recurrence are one pass over memory, so a recurrence term costs one
// read of x (its neighbours come from cache), one read of each combined
// vector and one write.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "devmath.hpp"
#include "fa_internal.hpp"

namespace fa {

// --------------------------------------------------------------------------
// 7-point / 5-point stencil, real FP64, zero Dirichlet boundary.
// A workgroup owns a 64 x 4 tile of the (x, y) plane (one wavefront per row
// segment, coalesced along x) and marches through kz planes in z, keeping the
// z-neighbours in registers, so x is read from memory about once per point;
// x/y neighbours come from L1/L2.
// The hardware deals consecutive workgroup ids round-robin to the eight XCDs,
// each with its own L2.  The id is remapped so that every XCD gets one
// contiguous slab of tiles: the halo rows and planes a tile shares with its
// neighbours are then fetched once into that XCD's L2 instead of once per XCD.
// --------------------------------------------------------------------------
struct St7 {
  int nx, ny, nz;
  double c0, cxm, cxp, cym, cyp, czm, czp;
};

constexpr int ST_TX = 64, ST_TY = 4;

// Storage types: TX for every input vector (x, y0, y1), TO for the output.
// Arithmetic is FP64 when both are double and FP32 otherwise (the mixed
// precision mode keeps the polynomial chain in FP32 storage with FP32
// accumulation; the first launch reads the FP64 basis vector, the last one
// writes the FP64 result).
template <typename TX, typename TO>
using calc_t = typename std::conditional<std::is_same<TX, double>::value &&
                                             std::is_same<TO, double>::value,
                                         double, float>::type;

template <typename TX, typename TO, bool Y0, bool Y1>
__global__ __launch_bounds__(ST_TX* ST_TY) void st7_chain(St7 s, int kz, int gx, int gy, int nwg,
                                                          int64_t bstride,
                                                          const TX* __restrict__ x,
                                                          const TX* __restrict__ y0,
                                                          const TX* y1, TO* out, double al_,
                                                          double be_, double g0_, double g1_) {
  using T = calc_t<TX, TO>;
  const T al = (T)al_, be = (T)be_, g0 = (T)g0_, g1 = (T)g1_;
  const T c0 = (T)s.c0, cxm = (T)s.cxm, cxp = (T)s.cxp, cym = (T)s.cym, cyp = (T)s.cyp,
          czm = (T)s.czm, czp = (T)s.czp;
  // a batch of vectors (bstride elements apart): vector blockIdx.y
  const int col = blockIdx.y, lid = xcd_contiguous(blockIdx.x, nwg);
  {
    const int64_t o = (int64_t)col * bstride;
    x += o;
    if (Y0) y0 += o;
    if (Y1) y1 += o;
    out += o;
  }
  const int bx = lid % gx, by = (lid / gx) % gy, bz = lid / (gx * gy);
  const int i = bx * ST_TX + (threadIdx.x & (ST_TX - 1));
  const int j = by * ST_TY + (threadIdx.x / ST_TX);
  const int k0 = bz * kz;
  const int k1 = min(k0 + kz, s.nz);
  if (i >= s.nx || j >= s.ny || k0 >= s.nz) return;
  const int64_t plane = (int64_t)s.nx * s.ny;
  int64_t p = (int64_t)k0 * plane + (int64_t)j * s.nx + i;
  const bool hx0 = i > 0, hx1 = i + 1 < s.nx, hy0 = j > 0, hy1 = j + 1 < s.ny;
  T xz0 = (k0 > 0) ? (T)x[p - plane] : T(0);
  T xc = (T)x[p];
  for (int k = k0; k < k1; ++k, p += plane) {
    const T xz1 = (k + 1 < s.nz) ? (T)x[p + plane] : T(0);
    T ax = c0 * xc;
    ax = fma(czm, xz0, ax);
    ax = fma(czp, xz1, ax);
    if (hx0) ax = fma(cxm, (T)x[p - 1], ax);
    if (hx1) ax = fma(cxp, (T)x[p + 1], ax);
    if (hy0) ax = fma(cym, (T)x[p - s.nx], ax);
    if (hy1) ax = fma(cyp, (T)x[p + s.nx], ax);
    T r = fma(al, ax, be * xc);
    if (Y0) r = fma(g0, (T)y0[p], r);
    if (Y1) r = fma(g1, (T)y1[p], r);
    out[p] = (TO)r;
    xz0 = xc;
    xc = xz1;
  }
}

template <typename TX, typename TO>
static hipError_t launch_st7_t(const Op& op, const void* xv, const void* y0v, const void* y1v,
                               void* outv, const ChainCoef& k, hipStream_t st) {
  const TX* x = (const TX*)xv;
  const TX* y0 = (const TX*)y0v;
  const TX* y1 = (const TX*)y1v;
  TO* out = (TO*)outv;
  St7 s{op.dims[0], op.dims[1], op.dims[2], op.coef[0], op.coef[1], op.coef[2],
        op.coef[3], op.coef[4], op.coef[5], op.coef[6]};
  const int gx = (s.nx + ST_TX - 1) / ST_TX, gy = (s.ny + ST_TY - 1) / ST_TY;
  // enough z-slabs for ~2048 workgroups over the batch, at least one plane
  // per thread
  const int nb = std::max(1, op.nbatch);
  const int64_t want = 2048;
  int gz = (int)std::min<int64_t>(s.nz, std::max<int64_t>(1, want / ((int64_t)gx * gy * nb)));
  const int kz = (s.nz + gz - 1) / gz;
  gz = (s.nz + kz - 1) / kz;
  const int nwg = gx * gy * gz;
  const int64_t bs = nb > 1 ? op.bstride : 0;
  const double al = k.alpha.real(), be = k.beta.real(), g0 = k.g0.real(), g1 = k.g1.real();
  const dim3 grid(nwg, nb), block(ST_TX * ST_TY);
#define FA_ST7(A, B) \
  st7_chain<TX, TO, A, B><<<grid, block, 0, st>>>(s, kz, gx, gy, nwg, bs, x, y0, y1, out, al, be, g0, g1)
  if (y0 && y1)
    FA_ST7(true, true);
  else if (y0)
    FA_ST7(true, false);
  else if (y1)
    FA_ST7(false, true);
  else
    FA_ST7(false, false);
#undef FA_ST7
  return hipGetLastError();
}

static hipError_t launch_st7(const Op& op, const void* x, const void* y0, const void* y1, void* out,
                             const ChainCoef& k, hipStream_t st, Prec pin, Prec pout) {
  if (pin == P64 && pout == P64) return launch_st7_t<double, double>(op, x, y0, y1, out, k, st);
  if (pin == P64) return launch_st7_t<double, float>(op, x, y0, y1, out, k, st);
  if (pout == P64) return launch_st7_t<float, double>(op, x, y0, y1, out, k, st);
  return launch_st7_t<float, float>(op, x, y0, y1, out, k, st);
}

// --------------------------------------------------------------------------
// Two consecutive recurrence terms of the 7-point stencil in one launch:
//     s    = a1 A x + b1 x + g01 y0 + g11 y1        (term t, on the tile + 1 halo)
//     out2 = a2 A s + b2 s + g02 y0 + g12 x         (term t + 1, on the tile)
// For the Clenshaw recurrence x = b_{k+1}, y0 = v, y1 = b_{k+2}, s = b_k and
// out2 = b_{k-1}: a pair of terms reads x, v, b_{k+2} and writes b_k, b_{k-1}
// (5 vector passes instead of 8 for two single-term launches).  s never leaves
// the chip except for the tile written to out1 (skipped when nothing reads it).
// A workgroup owns a 64 x 8 tile and marches through kz planes in z with three
// LDS rings: x on the tile + 2 halo (three planes), s on the tile + 1 halo
// (three planes).  The values outside the grid are zero (Dirichlet), so s is
// zero there too.  out1 and out2 must not alias x, y0 or y1, which are read on
// the halo of neighbouring tiles.
// --------------------------------------------------------------------------
#ifndef FA_PAIR_TY
#define FA_PAIR_TY 8
#endif
#ifndef FA_PAIR_ZFIRST
#define FA_PAIR_ZFIRST 0
#endif
#ifndef FA_PAIR_BLOCKS
#define FA_PAIR_BLOCKS 512
#endif
constexpr int P_TX = 64, P_TY = FA_PAIR_TY;
constexpr int P_XW = P_TX + 4, P_XH = P_TY + 4;  // x region (tile + 2)
constexpr int P_SW = P_TX + 2, P_SH = P_TY + 2;  // s region (tile + 1)
constexpr int P_THREADS = P_TX * P_TY;
constexpr int P_XPT = (P_XW * P_XH + P_THREADS - 1) / P_THREADS;  // x points per thread
constexpr int P_SPT = (P_SW * P_SH + P_THREADS - 1) / P_THREADS;  // s points per thread

struct PairCoef {
  double a1, b1, g01, g11, a2, b2, g02, g12;
};

// Software pipeline: the global loads for the next plane (x on the x region,
// y0 / y1 on the s region, y0 on the tile) are issued into registers before
// the current plane is computed from LDS, so their latency overlaps the work
// of the current step instead of stalling at a barrier.  The x ring has four
// planes so that the prefetched plane can be stored while the previous one is
// still being read: two barriers per plane.
__device__ __forceinline__ int xslot(int q) { return (q + 8) & 3; }
__device__ __forceinline__ int sslot(int q) { return (q + 6) % 3; }

template <typename TX, typename TO, bool Y0, bool Y1, bool W1>
__global__ __launch_bounds__(P_THREADS) void st7_pair(St7 s, int kz, int gx, int gy, int nwg,
                                                      int64_t bstride,
                                                      const TX* __restrict__ x,
                                                      const TX* __restrict__ y0,
                                                      const TX* __restrict__ y1,
                                                      TO* __restrict__ out1,
                                                      TO* __restrict__ out2, PairCoef cd_) {
  using T = calc_t<TX, TO>;
  struct {
    T a1, b1, g01, g11, a2, b2, g02, g12;
  } c{(T)cd_.a1, (T)cd_.b1, (T)cd_.g01, (T)cd_.g11, (T)cd_.a2, (T)cd_.b2, (T)cd_.g02, (T)cd_.g12};
  const T c0 = (T)s.c0, cxm = (T)s.cxm, cxp = (T)s.cxp, cym = (T)s.cym, cyp = (T)s.cyp,
          czm = (T)s.czm, czp = (T)s.czp;
  __shared__ T xs[4][P_XH][P_XW];
  __shared__ T ss[3][P_SH][P_SW];
  // a batch of vectors (bstride elements apart): vector blockIdx.y
  const int col = blockIdx.y, lid = xcd_contiguous(blockIdx.x, nwg);
  {
    const int64_t o = (int64_t)col * bstride;
    x += o;
    if (Y0) y0 += o;
    if (Y1) y1 += o;
    if (W1) out1 += o;
    out2 += o;
  }
#if FA_PAIR_ZFIRST
  const int gz = nwg / (gx * gy);
  const int bz = lid % gz, bx = (lid / gz) % gx, by = lid / (gz * gx);
#else
  const int bx = lid % gx, by = (lid / gx) % gy, bz = lid / (gx * gy);
#endif
  const int i0 = bx * P_TX, j0 = by * P_TY;
  const int k0 = bz * kz, k1 = min(k0 + kz, s.nz);
  const int tid = threadIdx.x;
  const int tx = tid % P_TX, ty = tid / P_TX;
  const int64_t plane = (int64_t)s.nx * s.ny;
  auto in_grid = [&](int i, int j) { return i >= 0 && i < s.nx && j >= 0 && j < s.ny; };

  // per-thread fixed points of the x region, the s region and the tile
  int64_t xoff[P_XPT];
  bool xok[P_XPT], xin[P_XPT];
#pragma unroll
  for (int u = 0; u < P_XPT; ++u) {
    const int r = tid + u * P_THREADS;
    const int rx = r % P_XW, ry = r / P_XW;
    const int i = i0 - 2 + rx, j = j0 - 2 + ry;
    xin[u] = r < P_XW * P_XH;
    xok[u] = xin[u] && in_grid(i, j);
    xoff[u] = (int64_t)j * s.nx + i;
  }
  int64_t soff[P_SPT];
  bool sok[P_SPT], sin_[P_SPT], stile[P_SPT];
  int sxx[P_SPT], syy[P_SPT];
#pragma unroll
  for (int u = 0; u < P_SPT; ++u) {
    const int r = tid + u * P_THREADS;
    const int sx = r % P_SW, sy = r / P_SW;
    const int i = i0 - 1 + sx, j = j0 - 1 + sy;
    sxx[u] = sx;
    syy[u] = sy;
    sin_[u] = r < P_SW * P_SH;
    sok[u] = sin_[u] && in_grid(i, j);
    stile[u] = sx >= 1 && sx <= P_TX && sy >= 1 && sy <= P_TY;
    soff[u] = (int64_t)j * s.nx + i;
  }
  const bool tok = in_grid(i0 + tx, j0 + ty);
  const int64_t toff = (int64_t)(j0 + ty) * s.nx + (i0 + tx);

  auto fetch_x = [&](int q, T* reg) {
    const bool zin = q >= 0 && q < s.nz;
#pragma unroll
    for (int u = 0; u < P_XPT; ++u)
      reg[u] = (zin && xok[u]) ? (T)x[(int64_t)q * plane + xoff[u]] : T(0);
  };
  auto store_x = [&](int q, const T* reg) {
    T* dst = &xs[xslot(q)][0][0];
#pragma unroll
    for (int u = 0; u < P_XPT; ++u)
      if (xin[u]) dst[tid + u * P_THREADS] = reg[u];
  };
  auto fetch_y = [&](int q, T* r0, T* r1) {
    const bool zin = q >= 0 && q < s.nz;
#pragma unroll
    for (int u = 0; u < P_SPT; ++u) {
      const bool ok = zin && sok[u];
      r0[u] = (Y0 && ok) ? (T)y0[(int64_t)q * plane + soff[u]] : T(0);
      r1[u] = (Y1 && ok) ? (T)y1[(int64_t)q * plane + soff[u]] : T(0);
    }
  };
  auto stage1 = [&](int q, const T* r0, const T* r1) {
    T(*dst)[P_SW] = ss[sslot(q)];
    const bool zin = q >= 0 && q < s.nz;
    const T(*xm)[P_XW] = xs[xslot(q - 1)];
    const T(*xc)[P_XW] = xs[xslot(q)];
    const T(*xp)[P_XW] = xs[xslot(q + 1)];
#pragma unroll
    for (int u = 0; u < P_SPT; ++u) {
      if (!sin_[u]) continue;
      const int sx = sxx[u], sy = syy[u];
      T v = T(0);
      if (zin && sok[u]) {
        const int cx = sx + 1, cy = sy + 1;
        const T xv = xc[cy][cx];
        T ax = c0 * xv;
        ax = fma(czm, xm[cy][cx], ax);
        ax = fma(czp, xp[cy][cx], ax);
        ax = fma(cxm, xc[cy][cx - 1], ax);
        ax = fma(cxp, xc[cy][cx + 1], ax);
        ax = fma(cym, xc[cy - 1][cx], ax);
        ax = fma(cyp, xc[cy + 1][cx], ax);
        v = fma(c.a1, ax, c.b1 * xv);
        if (Y0) v = fma(c.g01, r0[u], v);
        if (Y1) v = fma(c.g11, r1[u], v);
        if (W1 && q >= k0 && q < k1 && stile[u]) out1[(int64_t)q * plane + soff[u]] = (TO)v;
      }
      dst[sy][sx] = v;
    }
  };
  auto stage2 = [&](int z, T yt) {
    if (!tok) return;
    const T(*sm)[P_SW] = ss[sslot(z - 1)];
    const T(*sc)[P_SW] = ss[sslot(z)];
    const T(*sp)[P_SW] = ss[sslot(z + 1)];
    const int cx = tx + 1, cy = ty + 1;
    const T sv = sc[cy][cx];
    T as = c0 * sv;
    as = fma(czm, sm[cy][cx], as);
    as = fma(czp, sp[cy][cx], as);
    as = fma(cxm, sc[cy][cx - 1], as);
    as = fma(cxp, sc[cy][cx + 1], as);
    as = fma(cym, sc[cy - 1][cx], as);
    as = fma(cyp, sc[cy + 1][cx], as);
    T r = fma(c.a2, as, c.b2 * sv);
    if (Y0) r = fma(c.g02, yt, r);
    r = fma(c.g12, xs[xslot(z)][ty + 2][tx + 2], r);
    out2[(int64_t)z * plane + toff] = (TO)r;
  };

  // s(q) needs x planes q-1..q+1; out2(z) needs s planes z-1..z+1.  Loads run
  // two steps ahead: at step q the registers receive x plane q+3, y0 / y1 of
  // plane q+2 and y0 of the tile at plane q+1.
  {
    T t[P_XPT];
    fetch_x(k0 - 2, t);
    store_x(k0 - 2, t);
    fetch_x(k0 - 1, t);
    store_x(k0 - 1, t);
    fetch_x(k0, t);
    store_x(k0, t);
  }
  T xa[P_XPT];  // x plane q + 2
  fetch_x(k0 + 1, xa);
  T y0c[P_SPT], y1c[P_SPT], y0n[P_SPT], y1n[P_SPT];  // y at planes q, q + 1
  fetch_y(k0 - 1, y0c, y1c);
  fetch_y(k0, y0n, y1n);
  T ytc = T(0);  // y0 on the tile at plane q - 1 (for stage2(q - 1))
  T ytn = (Y0 && tok && k0 < k1) ? (T)y0[(int64_t)k0 * plane + toff] : T(0);  // plane q
  __syncthreads();
  for (int q = k0 - 1; q <= k1; ++q) {
    T xb[P_XPT], y0m[P_SPT], y1m[P_SPT];
    const bool fx = q + 3 <= k1 + 1, fy = q + 2 <= k1;
    if (fx) fetch_x(q + 3, xb);
    if (fy) fetch_y(q + 2, y0m, y1m);
    T ytm = T(0);
    if (Y0 && tok && q + 1 >= k0 && q + 1 < k1) ytm = (T)y0[(int64_t)(q + 1) * plane + toff];
    stage1(q, y0c, y1c);
    __syncthreads();  // s(q) complete
    if (q - 1 >= k0) stage2(q - 1, ytc);
    // the slot of plane q + 2 held plane q - 2, last read before the barrier above
    if (q + 2 <= k1 + 1) store_x(q + 2, xa);
    __syncthreads();  // x(q + 2) visible; stage2 done with s(q - 2)
#pragma unroll
    for (int u = 0; u < P_XPT; ++u) xa[u] = xb[u];
#pragma unroll
    for (int u = 0; u < P_SPT; ++u) {
      y0c[u] = y0n[u];
      y1c[u] = y1n[u];
      y0n[u] = y0m[u];
      y1n[u] = y1m[u];
    }
    ytc = ytn;
    ytn = ytm;
  }
}

template <typename TX, typename TO>
static hipError_t launch_st7_pair_t(const Op& op, const void* xv, const void* y0v,
                                    const void* y1v, void* out1v, void* out2v,
                                    const PairCoef& c, hipStream_t st) {
  const TX* x = (const TX*)xv;
  const TX* y0 = (const TX*)y0v;
  const TX* y1 = (const TX*)y1v;
  TO* out1 = (TO*)out1v;
  TO* out2 = (TO*)out2v;
  St7 s{op.dims[0], op.dims[1], op.dims[2], op.coef[0], op.coef[1], op.coef[2],
        op.coef[3], op.coef[4], op.coef[5], op.coef[6]};
  const int gx = (s.nx + P_TX - 1) / P_TX, gy = (s.ny + P_TY - 1) / P_TY;
  // about FA_PAIR_BLOCKS workgroups, at least 2 planes each (the x ring reads
  // 2 extra planes on each side of a workgroup's slab)
  const int nb = std::max(1, op.nbatch);
  int gz = (int)std::max<int64_t>(
      1, std::min<int64_t>(s.nz / 2, FA_PAIR_BLOCKS / ((int64_t)gx * gy * nb)));
  const int kz = (s.nz + gz - 1) / gz;
  gz = (s.nz + kz - 1) / kz;
  const int nwg = gx * gy * gz;
  const int64_t bs = nb > 1 ? op.bstride : 0;
  const bool w1 = out1 != nullptr;
  const dim3 grid(nwg, nb), block(P_THREADS);
#define FA_PAIR(A, B, C) \
  st7_pair<TX, TO, A, B, C><<<grid, block, 0, st>>>(s, kz, gx, gy, nwg, bs, x, y0, y1, out1, out2, c)
  if (y0 && y1) {
    if (w1) FA_PAIR(true, true, true); else FA_PAIR(true, true, false);
  } else if (y0) {
    if (w1) FA_PAIR(true, false, true); else FA_PAIR(true, false, false);
  } else if (y1) {
    if (w1) FA_PAIR(false, true, true); else FA_PAIR(false, true, false);
  } else {
    if (w1) FA_PAIR(false, false, true); else FA_PAIR(false, false, false);
  }
#undef FA_PAIR
  return hipGetLastError();
}

hipError_t launch_chain_pair(const Op& op, const void* x, const void* y0, const void* y1,
                             void* out1, void* out2, const ChainCoef& t1, const ChainCoef& t2,
                             hipStream_t s, Prec pin, Prec pout) {
  if (op.kind != OP_STENCIL7) return hipErrorInvalidValue;
  const PairCoef c{t1.alpha.real(), t1.beta.real(), t1.g0.real(), t1.g1.real(),
                   t2.alpha.real(), t2.beta.real(), t2.g0.real(), t2.g1.real()};
  if (pin == P64 && pout == P64)
    return launch_st7_pair_t<double, double>(op, x, y0, y1, out1, out2, c, s);
  if (pin == P32 && pout == P32)
    return launch_st7_pair_t<float, float>(op, x, y0, y1, out1, out2, c, s);
  if (pin == P32 && pout == P64 && out1 == nullptr)
    return launch_st7_pair_t<float, double>(op, x, y0, y1, out1, out2, c, s);
  return hipErrorInvalidValue;
}

// --------------------------------------------------------------------------
// CSR, real or complex values, as a stream of row blocks (the CSR-stream
// scheme of Greathouse and Daga's CSR-Adaptive, written for 512-thread
// workgroups): at creation the rows are cut into blocks of consecutive rows
// holding at most kCsrBlockEntries entries and kCsrBlockRows rows.  A block's
// workgroup
//   1. loads the block's entries, kCsrPer per thread, coalesced (column
//      index and value of entry e0 + tid + 512 k), gathers x at the columns
//      with all of a thread's loads in flight, and stores the products in LDS;
//   2. sums each row's products out of LDS with a lane group of tr lanes, tr
//      the largest power of two <= 512 / rows (at most 64), in a fixed order,
//      and writes the rows of the block in order (coalesced).
// So every thread has several independent entries in flight instead of one.
// Rows with more than kCsrBlockEntries entries (the tail of a skewed degree
// distribution) are cut into chunks of kCsrBlockEntries: one CU gathers about
// one cache line per clock, so a row of tens of thousands of entries must be
// spread over many CUs.  With scratch for the chunks' partial sums (SPLIT),
// every chunk is a workgroup of its own (the first ones of the launch); the
// workgroup that finishes a row's last chunk adds the row's partial sums in
// chunk order and writes the row, so the result does not depend on the
// order the chunks finish.  Without scratch one workgroup walks all chunks of
// the row and adds the same partial sums in the same order: the same bits.
// --------------------------------------------------------------------------
static_assert(kCsrBlockEntries == kCsrThreads * kCsrPer, "one pass of loads per block or chunk");
static_assert(kCsrBlockRows == kCsrThreads, "at most one row per lane group");
static_assert(kCsrThreads % 64 == 0 && kCsrThreads <= 1024, "whole wavefronts");

// the sum of the products of entries [eb, ee) (at most kCsrBlockEntries) by
// the whole workgroup: per-thread sums in entry order, then the wavefront
// sums, then the 8 wavefront sums in order; every thread returns it.  ws:
// 8 LDS slots, free again when the call returns.
template <typename T>
__device__ __forceinline__ T csr_chunk_sum(const int32_t* __restrict__ colind,
                                           const T* __restrict__ vals, const T* __restrict__ x,
                                           int eb, int ee, T* ws) {
  const int tid = threadIdx.x;
  int c[kCsrPer];
  T v[kCsrPer];
#pragma unroll
  for (int k = 0; k < kCsrPer; ++k) {
    const int e = min(eb + tid + k * kCsrThreads, ee - 1);
    c[k] = colind[e];
    v[k] = vals[e];
  }
  T acc = zero(T{});
#pragma unroll
  for (int k = 0; k < kCsrPer; ++k) {
    const T t = mad(v[k], x[c[k]], acc);
    acc = (eb + tid + k * kCsrThreads < ee) ? t : acc;
  }
  acc = wave_sum(acc);
  if ((tid & 63) == 0) ws[tid >> 6] = acc;
  __syncthreads();
  T t = ws[0];
#pragma unroll
  for (int w = 1; w < kCsrThreads / 64; ++w) t += ws[w];
  __syncthreads();
  return t;
}

__device__ __forceinline__ void agent_store(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void agent_store(cplx* p, cplx v) {
  __hip_atomic_store(&p->x, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&p->y, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double agent_load(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ cplx agent_load(const cplx* p) {
  return {__hip_atomic_load(&p->x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
          __hip_atomic_load(&p->y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)};
}

template <typename T, bool Y0, bool Y1>
__device__ __forceinline__ void csr_write_row(int row, T sum, const T* __restrict__ x,
                                              const T* __restrict__ y0, const T* y1, T* out,
                                              T al, T be, T g0, T g1, bool use_x) {
  T r = al * sum;
  if (use_x) r = mad(be, x[row], r);
  if (Y0) r = mad(g0, y0[row], r);
  if (Y1) r = mad(g1, y1[row], r);
  out[row] = r;
}

// Work tables (operator memory):
//   blk  : per block 4 int32 {r0, r1, e0 = rowptr[r0], e1 = rowptr[r1]}
//   chunk: per chunk of a long row 4 int32 {row, eb, ee, long index}
//   lng  : per long row 3 int32 {row, first chunk, chunks}
// Scratch (SPLIT): the chunks' partial sums, then one counter per long row
// (zero before the launch; the row's last chunk sets it back to zero).
template <typename T, bool Y0, bool Y1, bool SPLIT>
__global__ __launch_bounds__(kCsrThreads) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 || kCsrThreads <= 256 ? 8 : 4))) void csr_chain(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
    const T* __restrict__ vals, const T* __restrict__ x, const T* __restrict__ y0, const T* y1,
    T* out, T al, T be, T g0, T g1, int nfirst, const int4* __restrict__ blk,
    const int4* __restrict__ chunk, const int32_t* __restrict__ lng, T* part, int* cnt) {
  __shared__ T prod[kCsrBlockEntries];
  __shared__ int lrp[kCsrBlockRows + 1];
  __shared__ T ws[kCsrThreads / 64];
  __shared__ int last;
  const int tid = threadIdx.x;
  const bool use_x = !is_zero(be);
  if ((int)blockIdx.x < nfirst) {
    if (SPLIT) {  // one chunk of a long row
      const int4 ck = chunk[blockIdx.x];
      const T sum = csr_chunk_sum(colind, vals, x, ck.y, ck.z, ws);
      const int row = lng[3 * ck.w], c0 = lng[3 * ck.w + 1], nc = lng[3 * ck.w + 2];
      if (tid == 0) {
        agent_store(part + blockIdx.x, sum);
        // release: the partial sum is visible before the count says so
        const int prev = __hip_atomic_fetch_add(cnt + ck.w, 1, __ATOMIC_ACQ_REL,
                                                __HIP_MEMORY_SCOPE_AGENT);
        last = prev == nc - 1;
      }
      __syncthreads();
      if (last && tid == 0) {  // every chunk of the row is done: add them in order
        T t = agent_load(part + c0);
        for (int c = 1; c < nc; ++c) t += agent_load(part + c0 + c);
        csr_write_row<T, Y0, Y1>(row, t, x, y0, y1, out, al, be, g0, g1, use_x);
        __hip_atomic_store(cnt + ck.w, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    } else {  // a whole long row: its chunks one after the other
      const int row = lng[3 * blockIdx.x], c0 = lng[3 * blockIdx.x + 1],
                nc = lng[3 * blockIdx.x + 2];
      T t = zero(T{});
      for (int c = 0; c < nc; ++c) {
        const int4 ck = chunk[c0 + c];
        const T sum = csr_chunk_sum(colind, vals, x, ck.y, ck.z, ws);
        t = (c == 0) ? sum : t + sum;
      }
      if (tid == 0) csr_write_row<T, Y0, Y1>(row, t, x, y0, y1, out, al, be, g0, g1, use_x);
    }
    return;
  }
  const int4 bk = blk[(int)blockIdx.x - nfirst];
  const int r0 = bk.x, R = bk.y - bk.x, e0 = bk.z, ne = bk.w - bk.z;
  // the lane group of this thread and its row (known before any load)
  int tr = 64;
  while (tr > 1 && tr * R > kCsrThreads) tr >>= 1;
  const int gi = tid / tr, li = tid % tr;
  // loads that do not depend on each other, all issued first: this thread's
  // row pointer, the row's epilogue operands, the block's entries
  const int rpv = rowptr[r0 + min(tid, R)] - e0;
  T xr = zero(T{}), y0r = zero(T{}), y1r = zero(T{});
  if (gi < R && li == 0) {
    if (use_x) xr = x[r0 + gi];
    if (Y0) y0r = y0[r0 + gi];
    if (Y1) y1r = y1[r0 + gi];
  }
  if (ne > 0) {
    int c[kCsrPer];
    T v[kCsrPer];
#pragma unroll
    for (int k = 0; k < kCsrPer; ++k) {
      const int e = e0 + min(tid + k * kCsrThreads, ne - 1);
      c[k] = colind[e];
      v[k] = vals[e];
    }
#pragma unroll
    for (int k = 0; k < kCsrPer; ++k) {
      const T t = v[k] * x[c[k]];
      if (tid + k * kCsrThreads < ne) prod[tid + k * kCsrThreads] = t;
    }
  }
  if (tid <= R) lrp[tid] = rpv;
  if (tid == 0) lrp[R] = ne;  // (R may equal the thread count)
  __syncthreads();
  if (gi < R) {  // whole lane groups (tr divides 64) take this branch together
    const int lo = lrp[gi], hi = lrp[gi + 1];
    T acc = zero(T{});
    for (int e = lo + li; e < hi; e += tr) acc += prod[e];
    for (int off = tr / 2; off > 0; off >>= 1) acc += shfl_down(acc, off, tr);
    if (li == 0) {
      T r = al * acc;
      if (use_x) r = mad(be, xr, r);
      if (Y0) r = mad(g0, y0r, r);
      if (Y1) r = mad(g1, y1r, r);
      out[r0 + gi] = r;
    }
  }
}

template <typename T>
__global__ void csr_zero_counters(int* cnt, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) cnt[i] = 0;
}

namespace {
thread_local void* t_op_scratch = nullptr;
}
void* set_op_scratch(void* p) {
  void* old = t_op_scratch;
  t_op_scratch = p;
  return old;
}

size_t op_scratch_bytes(const Op& op) {
  if (op.kind == OP_WILSON && op.q2) return (size_t)round_up(op.n * 16, 256);
  if (op.kind != OP_CSR || op.csr_nlong == 0) return 0;
  return (size_t)round_up((int64_t)op.csr_nchunk * (int64_t)elem_size(op.dtype), 256) +
         (size_t)round_up((int64_t)op.csr_nlong * 4, 256);
}

hipError_t op_scratch_clear(const Op& op, void* scratch, hipStream_t st) {
  if (op.kind != OP_CSR || op.csr_nlong == 0 || !scratch) return hipSuccess;
  int* cnt = (int*)((char*)scratch +
                    round_up((int64_t)op.csr_nchunk * (int64_t)elem_size(op.dtype), 256));
  csr_zero_counters<int><<<(op.csr_nlong + 255) / 256, 256, 0, st>>>(cnt, op.csr_nlong);
  return hipGetLastError();
}

template <typename T, bool Y0, bool Y1>
static void launch_csr_y(const Op& op, const T* x, const T* y0, const T* y1, T* out, T al, T be,
                         T g0, T g1, hipStream_t st) {
  auto rp = op.rowptr;
  auto ci = op.colind;
  auto va = (const T*)op.vals;
  const int4* bk = (const int4*)op.csr_blk_dev;
  const int4* ck = (const int4*)op.csr_chunk_dev;
  const int32_t* lg = op.csr_long_dev;
  void* sc = op.csr_nlong ? t_op_scratch : nullptr;
  if (sc) {
    T* part = (T*)sc;
    int* cnt = (int*)((char*)sc + round_up((int64_t)op.csr_nchunk * (int64_t)sizeof(T), 256));
    const int grid = op.csr_nchunk + op.csr_nblk;
    csr_chain<T, Y0, Y1, true><<<grid, kCsrThreads, 0, st>>>(
        rp, ci, va, x, y0, y1, out, al, be, g0, g1, op.csr_nchunk, bk, ck, lg, part, cnt);
  } else {
    const int grid = op.csr_nlong + op.csr_nblk;
    csr_chain<T, Y0, Y1, false><<<grid, kCsrThreads, 0, st>>>(
        rp, ci, va, x, y0, y1, out, al, be, g0, g1, op.csr_nlong, bk, ck, lg, nullptr, nullptr);
  }
}

template <typename T>
static hipError_t launch_csr(const Op& op, const T* x, const T* y0, const T* y1, T* out,
                             const ChainCoef& k, hipStream_t st) {
  const T al = host_to_dev<T>::conv(k.alpha), be = host_to_dev<T>::conv(k.beta),
          g0 = host_to_dev<T>::conv(k.g0), g1 = host_to_dev<T>::conv(k.g1);
  if (op.csr_nlong + op.csr_nblk == 0) return hipSuccess;
  if (y0 && y1)
    launch_csr_y<T, true, true>(op, x, y0, y1, out, al, be, g0, g1, st);
  else if (y0)
    launch_csr_y<T, true, false>(op, x, y0, y1, out, al, be, g0, g1, st);
  else if (y1)
    launch_csr_y<T, false, true>(op, x, y0, y1, out, al, be, g0, g1, st);
  else
    launch_csr_y<T, false, false>(op, x, y0, y1, out, al, be, g0, g1, st);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Wilson-Dirac-like operator, complex FP64.
//   (D x)(s) = (4 + m0) x(s) - 1/2 sum_mu [(1 - g_mu) U_mu(s) x(s + mu)
//                                         + (1 + g_mu) U_mu(s - mu)^H x(s - mu)]
// Chiral basis: g_k = [[0, -i s_k], [i s_k, 0]] (k = x, y, z), g_t = [[0, I], [I, 0]].
// (1 + sg g_mu), sg = -1 or +1, has rank 2 in spin space: with u, d the upper
// and lower spin pairs, h = u + sg M_mu d and the lower pair of the result is
// sg M_mu^{-1} h, where M_k = -i s_k and M_t = I.  A hop therefore projects the
// 4-spinor to the 2-spinor h, multiplies h by the 3x3 link (6 colour matvecs
// instead of 12) and rebuilds the lower pair from the transported h.
// Every M_mu is diagonal or anti-diagonal with entries in {+-1, +-i}.
//
// Work split: a workgroup of four waves owns 64 consecutive sites; wave mu
// does the forward and the backward hop in direction mu for all of them
// (lane = site), so M_mu, M_mu^{-1} and the hop signs are compile-time
// constants: multiplying by them is a sign change or a swap of real and
// imaginary parts, exact, and no lane holds per-direction coefficients.
// Memory access: a spinor is 192 contiguous bytes, so a lane that read its
// own neighbour's spinor would make every load touch 64 cache lines.  Instead
// the wave stages the 64 neighbours' projected half spinors h (6 complex each)
// in its LDS slice: item p = 64 kk + lane is component p % 6 of neighbour
// p / 6, formed from two 16-byte chunks of that spinor, so the lanes read
// each spinor's upper and lower six chunks as contiguous runs; each lane then
// takes its site's h from the slice.  The four directions' sums are added as
// ((mu 0 + mu 2) + (mu 1 + mu 3)) through LDS and the workgroup writes the
// result with coalesced stores.  The links are kept in a structure-of-arrays
// copy Us[mu][e][s] (made once at creation), so that link element e of 64
// consecutive sites is 1 KB contiguous.
// --------------------------------------------------------------------------
struct Wil {
  int L0, L1, L2, L3;  // x, y, z, t extents
  int V;
  // site-block order (workgroup w -> sites): P blocks of 64 sites per (x, y)
  // plane, T t-slices per XCD (0: lexicographic), ZB z-planes per z-block
  int P, T, ZB;
  double diag;         // 4 + m0
  double ef, eb;       // e^{+mu}, e^{-mu}: the forward / backward temporal hop
};

constexpr int kWilDSites = 64;  // sites per workgroup (one per lane)

// p * a for a compile-time unit p = R + i I in {+-1, +-i}: exact
template <int R, int I>
__device__ __forceinline__ cplx umul(cplx a) {
  static_assert((R == 0) != (I == 0) && R * R + I * I == 1, "a unit");
  if constexpr (R == 1) return a;
  else if constexpr (R == -1) return cplx{-a.x, -a.y};
  else if constexpr (I == 1) return cplx{-a.y, a.x};
  else return cplx{a.y, -a.x};
}

// M_mu (rows 0 and 1 of the lower-to-upper map) and M_mu^{-1}, as above:
// x, y anti-diagonal (-i, -i), (-1, 1); z diagonal (-i, i); t identity
template <int MU> struct WilDir;
template <> struct WilDir<0> {
  static constexpr bool swap = true;
  template <int SP> static __device__ cplx m(cplx a) { return umul<0, -1>(a); }
  template <int SP> static __device__ cplx mi(cplx a) { return umul<0, 1>(a); }
};
template <> struct WilDir<1> {
  static constexpr bool swap = true;
  template <int SP> static __device__ cplx m(cplx a) {
    if constexpr (SP == 0) return umul<-1, 0>(a); else return umul<1, 0>(a);
  }
  template <int SP> static __device__ cplx mi(cplx a) {
    if constexpr (SP == 0) return umul<1, 0>(a); else return umul<-1, 0>(a);
  }
};
template <> struct WilDir<2> {
  static constexpr bool swap = false;
  template <int SP> static __device__ cplx m(cplx a) {
    if constexpr (SP == 0) return umul<0, -1>(a); else return umul<0, 1>(a);
  }
  template <int SP> static __device__ cplx mi(cplx a) {
    if constexpr (SP == 0) return umul<0, 1>(a); else return umul<0, -1>(a);
  }
};
template <> struct WilDir<3> {
  static constexpr bool swap = false;
  template <int SP> static __device__ cplx m(cplx a) { return a; }
  template <int SP> static __device__ cplx mi(cplx a) { return a; }
};

// sg * a for a compile-time sign
template <int SG>
__device__ __forceinline__ cplx sgn(cplx a) {
  if constexpr (SG > 0) return a; else return cplx{-a.x, -a.y};
}

// stage h of the neighbour of every lane's site (nb: this lane's neighbour):
// item p = 64 kk + lane is component (sp, c) = (comp / 3, comp % 3), comp =
// p % 6, of the neighbour of site p / 6: h_sp,c = u_sp,c + sg M_sp d_sp',c
template <int MU, int SG>
__device__ __forceinline__ void wilson_dir_stage(const cplx* __restrict__ x, int nb, int lane,
                                                 double scale, cplx* slice) {
  using D = WilDir<MU>;
  cplx u[6], d[6];
#pragma unroll
  for (int kk = 0; kk < 6; ++kk) {
    const int p = kk * kWilDSites + lane, j = p / 6, comp = p - 6 * j;
    const int sp = comp >= 3 ? 1 : 0, c = comp - 3 * sp;
    const int dsp = D::swap ? 1 - sp : sp;
    const int nbj = __shfl(nb, j, 64);
    const cplx* xs = x + (int64_t)nbj * 12;
    u[kk] = xs[sp * 3 + c];
    d[kk] = xs[(2 + dsp) * 3 + c];
  }
#pragma unroll
  for (int kk = 0; kk < 6; ++kk) {
    const int p = kk * kWilDSites + lane;
    const bool s1 = p % 6 >= 3;
    const cplx md = s1 ? D::template m<1>(d[kk]) : D::template m<0>(d[kk]);
    const cplx h = u[kk] + sgn<SG>(md);
    // the temporal hops carry the chemical potential (x 1 exactly for mu = 0)
    slice[p] = MU == 3 ? scale * h : h;
  }
}

// one hop from the lane's staged h: acc += (1 + sg g_mu) W x(nb)
template <int MU, int SG, bool Adj, bool R12>
__device__ __forceinline__ void wilson_dir_hop(const cplx* hs, const cplx* __restrict__ Ue,
                                               int64_t V, cplx acc[4][3]) {
  using D = WilDir<MU>;
  cplx u[9];
#pragma unroll
  for (int e = 0; e < (R12 ? 6 : 9); ++e) u[e] = Ue[e * V];
  if (R12) {
    u[6] = conjg(u[1] * u[5] - u[2] * u[4]);
    u[7] = conjg(u[2] * u[3] - u[0] * u[5]);
    u[8] = conjg(u[0] * u[4] - u[1] * u[3]);
  }
  cplx h[2][3];
#pragma unroll
  for (int sp = 0; sp < 2; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) h[sp][c] = hs[sp * 3 + c];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    cplx g[2];
#pragma unroll
    for (int sp = 0; sp < 2; ++sp) {
      if (Adj)  // (U^H h)_a = sum_b conj(U_ba) h_b
        g[sp] = cmad(u[2 * 3 + a], h[sp][2],
                     cmad(u[1 * 3 + a], h[sp][1], cmad(u[0 * 3 + a], h[sp][0], cplx{0.0, 0.0})));
      else
        g[sp] = mad(u[a * 3 + 2], h[sp][2], mad(u[a * 3 + 1], h[sp][1], u[a * 3 + 0] * h[sp][0]));
    }
    acc[0][a] += g[0];
    acc[1][a] += g[1];
    const cplx f0 = D::swap ? g[1] : g[0], f1 = D::swap ? g[0] : g[1];
    acc[2][a] += sgn<SG>(D::template mi<0>(f0));
    acc[3][a] += sgn<SG>(D::template mi<1>(f1));
  }
}

template <int MU, bool R12>
__device__ __forceinline__ void wilson_dir_body(const Wil& w, const cplx* __restrict__ Us,
                                                const cplx* __restrict__ x, int s, int lane,
                                                cplx* slice, cplx acc[4][3]) {
  int c0, c1, c2, c3;
  {
    int r = s;
    c0 = r % w.L0; r /= w.L0;
    c1 = r % w.L1; r /= w.L1;
    c2 = r % w.L2;
    c3 = r / w.L2;
  }
  const int L = MU == 0 ? w.L0 : MU == 1 ? w.L1 : MU == 2 ? w.L2 : w.L3;
  const int co = MU == 0 ? c0 : MU == 1 ? c1 : MU == 2 ? c2 : c3;
  const int st = MU == 0 ? 1 : MU == 1 ? w.L0 : MU == 2 ? w.L0 * w.L1 : w.L0 * w.L1 * w.L2;
  const int sf = (co + 1 < L) ? s + st : s - (L - 1) * st;
  const int sb = (co > 0) ? s - st : s + (L - 1) * st;
  constexpr int NE = R12 ? 6 : 9;  // link elements stored per site and direction
  const cplx* Um = Us + (int64_t)MU * NE * w.V;
  const cplx* mine = slice + lane * 6;
  // forward hop: (1 - g_mu) U_mu(s) x(s + mu)
  wilson_dir_stage<MU, -1>(x, sf, lane, w.ef, slice);
  __builtin_amdgcn_wave_barrier();
  wilson_dir_hop<MU, -1, false, R12>(mine, Um + s, w.V, acc);
  __builtin_amdgcn_wave_barrier();
  // backward hop: (1 + g_mu) U_mu(s - mu)^H x(s - mu)
  wilson_dir_stage<MU, 1>(x, sb, lane, w.eb, slice);
  __builtin_amdgcn_wave_barrier();
  wilson_dir_hop<MU, 1, true, R12>(mine, Um + sb, w.V, acc);
}

// out = al G (D x) + be xb + g0 y0 + g1 y1, G = Gamma_5 (G5) or I; xb is x
// itself except in the second product of a Q^2 term
template <bool Y0, bool Y1, bool R12, bool G5>
__global__ __launch_bounds__(256) void wilson_dir_k(Wil w, const cplx* __restrict__ Us,
                                                    const cplx* __restrict__ x,
                                                    const cplx* __restrict__ xb,
                                                    const cplx* __restrict__ y0,
                                                    const cplx* y1, cplx* out, cplx al,
                                                    cplx be, cplx g0, cplx g1) {
  // four slices of 64 x 6 staged values; after the hops the same memory
  // holds two 64 x 12 partial sums
  __shared__ cplx lds[4 * kWilDSites * 6];
  constexpr int kAcc = kWilDSites * 12;
  const int lane = threadIdx.x & 63;
  const int mu = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // each XCD takes one contiguous range of sites: T whole t-slices when the
  // lattice allows it, walked in the order (z-block, xy-block, t, z within
  // the block), so that the t- and z-neighbours of a workgroup's sites are
  // read by workgroups the same XCD runs at about the same time (its L2);
  // otherwise the lexicographic order
  int blk = xcd_contiguous(blockIdx.x, gridDim.x);
  if (w.T > 0) {
    const int per = w.P * w.L2 * w.T;
    const int xc = blk / per, r = blk - xc * per;
    const int zi = r % w.ZB, r2 = r / w.ZB;
    const int tr = r2 % w.T, r3 = r2 / w.T;
    const int xy = r3 % w.P, z = (r3 / w.P) * w.ZB + zi;
    blk = ((xc * w.T + tr) * w.L2 + z) * w.P + xy;
  }
  const int s0 = blk * kWilDSites;
  const int nsite = min(kWilDSites, w.V - s0);
  // lanes past the last site work on site V - 1 and store nothing
  const int s = min(s0 + lane, w.V - 1);
  cplx acc[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[a][c] = cplx{0.0, 0.0};
  cplx* slice = lds + mu * kWilDSites * 6;
  switch (mu) {
    case 0: wilson_dir_body<0, R12>(w, Us, x, s, lane, slice, acc); break;
    case 1: wilson_dir_body<1, R12>(w, Us, x, s, lane, slice, acc); break;
    case 2: wilson_dir_body<2, R12>(w, Us, x, s, lane, slice, acc); break;
    default: wilson_dir_body<3, R12>(w, Us, x, s, lane, slice, acc); break;
  }
  // (mu 0 + mu 2) + (mu 1 + mu 3), element (site, 3 row + colour)
  __syncthreads();
  if (mu >= 2) {
    cplx* R = lds + (mu - 2) * kAcc;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) R[lane * 12 + a * 3 + c] = acc[a][c];
  }
  __syncthreads();
  if (mu < 2) {
    const cplx* R = lds + mu * kAcc;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[a][c] += R[lane * 12 + a * 3 + c];
  }
  __syncthreads();
  if (mu == 1) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) lds[lane * 12 + a * 3 + c] = acc[a][c];
  }
  __syncthreads();
  if (mu == 0) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int e = lane * 12 + a * 3 + c;
        lds[kAcc + e] = acc[a][c] + lds[e];
      }
  }
  __syncthreads();
  // out = al G (diag x - sum / 2) + be xb + g0 y0 + g1 y1, value by value
  // (value q of a site is spin q % 12 / 3: Gamma_5 negates spins 2 and 3)
  const int64_t base = (int64_t)s0 * 12;
  const cplx* S = lds + kAcc;
#pragma unroll
  for (int i = 0; i < kAcc / 256; ++i) {
    const int q = threadIdx.x + 256 * i;
    if (q < nsite * 12) {
      const cplx xc = x[base + q];
      cplx dx = w.diag * xc - 0.5 * S[q];
      if (G5 && q % 12 >= 6) dx = cplx{-dx.x, -dx.y};
      cplx r = mad(al, dx, be * (G5 ? xb[base + q] : xc));
      if (Y0) r = mad(g0, y0[base + q], r);
      if (Y1) r = mad(g1, y1[base + q], r);
      out[base + q] = r;
    }
  }
}

static hipError_t launch_wilson(const Op& op, const cplx* x, const cplx* y0, const cplx* y1,
                                cplx* out, const ChainCoef& k, hipStream_t st) {
  const int plane = op.dims[0] * op.dims[1];
  const bool zt = plane % kWilDSites == 0 && op.dims[3] % kXcds == 0;
  const int zb = op.dims[2] % 2 == 0 ? 2 : 1;
  Wil w{op.dims[0], op.dims[1], op.dims[2], op.dims[3],
        op.dims[0] * op.dims[1] * op.dims[2] * op.dims[3],
        zt ? plane / kWilDSites : 0, zt ? op.dims[3] / kXcds : 0, zb,
        4.0 + op.m0, std::exp(op.mu), std::exp(-op.mu)};
  const cplx al = host_to_dev<cplx>::conv(k.alpha), be = host_to_dev<cplx>::conv(k.beta),
             g0 = host_to_dev<cplx>::conv(k.g0), g1 = host_to_dev<cplx>::conv(k.g1);
  const cplx* U = (const cplx*)op.links;
  const int grid = (w.V + kWilDSites - 1) / kWilDSites;
  // Q^2: t = Gamma_5 D x into the operator scratch, then out = al Gamma_5 D t
  // + be x + g0 y0 + g1 y1
  const cplx* hx = x;  // the vector the hops of the (last) product read
  if (op.q2) {
    cplx* t = (cplx*)t_op_scratch;
    if (!t) return hipErrorInvalidValue;
    const cplx one{1.0, 0.0}, zero{0.0, 0.0};
    if (op.links_rows == 2)
      wilson_dir_k<false, false, true, true><<<grid, 256, 0, st>>>(w, U, x, x, nullptr, nullptr,
                                                                   t, one, zero, zero, zero);
    else
      wilson_dir_k<false, false, false, true><<<grid, 256, 0, st>>>(w, U, x, x, nullptr, nullptr,
                                                                    t, one, zero, zero, zero);
    hx = t;
  }
#define FA_WIL(A, B, R)                                                                         \
  do {                                                                                          \
    if (op.q2)                                                                                  \
      wilson_dir_k<A, B, R, true><<<grid, 256, 0, st>>>(w, U, hx, x, y0, y1, out, al, be, g0, g1);  \
    else                                                                                        \
      wilson_dir_k<A, B, R, false><<<grid, 256, 0, st>>>(w, U, hx, x, y0, y1, out, al, be, g0, g1); \
  } while (0)
#define FA_WIL_R(A, B)  \
  if (op.links_rows == 2) \
    FA_WIL(A, B, true);   \
  else                    \
    FA_WIL(A, B, false)
  if (y0 && y1) {
    FA_WIL_R(true, true);
  } else if (y0) {
    FA_WIL_R(true, false);
  } else if (y1) {
    FA_WIL_R(false, true);
  } else {
    FA_WIL_R(false, false);
  }
#undef FA_WIL_R
#undef FA_WIL
  return hipGetLastError();
}

// Us[mu][e][s] = U[mu][s][e] for the 4 directions, the first ne of the 9
// link elements (row-major: 9 = all, 6 = rows 0 and 1), V sites
__global__ void wilson_links_soa_k(int64_t V, int ne, const cplx* __restrict__ U,
                                   cplx* __restrict__ Us) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // over Us
  if (i >= 4 * ne * V) return;
  const int64_t s = i % V, me = i / V, mu = me / ne, e = me - ne * mu;
  Us[i] = U[(mu * V + s) * 9 + e];
}

hipError_t launch_wilson_links_soa(int64_t V, int ne, const void* U, void* Us, hipStream_t st) {
  if (ne != 6 && ne != 9) return hipErrorInvalidValue;
  const int64_t n = 4 * ne * V;
  wilson_links_soa_k<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(V, ne, (const cplx*)U,
                                                                 (cplx*)Us);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
hipError_t launch_chain(const Op& op, const void* x, const void* y0, const void* y1, void* out,
                        const ChainCoef& k, hipStream_t s, Prec pin, Prec pout) {
  if ((pin != P64 || pout != P64 || op.nbatch > 1) && op.kind != OP_STENCIL7)
    return hipErrorInvalidValue;
  switch (op.kind) {
    case OP_STENCIL7:
      return launch_st7(op, x, y0, y1, out, k, s, pin, pout);
    case OP_CSR:
      if (op.dtype == FA_C128)
        return launch_csr<cplx>(op, (const cplx*)x, (const cplx*)y0, (const cplx*)y1,
                                (cplx*)out, k, s);
      return launch_csr<double>(op, (const double*)x, (const double*)y0, (const double*)y1,
                                (double*)out, k, s);
    case OP_WILSON:
      return launch_wilson(op, (const cplx*)x, (const cplx*)y0, (const cplx*)y1, (cplx*)out, k,
                           s);
  }
  return hipErrorInvalidValue;
}

double chain_pair_bytes(const Op& op, bool has_y0, bool has_y1, bool has_out1, Prec p) {
  const double vec = (double)op.n * (p == P32 ? 4.0 : (double)elem_size(op.dtype));
  return vec * (2.0 + (has_y0 ? 1.0 : 0.0) + (has_y1 ? 1.0 : 0.0) + (has_out1 ? 1.0 : 0.0));
}

double chain_bytes(const Op& op, bool has_y0, bool has_y1, Prec p) {
  const double vec = (double)op.n * (p == P32 ? 4.0 : (double)elem_size(op.dtype));
  const double nvec = 2.0 + (has_y0 ? 1.0 : 0.0) + (has_y1 ? 1.0 : 0.0);
  double extra = 0.0;
  if (op.kind == OP_CSR)
    extra = (double)(op.n + 1) * 4 + (double)op.nnz * (4 + elem_size(op.dtype));
  if (op.kind == OP_WILSON) extra = 4.0 * (double)(op.n / 12) * (3 * op.links_rows) * 16;
  if (op.kind == OP_WILSON && op.q2) {  // two products: x -> t, then t (and x) -> out
    extra *= 2.0;
    return (nvec + 3.0) * vec + extra;
  }
  return nvec * vec + extra;
}

}  // namespace fa
