// Temporal blocking of a polynomial recurrence on the 7-point stencil: NT
// consecutive terms of
//     s_t = a_t A s_{t-1} + b_t s_{t-1} + g0_t v + g1_t s_{t-2},   t = 1..NT,
// with s_0 = x and s_{-1} = y1, in one launch (the Clenshaw recurrence of a
// Chebyshev polynomial, Sec. 5.1: s_{t-2} is b_{k+2}, v the vector q(A) acts
// on).  Memory sees x, y1 and v read and s_{NT-1}, s_NT written: 5 vector
// passes for NT terms (NT = 4: 5/4 per term, NT = 3: 5/3, against 5/2 for two
// terms and 4 for one).  The intermediate terms never leave the chip.  NT = 4
// in FP64 takes 79.9 KB of LDS and 124 VGPRs: two workgroups per CU.
//
// A workgroup owns a TW x TY tile of the (x, y) plane (64 x 8, 32 x 16 or
// 56 x 8, whichever wastes the fewest points along x) and marches through its slab of kz
// planes in z.  Term t is needed on the tile grown by NT - t
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
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "devmath.hpp"
#include "fa_internal.hpp"


#ifndef FA_MULTI_BLOCKS
#define FA_MULTI_BLOCKS 512
#endif
// LDS row pitch beyond the region width: 2 elements (72 -> 74 doubles for
// the 64 x 8 tile) move the ring's column points, 16 dwords apart per row
// at pitch 72, onto more banks (29.7 -> 29.4 us per 128^3 launch)
#ifndef FA_MULTI_LDS_PAD
#define FA_MULTI_LDS_PAD 2
#endif
// Two workgroups share each CU, and the one dispatched first gets more of it:
// on 128^3 (8-plane slabs) the first finished its slab in 22.5 us, the
// second in 28.4, so the launch waited on the second.  Slabs are therefore
// paired on a CU with the first one FA_MULTI_PAIR_SHIFT planes longer (10
// and 6 planes: 25.3 and 27.4 us; the solve 137.5 -> 140.7 solves/s)
#ifndef FA_MULTI_PAIR_SHIFT
#define FA_MULTI_PAIR_SHIFT 2
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

template <int NT, int TW, int TY>
struct Geo {
  static constexpr int TX = TW, P = TX * TY;
  // region of term t: the tile grown by NT - t on each side
  static constexpr int W(int t) { return TX + 2 * (NT - t); }
  static constexpr int H(int t) { return TY + 2 * (NT - t); }
  static constexpr int N(int t) { return W(t) * H(t); }
  static constexpr int RING = N(1) - P;   // region 1 minus the tile
  static constexpr int HALO = N(0) - N(1);  // region 0 minus region 1 (x only)
  // LDS row pitch (elements)
  static constexpr int RP = W(0) + FA_MULTI_LDS_PAD;
  // LDS (elements): two plane buffers of region-0 size for x and for each of
  // the terms 1 .. NT-1, then one slot per thread for lanes with nothing to
  // store
  static constexpr int BUF = H(0) * RP;
  static constexpr int DUMMY = 2 * NT * BUF;
  static constexpr int total() { return DUMMY + P; }
};

// (a, b) coordinates in region 1 of ring point h (region 1 minus the tile):
// NT - 1 rows above and below the tile, NT - 1 columns left and right
template <int NT, int TW, int TY>
__device__ __forceinline__ void ring_point(int h, int& a, int& b) {
  using G = Geo<NT, TW, TY>;
  constexpr int w = NT - 1, W1 = G::W(1);
  if (h < w * W1) {  // rows above
    a = h % W1;
    b = h / W1;
  } else if (h < 2 * w * W1) {  // rows below
    const int k = h - w * W1;
    a = k % W1;
    b = w + TY + k / W1;
  } else {  // columns left and right of the tile rows
    const int k = h - 2 * w * W1;
    const int side = k / (w * TY), r = k % (w * TY);
    a = (side == 0 ? 0 : w + G::TX) + r % w;
    b = w + r / w;
  }
}

template <typename T, typename TX, typename TO, int NT, int TW, int TY, bool Y1G, bool W1>
// at least 4 waves per SIMD: two 512-thread workgroups per CU
__global__ __launch_bounds__(TW * TY) __attribute__((amdgpu_waves_per_eu(4))) void st7_multi(
    St7M g, int kz, int gx, int gy, int nwg, int pd, int64_t bstride, const TX* __restrict__ x,
    const TX* __restrict__ v, const TX* __restrict__ y1, TO* __restrict__ out1,
    TO* __restrict__ out2, MultiCoef<NT> cd) {
  using G = Geo<NT, TW, TY>;
  static_assert(G::RING <= G::P && G::HALO <= G::P, "one ring and one halo point per thread");
  constexpr int W0 = G::W(0), RP = G::RP;
  __shared__ T lds[G::total()];
  const T c0 = (T)g.c0, cxm = (T)g.cxm, cxp = (T)g.cxp, cym = (T)g.cym, cyp = (T)g.cyp,
          czm = (T)g.czm, czp = (T)g.czp;
  // a batch of vectors (bstride elements apart): vector blockIdx.y
  const int col = blockIdx.y, lid = xcd_contiguous(blockIdx.x, nwg);
  {
    const int64_t o = (int64_t)col * bstride;
    x += o;
    v += o;
    if (Y1G) y1 += o;
    if (W1) out1 += o;
    out2 += o;
  }
  int bx, by, bz;
  if (pd >= 0) {
    // paired slabs: the two workgroups that share a CU (the k-th and the
    // (k + 32)-th an XCD receives) take slabs 2p and 2p + 1 of one column,
    // the first one pd planes more (it gets more of the CU)
    const int xc = lid / 64, k = lid % 64, G = gx * gy / 32;
    const int cid = (xc % G) * 32 + (k & 31);
    bx = cid % gx;
    by = cid / gx;
    bz = 2 * (xc / G) + (k >> 5);
  } else {
    bx = lid % gx;
    by = (lid / gx) % gy;
    bz = lid / (gx * gy);
  }
  const int i0 = bx * G::TX, j0 = by * TY;
  const int k0 = pd >= 0 ? (bz >> 1) * 2 * kz + ((bz & 1) ? kz + pd : 0) : bz * kz;
  const int k1 = min(pd >= 0 ? (bz >> 1) * 2 * kz + ((bz & 1) ? 2 * kz : kz + pd) : k0 + kz, g.nz);
  const int tid = threadIdx.x;
  const int64_t plane = (int64_t)g.nx * g.ny;

  // Two points per thread: u = 0 its tile point, u = 1 a point of the ring
  // of region 1 around the tile (threads past the ring size repeat ring
  // point 0 and store into their LDS dummy slot).  Every term is computed on
  // every owned point, so no lane takes a branch of its own: a term t value
  // outside region t is not valid (its neighbours lie outside what term t - 1
  // has), but only region t of it is ever read.  Points outside the grid
  // are set to zero; their loads read a clamped in-grid address.
  int ci[2];        // LDS index (region-0 layout) of the point, or the dummy slot
  bool ing[2];      // inside the grid
  int64_t soff[2];  // in-plane offset of the point (clamped into the grid)
  {
    int a[2], b[2];
    a[0] = tid % G::TX + (NT - 1);
    b[0] = tid / G::TX + (NT - 1);
    ring_point<NT, TW, TY>(tid < G::RING ? tid : 0, a[1], b[1]);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int i = i0 - (NT - 1) + a[u], j = j0 - (NT - 1) + b[u];
      ing[u] = i >= 0 && i < g.nx && j >= 0 && j < g.ny;
      soff[u] = (int64_t)min(max(j, 0), g.ny - 1) * g.nx + min(max(i, 0), g.nx - 1);
      ci[u] = (b[u] + 1) * RP + (a[u] + 1);
    }
    if (tid >= G::RING) ci[1] = G::DUMMY + tid;
  }
  // one point of region 0 outside region 1 per thread tid < HALO (x only)
  int hci = G::DUMMY + tid;
  bool hing = false;
  int64_t hoff = 0;
  {
    const int h = tid < G::HALO ? tid : 0;
    int xa, ya;
    if (h < W0) {
      xa = h;
      ya = 0;
    } else if (h < 2 * W0) {
      xa = h - W0;
      ya = G::H(0) - 1;
    } else if (h < 2 * W0 + G::H(1)) {
      xa = 0;
      ya = 1 + (h - 2 * W0);
    } else {
      xa = W0 - 1;
      ya = 1 + (h - 2 * W0 - G::H(1));
    }
    if (tid < G::HALO) hci = ya * RP + xa;
    const int i = i0 - NT + xa, j = j0 - NT + ya;
    hing = i >= 0 && i < g.nx && j >= 0 && j < g.ny;
    hoff = (int64_t)min(max(j, 0), g.ny - 1) * g.nx + min(max(i, 0), g.nx - 1);
  }
  auto zin = [&](int p) { return p >= 0 && p < g.nz; };
  // steps q0 .. qlast; the loop runs an even number of steps (unrolled by
  // two), the extra one computing nothing (its planes are past the slab's)
  const int q0 = k0 - NT + 1, qlast = k1 + NT - 2;
  const int qend = q0 + ((qlast - q0 + 2) & ~1) - 1;

  // rings: ring[s][k][u] = term s at owned point u, produced two steps ago
  // (k = 0), one step ago (k = 1), this step (k = 2); s = 0 is x
  T ring[NT][3][2];
  T vr[NT][2];  // v at planes q, q - 1, .., q - NT + 1
#pragma unroll
  for (int s = 0; s < NT; ++s)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      ring[s][0][u] = ring[s][1][u] = ring[s][2][u] = T(0);
      vr[s][u] = T(0);
    }

  // Loads in flight, two steps ahead, in two slots: step q consumes slot
  // q - q0 mod 2 (x at plane q + 1, v and y1 at plane q) and refills it for
  // step q + 2.  The loop is unrolled by two so that the slot is fixed at
  // compile time: a register that a load is still filling is never copied
  // (a copy would make the wave wait for the load then and there), and the
  // loads read a clamped plane and point, the zero of points and planes
  // outside the grid being applied only when the value is used.
  T xq[2][2], xhq[2], vq[2][2], yq[2][2];
  auto plane_off = [&](int p) { return (int64_t)min(max(p, 0), g.nz - 1) * plane; };
  // (past the last plane the slab needs, the loads repeat that plane: they
  // stay unconditional, so no slot register is ever merged with an older
  // value, which would cost a copy and the wait it implies)
  auto issue = [&](int qs, auto slot) {
    constexpr int S = decltype(slot)::value;
    const TX* xp = x + plane_off(min(qs + 1, k1 + NT - 1));
    const TX* vp = v + plane_off(min(qs, qlast));
    const TX* yp = y1 + plane_off(min(qs, qlast));
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      xq[S][u] = (T)xp[soff[u]];
      vq[S][u] = (T)vp[soff[u]];
      yq[S][u] = Y1G ? (T)yp[soff[u]] : T(0);
    }
    xhq[S] = (T)xp[hoff];
  };
  // x plane p at the owned points and the halo point, zero outside the grid
  // (used right away: the prologue)
  auto load_x = [&](int p, T* r, T& h) {
    const TX* xp = x + plane_off(p);
    const bool z = zin(p);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const T w = (T)xp[soff[u]];
      r[u] = (z && ing[u]) ? w : T(0);
    }
    const T w = (T)xp[hoff];
    h = (z && hing) ? w : T(0);
  };
  // x plane p into its LDS buffer
  auto put_x = [&](int p, const T* r, T h) {
    T* X = lds + (p & 1) * G::BUF;
    const int dummy_shift = (p & 1) * G::BUF;  // keep dummy slots where they are
    X[ci[0]] = r[0];
    X[ci[1] - (ci[1] >= G::DUMMY ? dummy_shift : 0)] = r[1];
    X[hci - (hci >= G::DUMMY ? dummy_shift : 0)] = h;
  };

  // prologue: x(q0 - 1) and x(q0) in the ring, x(q0) in LDS, the loads of
  // the first two steps in flight
  {
    T t0[2], t1[2], h1;
    load_x(q0 - 1, t0, h1);
    load_x(q0, t1, h1);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      ring[0][0][u] = t0[u];
      ring[0][1][u] = t1[u];
    }
    put_x(q0, t1, h1);
  }
  issue(q0, std::integral_constant<int, 0>());
  issue(q0 + 1, std::integral_constant<int, 1>());
  __syncthreads();

  auto step = [&](int q, auto slot) {
    constexpr int S = decltype(slot)::value;
    // term 0: x(q + 1) into the ring and LDS; v, y1 at plane q into use
    const bool zx = zin(q + 1), zv = zin(q);
    T xc[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      xc[u] = (zx && ing[u]) ? xq[S][u] : T(0);
      ring[0][2][u] = xc[u];
    }
    put_x(q + 1, xc, (zx && hing) ? xhq[S] : T(0));
    T ycur[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
      for (int s = NT - 1; s > 0; --s) vr[s][u] = vr[s - 1][u];
      vr[0][u] = (zv && ing[u]) ? vq[S][u] : T(0);
      ycur[u] = (zv && ing[u]) ? yq[S][u] : T(0);
    }
    // the slot's loads for step q + 2, kept after the reads of the slot (a
    // load scheduled above them would need another register and a copy)
    __builtin_amdgcn_sched_barrier(0);
    issue(q + 2, slot);

    // terms 1 .. NT (the last one on the tile points only)
#pragma unroll
    for (int t = 1; t <= NT; ++t) {
      const int p = q - t + 1;
      if (p >= max(k0 - (NT - t), 0) && p < min(k1 + (NT - t), g.nz)) {
        const T a = (T)cd.a[t - 1], b = (T)cd.b[t - 1], e0 = (T)cd.g0[t - 1],
                e1 = (T)cd.g1[t - 1];
        // in-plane neighbours of s_{t-1} at plane p (written at step q - 1)
        const T* L = lds + (t - 1) * 2 * G::BUF + (p & 1) * G::BUF;
        const bool outp = p >= k0 && p < k1;
        const int64_t po = (int64_t)p * plane;
#pragma unroll
        for (int u = 0; u < (t == NT ? 1 : 2); ++u) {
          const int c = u == 0 ? ci[0] : (ci[1] >= G::DUMMY ? RP + 1 : ci[1]);
          const T sv = ring[t - 1][1][u];
          T as = c0 * sv;
          as = fma(czm, ring[t - 1][0][u], as);
          as = fma(czp, ring[t - 1][2][u], as);
          as = fma(cxm, L[c - 1], as);
          as = fma(cxp, L[c + 1], as);
          as = fma(cym, L[c - RP], as);
          as = fma(cyp, L[c + RP], as);
          T val = fma(a, as, b * sv);
          val = fma(e0, vr[t - 1][u], val);
          if (t == 1) {
            if (Y1G) val = fma(e1, ycur[u], val);
          } else {
            val = fma(e1, ring[t - 2][0][u], val);
          }
          val = ing[u] ? val : T(0);
          if (t < NT) {
            ring[t][2][u] = val;
            T* D = lds + t * 2 * G::BUF + (p & 1) * G::BUF;
            D[ci[u] - (ci[u] >= G::DUMMY ? t * 2 * G::BUF + (p & 1) * G::BUF : 0)] = val;
          }
          if (u == 0 && outp && ing[0]) {
            if (t == NT) out2[po + soff[0]] = (TO)val;
            if (W1 && t == NT - 1) out1[po + soff[0]] = (TO)val;
          }
        }
      } else if (t < NT) {
        ring[t][2][0] = ring[t][2][1] = T(0);
      }
    }
    __syncthreads();  // this step's planes visible; last step's buffers free
#pragma unroll
    for (int s = 0; s < NT; ++s)
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        ring[s][0][u] = ring[s][1][u];
        ring[s][1][u] = ring[s][2][u];
      }
  };
  for (int q = q0; q <= qend; q += 2) {
    step(q, std::integral_constant<int, 0>());
    step(q + 1, std::integral_constant<int, 1>());
  }
}

template <typename T, typename TX, typename TO, int NT, int TW, int TY>
hipError_t launch_multi_t(const Op& op, const void* x, const void* v, const void* y1, void* out1,
                          void* out2, const MultiCoef<NT>& c, int blocks, hipStream_t st,
                          hipEvent_t ev0, hipEvent_t ev1) {
  St7M g{op.dims[0], op.dims[1], op.dims[2], op.coef[0], op.coef[1], op.coef[2],
         op.coef[3], op.coef[4], op.coef[5], op.coef[6]};
  const int gx = (g.nx + TW - 1) / TW, gy = (g.ny + TY - 1) / TY;
  // about `blocks` workgroups over the batch
  const int nb = std::max(1, op.nbatch);
  int gz = (int)std::max<int64_t>(
      1, std::min<int64_t>(g.nz / 2, blocks / ((int64_t)gx * gy * nb)));
  const int kz = (g.nz + gz - 1) / gz;
  gz = (g.nz + kz - 1) / kz;
  const int nwg = gx * gy * gz;
  // paired slabs (see the kernel) where the grid is two workgroups on each
  // of the 256 CUs, 32 per XCD, and every XCD takes whole slab pairs of 32
  // columns
  const int pd = (nb == 1 && nwg == 512 && (gx * gy) % 32 == 0 && gz % 2 == 0 &&
                  FA_MULTI_PAIR_SHIFT < kz)
                     ? FA_MULTI_PAIR_SHIFT
                     : -1;
  const dim3 grid(nwg, nb), block(TW * TY);
  const int64_t bs = nb > 1 ? op.bstride : 0;
  const TX* xp = (const TX*)x;
  const TX* vp = (const TX*)v;
  const TX* yp = (const TX*)y1;
  TO* o1 = (TO*)out1;
  TO* o2 = (TO*)out2;
  // the events (if any) take the start and end time of this dispatch itself
#define FA_MULTI(A, B)                                                                          \
  hipExtLaunchKernelGGL(st7_multi<T, TX, TO, NT, TW, TY, A, B>, grid, block, 0, st, ev0, ev1, 0, g, kz, \
                        gx, gy, nwg, pd, bs, xp, vp, yp, o1, o2, c)
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

template <int NT>
static hipError_t launch_multi_nt(const Op& op, const void* x, const void* v, const void* y1,
                                  void* out1, void* out2, const ChainCoef* k, hipStream_t s,
                                  Prec pin, Prec pout, int blocks, hipEvent_t e0, hipEvent_t e1) {
  MultiCoef<NT> c;
  for (int t = 0; t < NT; ++t) {
    c.a[t] = k[t].alpha.real();
    c.b[t] = k[t].beta.real();
    c.g0[t] = k[t].g0.real();
    c.g1[t] = k[t].g1.real();
  }
  // the tile that wastes the fewest points along x: 64 x 8, else 32 x 16
  // (nx = 96: three tiles of 32 instead of two of 64, the second half
  // empty), else 56 x 8 (448 threads; nx = 100: two tiles of 56 instead of
  // two of 64 or four of 32)
  const int nx = op.dims[0];
  auto waste = [nx](int w) { return (nx + w - 1) / w * w - nx; };
  const int tile = waste(64) <= std::min(waste(32), waste(56)) ? 64
                   : waste(32) <= waste(56)                     ? 32
                                                                : 56;
#define FA_MULTI_TILE(T_, TX_, TO_)                                                            \
  return tile == 64 ? launch_multi_t<T_, TX_, TO_, NT, 64, 8>(op, x, v, y1, out1, out2, c,     \
                                                              blocks, s, e0, e1)               \
         : tile == 32 ? launch_multi_t<T_, TX_, TO_, NT, 32, 16>(op, x, v, y1, out1, out2, c,  \
                                                                 blocks, s, e0, e1)            \
                      : launch_multi_t<T_, TX_, TO_, NT, 56, 8>(op, x, v, y1, out1, out2, c,   \
                                                                blocks, s, e0, e1)
  if (pin == P64 && pout == P64) FA_MULTI_TILE(double, double, double);
  if (pin == P32 && pout == P32) FA_MULTI_TILE(float, float, float);
  if (pin == P32 && pout == P64 && out1 == nullptr) FA_MULTI_TILE(float, float, double);
#undef FA_MULTI_TILE
  return hipErrorInvalidValue;
}

hipError_t launch_chain_multi(const Op& op, int nt, const void* x, const void* v, const void* y1,
                              void* out1, void* out2, const ChainCoef* k, hipStream_t s,
                              Prec pin, Prec pout, int blocks, hipEvent_t ev0, hipEvent_t ev1) {
  if (op.kind != OP_STENCIL7 || !x || !v || !out2) return hipErrorInvalidValue;
  if (blocks <= 0) blocks = op.multi_blocks > 0 ? op.multi_blocks : FA_MULTI_BLOCKS;
  if (nt == 3)
    return launch_multi_nt<3>(op, x, v, y1, out1, out2, k, s, pin, pout, blocks, ev0, ev1);
  if (nt == 4)
    return launch_multi_nt<4>(op, x, v, y1, out1, out2, k, s, pin, pout, blocks, ev0, ev1);
  return hipErrorInvalidValue;
}

}  // namespace fa
