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
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_contiguous(int bid, int nwg) {
  const int per = nwg / kXcds, rem = nwg % kXcds;
  const int xcd = bid % kXcds, k = bid / kXcds;
  return (xcd < rem) ? xcd * (per + 1) + k : rem * (per + 1) + (xcd - rem) * per + k;
}

template <bool Y0, bool Y1>
__global__ __launch_bounds__(ST_TX* ST_TY) void st7_chain(St7 s, int kz, int gx, int gy, int nwg,
                                                          const double* __restrict__ x,
                                                          const double* __restrict__ y0,
                                                          const double* y1, double* out,
                                                          double al, double be, double g0,
                                                          double g1) {
  const int lid = xcd_contiguous(blockIdx.x, nwg);
  const int bx = lid % gx, by = (lid / gx) % gy, bz = lid / (gx * gy);
  const int i = bx * ST_TX + (threadIdx.x & (ST_TX - 1));
  const int j = by * ST_TY + (threadIdx.x / ST_TX);
  const int k0 = bz * kz;
  const int k1 = min(k0 + kz, s.nz);
  if (i >= s.nx || j >= s.ny || k0 >= s.nz) return;
  const int64_t plane = (int64_t)s.nx * s.ny;
  int64_t p = (int64_t)k0 * plane + (int64_t)j * s.nx + i;
  const bool hx0 = i > 0, hx1 = i + 1 < s.nx, hy0 = j > 0, hy1 = j + 1 < s.ny;
  double xz0 = (k0 > 0) ? x[p - plane] : 0.0;
  double xc = x[p];
  for (int k = k0; k < k1; ++k, p += plane) {
    const double xz1 = (k + 1 < s.nz) ? x[p + plane] : 0.0;
    double ax = s.c0 * xc;
    ax = fma(s.czm, xz0, ax);
    ax = fma(s.czp, xz1, ax);
    if (hx0) ax = fma(s.cxm, x[p - 1], ax);
    if (hx1) ax = fma(s.cxp, x[p + 1], ax);
    if (hy0) ax = fma(s.cym, x[p - s.nx], ax);
    if (hy1) ax = fma(s.cyp, x[p + s.nx], ax);
    double r = fma(al, ax, be * xc);
    if (Y0) r = fma(g0, y0[p], r);
    if (Y1) r = fma(g1, y1[p], r);
    out[p] = r;
    xz0 = xc;
    xc = xz1;
  }
}

static hipError_t launch_st7(const Op& op, const double* x, const double* y0, const double* y1,
                             double* out, const ChainCoef& k, hipStream_t st) {
  St7 s{op.dims[0], op.dims[1], op.dims[2], op.coef[0], op.coef[1], op.coef[2],
        op.coef[3], op.coef[4], op.coef[5], op.coef[6]};
  const int gx = (s.nx + ST_TX - 1) / ST_TX, gy = (s.ny + ST_TY - 1) / ST_TY;
  // enough z-slabs for ~2048 workgroups, at least one plane per thread
  const int64_t want = 2048;
  int gz = (int)std::min<int64_t>(s.nz, std::max<int64_t>(1, want / ((int64_t)gx * gy)));
  const int kz = (s.nz + gz - 1) / gz;
  gz = (s.nz + kz - 1) / kz;
  const int nwg = gx * gy * gz;
  const double al = k.alpha.real(), be = k.beta.real(), g0 = k.g0.real(), g1 = k.g1.real();
  const dim3 grid(nwg), block(ST_TX * ST_TY);
  if (y0 && y1)
    st7_chain<true, true><<<grid, block, 0, st>>>(s, kz, gx, gy, nwg, x, y0, y1, out, al, be, g0, g1);
  else if (y0)
    st7_chain<true, false><<<grid, block, 0, st>>>(s, kz, gx, gy, nwg, x, y0, y1, out, al, be, g0, g1);
  else if (y1)
    st7_chain<false, true><<<grid, block, 0, st>>>(s, kz, gx, gy, nwg, x, y0, y1, out, al, be, g0, g1);
  else
    st7_chain<false, false><<<grid, block, 0, st>>>(s, kz, gx, gy, nwg, x, y0, y1, out, al, be, g0, g1);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// CSR, real or complex values: G lanes per row (G = power of two <= 64 close
// to the mean row length), row sums reduced with shuffles inside the group.
// --------------------------------------------------------------------------
template <typename T, int G, bool Y0, bool Y1>
__global__ __launch_bounds__(256) void csr_chain(int n, const int32_t* __restrict__ rowptr,
                                                 const int32_t* __restrict__ colind,
                                                 const T* __restrict__ vals,
                                                 const T* __restrict__ x,
                                                 const T* __restrict__ y0, const T* y1, T* out,
                                                 T al, T be, T g0, T g1) {
  const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t row = gt / G;
  const int lane = (int)(gt % G);
  if (row >= n) return;  // whole groups leave together (G divides 64)
  T acc = zero(T{});
  const int e1 = rowptr[row + 1];
  for (int e = rowptr[row] + lane; e < e1; e += G) acc = mad(vals[e], x[colind[e]], acc);
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) acc += shfl_down(acc, off, G);
  if (lane == 0) {
    T r = mad(al, acc, be * x[row]);
    if (Y0) r = mad(g0, y0[row], r);
    if (Y1) r = mad(g1, y1[row], r);
    out[row] = r;
  }
}

template <typename T, int G>
static void launch_csr_g(const Op& op, const T* x, const T* y0, const T* y1, T* out, T al,
                         T be, T g0, T g1, hipStream_t st) {
  const int n = (int)op.n;
  const int64_t threads = (int64_t)n * G;
  const int grid = (int)((threads + 255) / 256);
  auto rp = op.rowptr;
  auto ci = op.colind;
  auto va = (const T*)op.vals;
  if (y0 && y1)
    csr_chain<T, G, true, true><<<grid, 256, 0, st>>>(n, rp, ci, va, x, y0, y1, out, al, be, g0, g1);
  else if (y0)
    csr_chain<T, G, true, false><<<grid, 256, 0, st>>>(n, rp, ci, va, x, y0, y1, out, al, be, g0, g1);
  else if (y1)
    csr_chain<T, G, false, true><<<grid, 256, 0, st>>>(n, rp, ci, va, x, y0, y1, out, al, be, g0, g1);
  else
    csr_chain<T, G, false, false><<<grid, 256, 0, st>>>(n, rp, ci, va, x, y0, y1, out, al, be, g0, g1);
}

template <typename T>
static hipError_t launch_csr(const Op& op, const T* x, const T* y0, const T* y1, T* out,
                             const ChainCoef& k, hipStream_t st) {
  const T al = host_to_dev<T>::conv(k.alpha), be = host_to_dev<T>::conv(k.beta),
          g0 = host_to_dev<T>::conv(k.g0), g1 = host_to_dev<T>::conv(k.g1);
  switch (op.csr_group) {
    case 1: launch_csr_g<T, 1>(op, x, y0, y1, out, al, be, g0, g1, st); break;
    case 2: launch_csr_g<T, 2>(op, x, y0, y1, out, al, be, g0, g1, st); break;
    case 4: launch_csr_g<T, 4>(op, x, y0, y1, out, al, be, g0, g1, st); break;
    case 8: launch_csr_g<T, 8>(op, x, y0, y1, out, al, be, g0, g1, st); break;
    case 16: launch_csr_g<T, 16>(op, x, y0, y1, out, al, be, g0, g1, st); break;
    case 32: launch_csr_g<T, 32>(op, x, y0, y1, out, al, be, g0, g1, st); break;
    default: launch_csr_g<T, 64>(op, x, y0, y1, out, al, be, g0, g1, st); break;
  }
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Wilson-Dirac-like operator, complex FP64, one thread per lattice site.
//   (D x)(s) = (4 + m0) x(s) - 1/2 sum_mu [(1 - g_mu) U_mu(s) x(s + mu)
//                                         + (1 + g_mu) U_mu(s - mu)^H x(s - mu)]
// (1 -+ g_mu) has rank 2 in spin space: the hop projects the 4-spinor to a
// 2-spinor h, multiplies h by the 3x3 link (6 colour matvecs instead of 12) and
// rebuilds the lower two spins from h.  Chiral basis:
//   g_k = [[0, -i s_k], [i s_k, 0]] (k = x, y, z), g_t = [[0, I], [I, 0]].
// For (1 - g_k): h = u + i s_k d, lower = -i s_k h; for (1 + g_k): h = u - i s_k d,
// lower = i s_k h; for g_t: h = u -+ d, lower = -+ h  (u, d = upper / lower spins).
// --------------------------------------------------------------------------
struct Wil {
  int L0, L1, L2, L3;  // x, y, z, t extents
  int V;
  double diag;         // 4 + m0
};

// s_k applied with a factor i: returns i s_k [a; b]
__device__ __forceinline__ void isig(int k, cplx a, cplx b, cplx& o0, cplx& o1) {
  if (k == 0) {        // i s_x [a; b] = [i b; i a]
    o0 = times_i(b);
    o1 = times_i(a);
  } else if (k == 1) { // i s_y [a; b] = [b; -a]
    o0 = b;
    o1 = cplx{-a.x, -a.y};
  } else {             // i s_z [a; b] = [i a; -i b]
    o0 = times_i(a);
    o1 = times_mi(b);
  }
}

// h (2 spins x 3 colours) = upper half of (1 + sgn g_mu) psi; sgn = -1 or +1
__device__ __forceinline__ void spin_project(int mu, int sgn, const cplx* psi, cplx h[2][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cplx u0 = psi[0 * 3 + c], u1 = psi[1 * 3 + c], d0 = psi[2 * 3 + c], d1 = psi[3 * 3 + c];
    if (mu == 3) {  // g_t: h = u + sgn d
      h[0][c] = sgn > 0 ? u0 + d0 : u0 - d0;
      h[1][c] = sgn > 0 ? u1 + d1 : u1 - d1;
    } else {        // g_k: h = u - sgn i s_k d
      cplx t0, t1;
      isig(mu, d0, d1, t0, t1);
      h[0][c] = sgn > 0 ? u0 - t0 : u0 + t0;
      h[1][c] = sgn > 0 ? u1 - t1 : u1 + t1;
    }
  }
}

// acc += full spinor rebuilt from the projected-and-transported h
__device__ __forceinline__ void spin_accumulate(int mu, int sgn, const cplx g[2][3],
                                                cplx acc[4][3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    acc[0][c] += g[0][c];
    acc[1][c] += g[1][c];
    if (mu == 3) {  // lower = sgn h
      if (sgn > 0) { acc[2][c] += g[0][c]; acc[3][c] += g[1][c]; }
      else { acc[2][c] -= g[0][c]; acc[3][c] -= g[1][c]; }
    } else {        // lower = sgn i s_k h
      cplx t0, t1;
      isig(mu, g[0][c], g[1][c], t0, t1);
      if (sgn > 0) { acc[2][c] += t0; acc[3][c] += t1; }
      else { acc[2][c] -= t0; acc[3][c] -= t1; }
    }
  }
}

template <bool Y0, bool Y1>
__global__ __launch_bounds__(128) void wilson_chain(Wil w, const cplx* __restrict__ U,
                                                    const cplx* __restrict__ x,
                                                    const cplx* __restrict__ y0,
                                                    const cplx* y1, cplx* out, cplx al,
                                                    cplx be, cplx g0, cplx g1) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= w.V) return;
  int co[4];
  {
    int r = s;
    co[0] = r % w.L0; r /= w.L0;
    co[1] = r % w.L1; r /= w.L1;
    co[2] = r % w.L2; r /= w.L2;
    co[3] = r;
  }
  const int Ls[4] = {w.L0, w.L1, w.L2, w.L3};
  const int stride[4] = {1, w.L0, w.L0 * w.L1, w.L0 * w.L1 * w.L2};
  cplx acc[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[a][c] = cplx{0.0, 0.0};

#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    // forward hop: (1 - g_mu) U_mu(s) x(s + mu)
    {
      const int sf = (co[mu] + 1 < Ls[mu]) ? s + stride[mu] : s - (Ls[mu] - 1) * stride[mu];
      cplx psi[12];
#pragma unroll
      for (int e = 0; e < 12; ++e) psi[e] = x[(int64_t)sf * 12 + e];
      cplx h[2][3], g[2][3];
      spin_project(mu, -1, psi, h);
      const cplx* Um = U + ((int64_t)mu * w.V + s) * 9;
      cplx u[9];
#pragma unroll
      for (int e = 0; e < 9; ++e) u[e] = Um[e];
#pragma unroll
      for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a)
          g[sp][a] = mad(u[a * 3 + 2], h[sp][2], mad(u[a * 3 + 1], h[sp][1], u[a * 3 + 0] * h[sp][0]));
      spin_accumulate(mu, -1, g, acc);
    }
    // backward hop: (1 + g_mu) U_mu(s - mu)^H x(s - mu)
    {
      const int sb = (co[mu] > 0) ? s - stride[mu] : s + (Ls[mu] - 1) * stride[mu];
      cplx psi[12];
#pragma unroll
      for (int e = 0; e < 12; ++e) psi[e] = x[(int64_t)sb * 12 + e];
      cplx h[2][3], g[2][3];
      spin_project(mu, +1, psi, h);
      const cplx* Um = U + ((int64_t)mu * w.V + sb) * 9;
      cplx u[9];
#pragma unroll
      for (int e = 0; e < 9; ++e) u[e] = Um[e];
#pragma unroll
      for (int sp = 0; sp < 2; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a)  // (U^H h)_a = sum_b conj(U_ba) h_b
          g[sp][a] = cmad(u[2 * 3 + a], h[sp][2], cmad(u[1 * 3 + a], h[sp][1],
                          cmad(u[0 * 3 + a], h[sp][0], cplx{0.0, 0.0})));
      spin_accumulate(mu, +1, g, acc);
    }
  }
  const int64_t base = (int64_t)s * 12;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int e = a * 3 + c;
      const cplx xc = x[base + e];
      const cplx dx = w.diag * xc - 0.5 * acc[a][c];
      cplx r = mad(al, dx, be * xc);
      if (Y0) r = mad(g0, y0[base + e], r);
      if (Y1) r = mad(g1, y1[base + e], r);
      out[base + e] = r;
    }
}

static hipError_t launch_wilson(const Op& op, const cplx* x, const cplx* y0, const cplx* y1,
                                cplx* out, const ChainCoef& k, hipStream_t st) {
  Wil w{op.dims[0], op.dims[1], op.dims[2], op.dims[3],
        op.dims[0] * op.dims[1] * op.dims[2] * op.dims[3], 4.0 + op.m0};
  const int grid = (w.V + 127) / 128;
  const cplx al = host_to_dev<cplx>::conv(k.alpha), be = host_to_dev<cplx>::conv(k.beta),
             g0 = host_to_dev<cplx>::conv(k.g0), g1 = host_to_dev<cplx>::conv(k.g1);
  const cplx* U = (const cplx*)op.links;
  if (y0 && y1)
    wilson_chain<true, true><<<grid, 128, 0, st>>>(w, U, x, y0, y1, out, al, be, g0, g1);
  else if (y0)
    wilson_chain<true, false><<<grid, 128, 0, st>>>(w, U, x, y0, y1, out, al, be, g0, g1);
  else if (y1)
    wilson_chain<false, true><<<grid, 128, 0, st>>>(w, U, x, y0, y1, out, al, be, g0, g1);
  else
    wilson_chain<false, false><<<grid, 128, 0, st>>>(w, U, x, y0, y1, out, al, be, g0, g1);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
hipError_t launch_chain(const Op& op, const void* x, const void* y0, const void* y1, void* out,
                        const ChainCoef& k, hipStream_t s) {
  switch (op.kind) {
    case OP_STENCIL7:
      return launch_st7(op, (const double*)x, (const double*)y0, (const double*)y1,
                        (double*)out, k, s);
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

double chain_bytes(const Op& op, bool has_y0, bool has_y1) {
  const double vec = (double)op.n * elem_size(op.dtype);
  const double nvec = 2.0 + (has_y0 ? 1.0 : 0.0) + (has_y1 ? 1.0 : 0.0);
  double extra = 0.0;
  if (op.kind == OP_CSR)
    extra = (double)(op.n + 1) * 4 + (double)op.nnz * (4 + elem_size(op.dtype));
  if (op.kind == OP_WILSON) extra = 4.0 * (double)(op.n / 12) * 9 * 16;
  return nvec * vec + extra;
}

}  // namespace fa
