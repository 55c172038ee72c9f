// Small Hermitian problems: the Lanczos steps between two stopping checks in
// one launch of one workgroup.
//
// For an operator of a few thousand rows (the 2D Poisson matrix of the
// Laplace examples, n = 1,024) a Krylov step is a few microseconds of work
// but five to twenty launches (A, the Clenshaw terms of q(A) twice, the
// three-term recurrence, the normalization), each costing its launch
// latency.  Here one 1024-thread workgroup runs the steps j0 .. j1 - 1 of
// Algorithm 1 with the Lanczos recurrence (Sec. 6, Example 1):
//     u = A v_j,  y = q(A) u,  w = q(A) y     (Clenshaw terms of Sec. 5.1),
//     w -= beta_{j-1} v_{j-1},  alpha_j = v_j^T w,  w -= alpha_j v_j,
//     beta_j = ||w||,  v_{j+1} = w / beta_j,
// writing v_{j+1} to the basis and (alpha_j, beta_j) to the banded H exactly
// where the step-by-step kernels do, so the host's checks, the final
// combination and the stopping logic are unchanged.
//   * Each thread owns E vector entries (i = tid + 1024 e) in registers.
//   * The vector a product with A reads goes through LDS (two buffers, one
//     barrier per product); CSR rows of at most kSmallRow entries are held in
//     registers (padded with zero values), the 7-point stencil is its
//     coefficients.
//   * The two inner products of a step are workgroup reductions in a fixed
//     order (wavefront sums, then the 16 wavefront sums in order), so the
//     result is deterministic.
// --------------------------------------------------------------------------
#include <hip/hip_runtime.h>

#include "devmath.hpp"
#include "fa_internal.hpp"

namespace fa {

namespace {

constexpr int kSmallThreads = 1024;

template <int E, bool CSR>
__global__ __launch_bounds__(kSmallThreads) void small_lanczos_k(SmallLanczosArgs a) {
  __shared__ double buf[2][kSmallMaxN];
  __shared__ double red[2][kSmallThreads / 64];
  const int tid = threadIdx.x;
  const int n = a.n;
  // the operator at the owned entries
  int col[E][kSmallRow];
  double val[E][kSmallRow];
  int nb[E][7];  // stencil: centre and the six neighbours (index or -1)
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = tid + kSmallThreads * e;
    if (CSR) {
      const int e0 = i < n ? a.rowptr[i] : 0, e1 = i < n ? a.rowptr[i + 1] : 0;
#pragma unroll
      for (int r = 0; r < kSmallRow; ++r) {
        const bool in = e0 + r < e1;
        col[e][r] = in ? a.colind[e0 + r] : 0;
        val[e][r] = in ? a.vals[e0 + r] : 0.0;
      }
    } else {
      const int ii = i % a.nx, jj = (i / a.nx) % a.ny, kk = i / (a.nx * a.ny);
      const int pl = a.nx * a.ny;
      nb[e][0] = i;
      nb[e][1] = ii > 0 ? i - 1 : -1;
      nb[e][2] = ii + 1 < a.nx ? i + 1 : -1;
      nb[e][3] = jj > 0 ? i - a.nx : -1;
      nb[e][4] = jj + 1 < a.ny ? i + a.nx : -1;
      nb[e][5] = kk > 0 ? i - pl : -1;
      nb[e][6] = kk + 1 < a.nz ? i + pl : -1;
    }
  }
  int par = 0;
  // y = A x (x in registers; all threads take part: one barrier)
  auto op_A = [&](const double (&x)[E], double (&y)[E]) {
    double* B = buf[par];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = tid + kSmallThreads * e;
      if (i < n) B[i] = x[e];
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      double acc = 0.0;
      if (CSR) {
#pragma unroll
        for (int r = 0; r < kSmallRow; ++r) acc = fma(val[e][r], B[col[e][r]], acc);
      } else {
        const int i = tid + kSmallThreads * e;
        if (i < n) {
          acc = a.c[0] * B[nb[e][0]];
#pragma unroll
          for (int d = 1; d < 7; ++d)
            if (nb[e][d] >= 0) acc = fma(a.c[d], B[nb[e][d]], acc);
        }
      }
      y[e] = acc;
    }
    par ^= 1;
  };
  // out = q(A) in by the recurrence terms: out_i = a A x_i + b x_i + g0 in +
  // g1 out_{i-2}, x_i = out_{i-1}, x_0 = in
  auto op_q = [&](const double (&in)[E], double (&out)[E]) {
    double cur[E], pm2[E], ax[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      cur[e] = in[e];
      pm2[e] = 0.0;
    }
    for (int t = 0; t < a.nterms; ++t) {
      const SmallTerm T = a.t[t];
      op_A(cur, ax);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        double r = fma(T.a, ax[e], T.b * cur[e]);
        if (T.y0) r = fma(T.g0, in[e], r);
        if (T.y1) r = fma(T.g1, pm2[e], r);
        pm2[e] = cur[e];
        cur[e] = r;
      }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) out[e] = cur[e];
  };
  // sum over the workgroup of the per-thread values, in a fixed order
  auto wg_sum = [&](double p, int slot) {
    p = wave_sum(p);
    if ((tid & 63) == 0) red[slot][tid >> 6] = p;
    __syncthreads();
    double s = red[slot][0];
#pragma unroll
    for (int w = 1; w < kSmallThreads / 64; ++w) s += red[slot][w];
    return s;
  };

  double v[E], vp[E];
  double bprev = a.j0 > 0 ? a.H[(size_t)(a.j0 - 1) * 2 + 1] : 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = tid + kSmallThreads * e;
    v[e] = i < n ? a.V[(size_t)a.j0 * a.ldv + i] : 0.0;
    vp[e] = (i < n && a.j0 > 0) ? a.V[(size_t)(a.j0 - 1) * a.ldv + i] : 0.0;
  }
  for (int j = a.j0; j < a.j1; ++j) {
    double u[E], y[E], w[E];
    op_A(v, u);
    op_q(u, y);
    op_q(y, w);
    double p = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (j > 0) w[e] = fma(-bprev, vp[e], w[e]);
      p = fma(v[e], w[e], p);
    }
    const double alpha = wg_sum(p, 0);
    p = 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      w[e] = fma(-alpha, v[e], w[e]);
      p = fma(w[e], w[e], p);
    }
    const double beta = sqrt(wg_sum(p, 1));
    if (tid == 0) {
      a.H[(size_t)j * 2] = alpha;
      a.H[(size_t)j * 2 + 1] = beta;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = tid + kSmallThreads * e;
      const double vn = w[e] / beta;
      if (i < n) a.V[(size_t)(j + 1) * a.ldv + i] = vn;
      vp[e] = v[e];
      v[e] = vn;
    }
    bprev = beta;
  }
}

}  // namespace

bool small_lanczos_ok(const Op& op, const Poly& q) {
  if (op.dtype != FA_F64 || op.n > kSmallMaxN) return false;
  if (op.kind == OP_CSR ? op.csr_maxrow > kSmallRow : op.kind != OP_STENCIL7) return false;
  const int K = q.method < 0 ? 0 : q.degree;
  return K == 0 || (q.method == FA_POLY_CHEB && K <= kSmallMaxTerms);
}

hipError_t launch_small_lanczos(const Op& op, const std::vector<SmallTerm>& terms, int j0,
                                int j1, void* V, int64_t ldv, void* H, hipStream_t s) {
  if ((int)terms.size() > kSmallMaxTerms || op.n > kSmallMaxN) return hipErrorInvalidValue;
  SmallLanczosArgs a{};
  a.n = (int)op.n;
  a.j0 = j0;
  a.j1 = j1;
  a.nterms = (int)terms.size();
  a.ldv = ldv;
  a.V = (double*)V;
  a.H = (double*)H;
  for (size_t t = 0; t < terms.size(); ++t) a.t[t] = terms[t];
  const bool csr = op.kind == OP_CSR;
  if (csr) {
    a.rowptr = op.rowptr;
    a.colind = op.colind;
    a.vals = (const double*)op.vals;
  } else {
    a.nx = op.dims[0];
    a.ny = op.dims[1];
    a.nz = op.dims[2];
    for (int c = 0; c < 7; ++c) a.c[c] = op.coef[c];
  }
  if (op.n <= kSmallThreads) {
    if (csr)
      small_lanczos_k<1, true><<<1, kSmallThreads, 0, s>>>(a);
    else
      small_lanczos_k<1, false><<<1, kSmallThreads, 0, s>>>(a);
  } else {
    if (csr)
      small_lanczos_k<2, true><<<1, kSmallThreads, 0, s>>>(a);
    else
      small_lanczos_k<2, false><<<1, kSmallThreads, 0, s>>>(a);
  }
  return hipGetLastError();
}

}  // namespace fa
