// C ABI of the library (declared in include/fa.h): argument validation and
// dispatch to the runtime.  No exception crosses the boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <complex>
#include <vector>

#include "dense.hpp"
#include "fa_internal.hpp"
#include "solver.hpp"

using namespace fa;

namespace {
hipStream_t stream_of(void* s) { return (hipStream_t)s; }

// exact real eigenvalue interval of a 7-point stencil when every direction's
// off-diagonal pair has a positive product (diagonally similar to symmetric):
// c0 -+ sum_d 2 sqrt(c_dm c_dp) cos(pi / (N_d + 1))
bool stencil_interval(const Op& op, double* lo, double* hi) {
  double spread = 0.0;
  for (int d = 0; d < 3; ++d) {
    const int N = op.dims[d];
    const double p = op.coef[1 + 2 * d] * op.coef[2 + 2 * d];
    if (N == 1 || p == 0.0) continue;
    if (p < 0.0) return false;
    spread += 2.0 * std::sqrt(p) * std::cos(M_PI / (N + 1));
  }
  *lo = op.coef[0] - spread;
  *hi = op.coef[0] + spread;
  return true;
}

template <typename F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return FA_ERR_ARG;
  } catch (...) {
    return FA_ERR_ARG;
  }
}
}  // namespace

extern "C" {

size_t fa_op_device_bytes(int kind, const int32_t dims[4], int64_t n, int64_t nnz) {
  (void)n;
  (void)nnz;
  switch (kind) {
    case FA_STENCIL7:
      return 0;
    case FA_CSR: {  // the tables of row blocks, chunks of long rows and long rows
      if (n < 1 || nnz < 0) return 0;
      const int64_t nl = nnz / (kCsrBlockEntries + 1) + 1, nc = 2 * nl + nnz / kCsrBlockEntries;
      return (size_t)(round_up(16 * n, 256) + round_up(16 * nc, 256) + round_up(12 * nl, 256));
    }
    case FA_WILSON4D: {
      if (!dims) return 0;
      int64_t V = 1;
      for (int d = 0; d < 4; ++d) {
        if (dims[d] < 2) return 0;
        V *= dims[d];
      }
      return (size_t)round_up(V * 4 * 9 * 16, 256);  // whole links (the most kept)
    }
    default:
      return 0;
  }
}

int fa_create_csr(fa_op* out, int64_t n, int64_t nnz, const int32_t* d_rowptr,
                  const int32_t* d_colind, const void* d_vals, int dtype, uint32_t flags,
                  void* d_opmem, size_t opmem_bytes, void* hip_stream) {
  if (!out || n < 1 || n >= (int64_t(1) << 31) || nnz < 0 || nnz >= (int64_t(1) << 31) ||
      !d_rowptr || (nnz > 0 && (!d_colind || !d_vals)) || (dtype != FA_F64 && dtype != FA_C128) ||
      (flags & ~uint32_t(FA_HERMITIAN)))
    return FA_ERR_ARG;
  return guarded([&] {
    Op op;
    op.uid = next_op_uid();
    op.kind = OP_CSR;
    op.dtype = dtype;
    op.n = n;
    op.flags = flags;
    op.rowptr = d_rowptr;
    op.colind = d_colind;
    op.vals = d_vals;
    op.nnz = nnz;
    // the index arrays may still be in flight on the caller's stream
    hipStream_t st = stream_of(hip_stream);
    std::vector<int32_t> rp((size_t)n + 1), ci((size_t)nnz);
    if (hipStreamSynchronize(st) != hipSuccess ||
        hipMemcpy(rp.data(), d_rowptr, rp.size() * sizeof(int32_t), hipMemcpyDeviceToHost) !=
            hipSuccess ||
        (nnz > 0 &&
         hipMemcpy(ci.data(), d_colind, ci.size() * sizeof(int32_t), hipMemcpyDeviceToHost) !=
             hipSuccess))
      return FA_ERR_HIP;
    // the kernels index with both arrays unchecked: the row pointers must
    // describe nnz entries in order and every column index must lie in [0, n)
    if (rp[0] != 0 || rp[(size_t)n] != nnz) return FA_ERR_ARG;
    for (int64_t r = 0; r < n; ++r) {
      if (rp[r + 1] < rp[r]) return FA_ERR_ARG;
      op.csr_maxrow = std::max<int>(op.csr_maxrow, rp[r + 1] - rp[r]);
    }
    for (int64_t e = 0; e < nnz; ++e)
      if (ci[e] < 0 || ci[e] >= n) return FA_ERR_ARG;
    // the work split: blocks of consecutive rows with at most
    // kCsrBlockEntries entries and kCsrBlockRows rows, cut greedily; a row
    // with more entries than a block holds is cut into chunks of
    // kCsrBlockEntries, a workgroup each
    std::vector<int32_t> blk, chk, lng;
    for (int64_t r = 0; r < n;) {
      if (rp[r + 1] - rp[r] > kCsrBlockEntries) {
        const int32_t li = (int32_t)(lng.size() / 3), c0 = (int32_t)(chk.size() / 4);
        int32_t nc = 0;
        for (int64_t e = rp[r]; e < rp[r + 1]; e += kCsrBlockEntries, ++nc) {
          chk.push_back((int32_t)r);
          chk.push_back((int32_t)e);
          chk.push_back((int32_t)std::min<int64_t>(e + kCsrBlockEntries, rp[r + 1]));
          chk.push_back(li);
        }
        lng.push_back((int32_t)r);
        lng.push_back(c0);
        lng.push_back(nc);
        ++r;
        continue;
      }
      const int64_t r0 = r;
      while (r < n && r - r0 < kCsrBlockRows && rp[r + 1] - rp[r] <= kCsrBlockEntries &&
             rp[r + 1] - rp[r0] <= kCsrBlockEntries)
        ++r;
      blk.push_back((int32_t)r0);
      blk.push_back((int32_t)r);
      blk.push_back(rp[r0]);
      blk.push_back(rp[r]);
    }
    op.csr_nblk = (int)(blk.size() / 4);
    op.csr_nchunk = (int)(chk.size() / 4);
    op.csr_nlong = (int)(lng.size() / 3);
    // the three tables in the caller's operator memory, each 256-byte aligned
    const size_t b_blk = blk.size() * 4, b_chk = chk.size() * 4, b_lng = lng.size() * 4;
    const size_t off_chk = (size_t)round_up((int64_t)b_blk, 256);
    const size_t off_lng = off_chk + (size_t)round_up((int64_t)b_chk, 256);
    const size_t need = off_lng + b_lng;
    if (!d_opmem || opmem_bytes < need || ((uintptr_t)d_opmem & 255)) return FA_ERR_WORKSPACE;
    char* const m = (char*)d_opmem;
    op.csr_blk_dev = (const int32_t*)m;
    op.csr_chunk_dev = (const int32_t*)(m + off_chk);
    op.csr_long_dev = (const int32_t*)(m + off_lng);
    if ((b_blk && hipMemcpyAsync(m, blk.data(), b_blk, hipMemcpyHostToDevice, st) != hipSuccess) ||
        (b_chk &&
         hipMemcpyAsync(m + off_chk, chk.data(), b_chk, hipMemcpyHostToDevice, st) != hipSuccess) ||
        (b_lng &&
         hipMemcpyAsync(m + off_lng, lng.data(), b_lng, hipMemcpyHostToDevice, st) != hipSuccess) ||
        hipStreamSynchronize(st) != hipSuccess)
      return FA_ERR_HIP;
    fa_op h = new fa_op_s;
    h->op = op;
    *out = h;
    return FA_OK;
  });
}

int fa_create_stencil(fa_op* out, int kind, const int32_t dims[4], const double* params,
                      int nparams, const void* d_links, uint32_t flags, void* d_opmem,
                      size_t opmem_bytes, void* hip_stream) {
  if (!out || !dims || !params) return FA_ERR_ARG;
  if (flags & ~uint32_t(FA_HERMITIAN | FA_Q2)) return FA_ERR_ARG;
  if ((flags & FA_Q2) && kind != FA_WILSON4D) return FA_ERR_ARG;
  for (int d = 0; d < 4; ++d)
    if (dims[d] < 1) return FA_ERR_ARG;
  return guarded([&] {
    Op op;
    if (kind == FA_STENCIL7) {
      if (nparams != 7 || dims[3] != 1) return FA_ERR_ARG;
      const int64_t n = (int64_t)dims[0] * dims[1] * dims[2];
      if (n >= (int64_t(1) << 31)) return FA_ERR_ARG;
      op.kind = OP_STENCIL7;
      op.dtype = FA_F64;
      op.n = n;
      for (int i = 0; i < 7; ++i) {
        if (!std::isfinite(params[i])) return FA_ERR_ARG;
        op.coef[i] = params[i];
      }
      for (int d = 0; d < 3; ++d) op.dims[d] = dims[d];
      if (flags & FA_HERMITIAN)
        for (int d = 0; d < 3; ++d)
          if (op.coef[1 + 2 * d] != op.coef[2 + 2 * d]) return FA_ERR_ARG;
      double lo, hi;
      if (stencil_interval(op, &lo, &hi) && lo > 0.0) {
        op.has_interval = true;
        op.lo = lo;
        op.hi = hi;
      }
    } else if (kind == FA_WILSON4D) {
      if ((nparams != 1 && nparams != 2) || !d_links) return FA_ERR_ARG;
      for (int d = 0; d < 4; ++d)
        if (dims[d] < 2) return FA_ERR_ARG;
      const int64_t V = (int64_t)dims[0] * dims[1] * dims[2] * dims[3];
      if (V * 12 >= (int64_t(1) << 31)) return FA_ERR_ARG;
      op.kind = OP_WILSON;
      op.dtype = FA_C128;
      op.n = V * 12;
      for (int d = 0; d < 4; ++d) op.dims[d] = dims[d];
      op.m0 = params[0];
      op.mu = nparams > 1 ? params[1] : 0.0;
      op.q2 = (flags & FA_Q2) != 0;
      if (!std::isfinite(op.m0) || !std::isfinite(op.mu) || std::fabs(op.mu) > 20.0)
        return FA_ERR_ARG;
      // Gamma_5 D is Hermitian only without a chemical potential
      if ((flags & FA_HERMITIAN) && !(op.q2 && op.mu == 0.0)) return FA_ERR_ARG;
      // Special unitary links (det 1: row 2 = conj(row 0 x row 1) to within
      // 1e-13) are stored as their first two rows and the kernel rebuilds the
      // third (a third less link traffic); other links are stored whole.
      // operator memory: at least the two-row copy, checked again below
      // once the link format is known
      if (!d_opmem || opmem_bytes < (size_t)V * 4 * 6 * 16 || ((uintptr_t)d_opmem & 255))
        return FA_ERR_WORKSPACE;
      hipStream_t st = stream_of(hip_stream);
      std::vector<std::complex<double>> hu((size_t)V * 36);
      if (hipStreamSynchronize(st) != hipSuccess ||
          hipMemcpy(hu.data(), d_links, hu.size() * 16, hipMemcpyDeviceToHost) != hipSuccess)
        return FA_ERR_HIP;
      bool su3 = true;
      for (size_t l = 0; l < (size_t)V * 4 && su3; ++l) {
        const std::complex<double>* u = &hu[l * 9];
        const std::complex<double> c[3] = {u[1] * u[5] - u[2] * u[4], u[2] * u[3] - u[0] * u[5],
                                           u[0] * u[4] - u[1] * u[3]};
        for (int j = 0; j < 3; ++j)
          if (!(std::abs(u[6 + j] - std::conj(c[j])) <= 1e-13)) su3 = false;
      }
      op.links_rows = su3 ? 2 : 3;
      const int ne = 3 * op.links_rows;
      // structure-of-arrays copy of the links (coalesced link loads) in the
      // caller's operator memory
      const size_t need = (size_t)V * 4 * ne * 16;
      if (!d_opmem || opmem_bytes < need || ((uintptr_t)d_opmem & 255)) return FA_ERR_WORKSPACE;
      op.links = d_opmem;
      if (launch_wilson_links_soa(V, ne, d_links, d_opmem, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return FA_ERR_HIP;
    } else {
      return FA_ERR_ARG;
    }
    op.flags = flags;
    op.uid = next_op_uid();
    fa_op h = new fa_op_s;
    h->op = op;
    *out = h;
    return FA_OK;
  });
}

int fa_set_spectral_interval(fa_op op, double lo, double hi) {
  if (!op || !(lo > 0.0) || !(hi > lo) || !std::isfinite(hi)) return FA_ERR_ARG;
  op->op.has_interval = true;
  op->op.lo = lo;
  op->op.hi = hi;
  return FA_OK;
}

int fa_get_spectral_interval(fa_op op, double* lo, double* hi) {
  if (!op || !lo || !hi) return FA_ERR_ARG;
  if (!op->op.has_interval) return FA_ERR_NO_INTERVAL;
  *lo = op->op.lo;
  *hi = op->op.hi;
  return FA_OK;
}

size_t fa_poly_workspace_bytes(fa_op op, int degree, int method) {
  if (!op || degree < 0) return 0;
  if (method == FA_POLY_AUTO) method = op->op.has_interval ? FA_POLY_CHEB : FA_POLY_RITZ;
  return poly_workspace_bytes(op->op, degree, method);
}

int fa_poly_setup(fa_op op, int degree, int method, const void* d_start, void* d_workspace,
                  size_t ws_bytes, void* hip_stream) {
  if (!op || degree < 0 || method < FA_POLY_AUTO || method > FA_POLY_LS) return FA_ERR_ARG;
  return guarded([&] {
    int64_t mv = 0;
    return poly_setup(op->op, degree, method, d_start, d_workspace, ws_bytes,
                      stream_of(hip_stream), &mv);
  });
}

int fa_poly_setup_ls(fa_op op, int degree, int ritz_steps, double r_min, double step,
                     const void* d_start, void* d_workspace, size_t ws_bytes, void* hip_stream) {
  if (!op || degree < 1 || degree >= kLsMax || ritz_steps < 2 || !(r_min >= 0.0) ||
      !(step > 0.0) || !std::isfinite(r_min) || !std::isfinite(step))
    return FA_ERR_ARG;
  LsParams ls;
  ls.ritz_steps = ritz_steps;
  ls.r_min = r_min;
  ls.step = step;
  return guarded([&] {
    int64_t mv = 0;
    return poly_setup(op->op, degree, FA_POLY_LS, d_start, d_workspace, ws_bytes,
                      stream_of(hip_stream), &mv, ls);
  });
}

int fa_poly_get(fa_op op, int* degree, int* method, double* coef_re, double* coef_im,
                double* nodes_re, double* nodes_im, double* interval, double* rho) {
  if (!op) return FA_ERR_ARG;
  if (!op->op.poly_ready) return FA_ERR_NO_POLY;
  const Poly& q = op->op.poly;
  if (degree) *degree = q.degree;
  if (method) *method = q.harmonic ? FA_POLY_HARMONIC : q.method;
  if (q.method == FA_POLY_CHEB) {
    for (int i = 0; i <= q.degree; ++i) {
      if (coef_re) coef_re[i] = q.c[i];
      if (coef_im) coef_im[i] = 0.0;
    }
    if (interval) {
      interval[0] = q.a;
      interval[1] = q.b;
    }
  } else if (q.method == FA_POLY_RITZ) {
    for (int i = 0; i <= q.degree; ++i) {
      if (coef_re) coef_re[i] = q.eta[i].real();
      if (coef_im) coef_im[i] = q.eta[i].imag();
      if (nodes_re) nodes_re[i] = q.theta[i].real();
      if (nodes_im) nodes_im[i] = q.theta[i].imag();
    }
    if (rho) *rho = q.rho;
  } else if (q.method == FA_POLY_LS) {
    for (int i = 0; i <= q.degree; ++i) {
      if (coef_re) coef_re[i] = q.alpha[i].real();
      if (coef_im) coef_im[i] = q.alpha[i].imag();
    }
    if (rho) *rho = (double)q.npts;
  }
  return FA_OK;
}

int fa_poly_get_ls(fa_op op, int64_t* npts, double* h_re, double* h_im) {
  if (!op) return FA_ERR_ARG;
  if (!op->op.poly_ready) return FA_ERR_NO_POLY;
  const Poly& q = op->op.poly;
  if (q.method != FA_POLY_LS) return FA_ERR_ARG;
  if (npts) *npts = q.npts;
  for (size_t i = 0; i < q.hls.size(); ++i) {
    if (h_re) h_re[i] = q.hls[i].real();
    if (h_im) h_im[i] = q.hls[i].imag();
  }
  return FA_OK;
}

size_t fa_workspace_bytes(fa_op op, int m_max, uint32_t flags) {
  if (!op || m_max < 1) return 0;
  return make_layout(op->op, m_max, flags).bytes;
}

int fa_apply(fa_op op, int kind, const void* d_b, void* d_x, int m_max, double tol,
             int check_every, void* d_workspace, size_t ws_bytes, uint32_t flags,
             void* hip_stream, fa_stats* stats) {
  if (!op || !d_b || !d_x || d_b == d_x || m_max < 1 || check_every < 0 ||
      (kind != FA_INVSQRT && kind != FA_SQRT) || !std::isfinite(tol) ||
      (flags & ~uint32_t(FA_FORCE_ARNOLDI | FA_PROFILE | FA_NO_FUSION | FA_FUSE2 | FA_FUSE3 | FA_MIXED |
                         FA_TWO_PASS | FA_RIGHT_PREC | FA_CGS2)))
    return FA_ERR_ARG;
  if (!op->op.poly_ready) return FA_ERR_NO_POLY;
  if ((int64_t)m_max > op->op.n) return FA_ERR_ARG;
  return guarded([&] {
    return apply(op->op, kind, d_b, d_x, m_max, tol, check_every, d_workspace, ws_bytes, flags,
                 stream_of(hip_stream), stats);
  });
}

size_t fa_block_workspace_bytes(fa_op op, int s, int m_max, uint32_t flags) {
  if (!op || (s != 16 && s != 32 && s != 64) || m_max < 1) return 0;
  return block_workspace_bytes(op->op, s, m_max, flags);
}

int fa_block_apply(fa_op op, int kind, int s, const void* d_B, void* d_X, int m_max, double tol,
                   int check_every, void* d_workspace, size_t ws_bytes, uint32_t flags,
                   void* hip_stream, fa_block_stats* stats) {
  if (!op || !d_B || !d_X || d_B == d_X || (s != 16 && s != 32 && s != 64) || m_max < 1 ||
      check_every < 0 || (kind != FA_INVSQRT && kind != FA_SQRT) || !(tol == tol) ||
      (flags & ~uint32_t(FA_MIXED | FA_GRAPH)))
    return FA_ERR_ARG;
  if (!op->op.poly_ready) return FA_ERR_NO_POLY;
  return guarded([&] {
    return block_apply(op->op, kind, s, d_B, d_X, m_max, tol, check_every, d_workspace, ws_bytes,
                       flags, stream_of(hip_stream), stats);
  });
}

int fa_op_apply(fa_op op, const void* d_x, void* d_y, void* d_workspace, size_t ws_bytes,
                void* hip_stream) {
  if (!op || !d_x || !d_y || d_x == d_y) return FA_ERR_ARG;
  if (d_workspace && (ws_bytes < make_layout(op->op, 1, 0).bytes || ((uintptr_t)d_workspace & 255)))
    return FA_ERR_WORKSPACE;
  return guarded([&] { return op_apply(op->op, d_x, d_y, d_workspace, stream_of(hip_stream)); });
}

int fa_poly_apply(fa_op op, const void* d_x, void* d_y, void* d_workspace, size_t ws_bytes,
                  void* hip_stream) {
  if (!op || !d_x || !d_y || d_x == d_y) return FA_ERR_ARG;
  if (!op->op.poly_ready) return FA_ERR_NO_POLY;
  const Layout L = make_layout(op->op, 1, 0);  // includes the least-squares q's vectors
  if (!d_workspace || ws_bytes < L.bytes || ((uintptr_t)d_workspace & 255)) return FA_ERR_WORKSPACE;
  return guarded([&] {
    return poly_apply_public(op->op, d_x, d_y, d_workspace, stream_of(hip_stream));
  });
}

int fa_op_info(fa_op op, int64_t* n, int* dtype) {
  if (!op) return FA_ERR_ARG;
  if (n) *n = op->op.n;
  if (dtype) *dtype = op->op.dtype;
  return FA_OK;
}

int fa_destroy(fa_op op) {
  if (op) release_op_graphs(op->op.uid);
  delete op;
  return FA_OK;
}

const char* fa_status_string(int status) {
  switch (status) {
    case FA_OK: return "FA_OK";
    case FA_WARN_NOT_CONVERGED: return "FA_WARN_NOT_CONVERGED: m_max reached before the stopping test";
    case FA_ERR_ARG: return "FA_ERR_ARG: invalid argument";
    case FA_ERR_NO_POLY: return "FA_ERR_NO_POLY: fa_poly_setup has not been called";
    case FA_ERR_BRANCH: return "FA_ERR_BRANCH: polynomial not in the right half-plane on the spectrum";
    case FA_ERR_HESSENBERG: return "FA_ERR_HESSENBERG: H_m has an eigenvalue on (-inf, 0]";
    case FA_ERR_WORKSPACE: return "FA_ERR_WORKSPACE: workspace null, misaligned or too small";
    case FA_ERR_HIP: return "FA_ERR_HIP: a HIP runtime call failed";
    case FA_ERR_NONFINITE: return "FA_ERR_NONFINITE: NaN or Inf in the input or iteration";
    case FA_ERR_NO_INTERVAL: return "FA_ERR_NO_INTERVAL: no spectral interval for Chebyshev";
    case FA_ERR_UNSUPPORTED: return "FA_ERR_UNSUPPORTED: combination not available for this operator";
    default: return "unknown status";
  }
}

int fa_dense_invsqrt_e1(int m, int dtype, const double* h_H, int ldh, double beta, double* h_z) {
  if (m < 1 || ldh < m || !h_H || !h_z || (dtype != FA_F64 && dtype != FA_C128)) return FA_ERR_ARG;
  return guarded([&] {
    std::vector<cd> z(m);
    int st;
    if (dtype == FA_C128) {
      std::vector<cd> H((size_t)m * m);
      for (int j = 0; j < m; ++j)
        for (int i = 0; i < m; ++i) {
          const size_t k = (size_t)j * ldh + i;
          H[(size_t)j * m + i] = (i > j + 1) ? cd(0.0) : cd(h_H[2 * k], h_H[2 * k + 1]);
        }
      st = hess_invsqrt_e1(m, H.data(), m, beta, z.data());
    } else {
      st = real_hess_invsqrt_e1(m, h_H, ldh, beta, z.data());
    }
    if (st != DENSE_OK) return FA_ERR_HESSENBERG;
    for (int i = 0; i < m; ++i) {
      if (dtype == FA_C128) {
        h_z[2 * i] = z[i].real();
        h_z[2 * i + 1] = z[i].imag();
      } else {
        h_z[i] = z[i].real();
      }
    }
    return FA_OK;
  });
}

int fa_dense_tridiag_invsqrt_e1(int m, const double* alpha, const double* offd, double beta,
                                double* z) {
  if (m < 1 || !alpha || !z || (m > 1 && !offd)) return FA_ERR_ARG;
  return guarded([&] {
    std::vector<double> of(std::max(m - 1, 1), 0.0);
    for (int i = 0; i + 1 < m; ++i) of[i] = offd[i];
    const int st = tridiag_invsqrt_e1(m, alpha, of.data(), beta, z);
    return st == DENSE_OK ? FA_OK : FA_ERR_HESSENBERG;
  });
}

}  // extern "C"
