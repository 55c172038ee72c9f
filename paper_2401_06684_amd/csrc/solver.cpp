// Host runtime of the method: workspace layout, the polynomial chain, the
// preconditioned Arnoldi / Lanczos loop with host FP64 stopping checks, and
// the polynomial setup.  All device work is enqueued on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "dense.hpp"
#include "fa_internal.hpp"
#include "solver.hpp"

namespace fa {

// --------------------------------------------------------------------------
// workspace layout (every region 256-byte aligned)
// --------------------------------------------------------------------------
Layout make_layout(const Op& op, int m_max) {
  Layout L;
  const size_t es = elem_size(op.dtype);
  L.ldv = round_up(op.n, 32);
  L.ldh = m_max + 1;
  const RedPlan rp = red_plan(op.n);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (size_t)round_up((int64_t)bytes, 256);
    return o;
  };
  L.off_V = take((size_t)(m_max + 1) * L.ldv * es);
  L.off_U = take((size_t)L.ldv * es);
  L.off_P = take((size_t)L.ldv * es);
  L.off_Q = take((size_t)L.ldv * es);
  L.off_part = take((size_t)(m_max + 2) * rp.nblk * es + 64);
  L.off_h = take((size_t)(m_max + 2) * es);
  L.off_H = take((size_t)L.ldh * m_max * es);
  L.off_nrm = take(8 * sizeof(double));
  L.off_z = take((size_t)(m_max + 1) * es);
  L.bytes = off;
  return L;
}

// --------------------------------------------------------------------------
// profiling: HIP events around chain launches (thread-local pool)
// --------------------------------------------------------------------------
namespace {
thread_local std::vector<hipEvent_t> t_events;

// Profiling: one pair of timing events around each run of consecutive middle
// terms of a polynomial recurrence (the Clenshaw terms that read x, v and
// b_{k+2}; the Newton terms that read r and v), all launches of the same
// kernel on the same sizes.  Bracketing runs rather than single launches keeps
// the events (each waits for the preceding kernel) from inflating the timing.
struct Prof {
  bool on = false;
  size_t used = 0;
  int64_t launches = 0;
  double bytes = 0;  // algorithmic bytes of the timed launches
  hipError_t begin(hipStream_t s) {
    if (!on) return hipSuccess;
    if (used + 2 > t_events.size()) {
      for (int i = 0; i < 64; ++i) {
        hipEvent_t e;
        hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) return err;
        t_events.push_back(e);
      }
    }
    return hipEventRecord(t_events[used], s);
  }
  hipError_t end(hipStream_t s, int nlaunch, double bytes_each) {
    if (!on) return hipSuccess;
    hipError_t err = hipEventRecord(t_events[used + 1], s);
    used += 2;
    launches += nlaunch;
    bytes += nlaunch * bytes_each;
    return err;
  }
  // after a stream sync: summed milliseconds
  double total_ms() const {
    double t = 0.0;
    for (size_t i = 0; i + 1 < used; i += 2) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, t_events[i], t_events[i + 1]) == hipSuccess) t += ms;
    }
    return t;
  }
};

#define FA_HIP(expr)                          \
  do {                                        \
    hipError_t e_ = (expr);                   \
    if (e_ != hipSuccess) return FA_ERR_HIP;  \
  } while (0)

inline char* at(void* base, size_t off) { return (char*)base + off; }
inline const char* col(const void* V, int64_t ldv, int j, size_t es) {
  return (const char*)V + (size_t)j * ldv * es;
}
}  // namespace

// --------------------------------------------------------------------------
// chain: one launch of out = alpha A x + beta x + g0 y0 + g1 y1
// --------------------------------------------------------------------------
static int chain(const Op& op, const void* x, const void* y0, const void* y1, void* out,
                 const ChainCoef& k, hipStream_t s, Prof* prof) {
  (void)prof;
  FA_HIP(launch_chain(op, x, y0, y1, out, k, s));
  return FA_OK;
}

// y = A x
int op_apply(const Op& op, const void* x, void* y, hipStream_t s) {
  return chain(op, x, nullptr, nullptr, y, ChainCoef{1.0, 0.0, 0.0, 0.0}, s, nullptr);
}

// q(A) x by the recurrence of the polynomial (K products with A).  The result
// is written to `out` unless K == 1 and out == x (the single step reads x with
// neighbours), in which case it goes to t1.  out may equal x for K >= 2 (the
// last step reads x pointwise only).  t1, t2 must differ from x and out.
// Returns the buffer holding q(A) x through *res.
static int poly_apply(const Op& op, const Poly& q, const void* x, void* out, void* t1, void* t2,
                      const void** res, hipStream_t s, Prof* prof, int64_t* mvms) {
  const int K = q.degree;
  if (q.method < 0 || K == 0) {
    // q == 1: the caller treats x itself as the result
    *res = x;
    return FA_OK;
  }
  *mvms += K;
  if (K == 1 && out == x) out = t1;
  if (q.method == FA_POLY_CHEB) {
    // Clenshaw (Sec. 5.1) with Ahat = sig A + tau I:
    //   b_k = c_k x + 2 Ahat b_{k+1} - b_{k+2},  q(A) x = c_0 x + Ahat b_1 - b_2,
    // b_K = c_K x and b_{K+1} = 0 are folded into the first launches.
    const std::vector<double>& c = q.c;
    const double sig = 2.0 / (q.b - q.a), tau = -(q.a + q.b) / (q.b - q.a);
    if (K == 1) {
      int st = chain(op, x, nullptr, nullptr, out, ChainCoef{sig * c[1], tau * c[1] + c[0], 0, 0},
                     s, prof);
      *res = out;
      return st;
    }
    // b_{K-1} = 2 Ahat (c_K x) + c_{K-1} x
    int st = chain(op, x, nullptr, nullptr, t1,
                   ChainCoef{2 * sig * c[K], 2 * tau * c[K] + c[K - 1], 0, 0}, s, prof);
    if (st) return st;
    if (K == 2) {  // q(A) x = c_0 x + Ahat b_1 - b_2, b_2 = c_2 x
      st = chain(op, t1, x, nullptr, out, ChainCoef{sig, tau, c[0] - c[2], 0}, s, prof);
      *res = out;
      return st;
    }
    // b_{K-2} = 2 Ahat b_{K-1} + c_{K-2} x - c_K x
    st = chain(op, t1, x, nullptr, t2, ChainCoef{2 * sig, 2 * tau, c[K - 2] - c[K], 0}, s, prof);
    if (st) return st;
    void* bk1 = t2;  // b_{k+1}
    void* bk2 = t1;  // b_{k+2}, overwritten by b_k
    if (prof && K >= 4) FA_HIP(prof->begin(s));
    for (int k = K - 3; k >= 1; --k) {
      st = chain(op, bk1, x, bk2, bk2, ChainCoef{2 * sig, 2 * tau, c[k], -1.0}, s, prof);
      if (st) return st;
      std::swap(bk1, bk2);
    }
    if (prof && K >= 4) FA_HIP(prof->end(s, K - 3, chain_bytes(op, true, true)));
    st = chain(op, bk1, x, bk2, out, ChainCoef{sig, tau, c[0], -1.0}, s, prof);
    *res = out;
    return st;
  }
  // Newton form on Leja points, Horner-type recurrence (Sec. 5.2):
  //   r_K = eta_K x,  r_j = (A - theta_j) r_{j+1} / rho + eta_j x
  const std::vector<cd>& th = q.theta;
  const std::vector<cd>& eta = q.eta;
  const double rho = q.rho;
  void* cur = nullptr;
  {
    void* dst = (K == 1) ? out : t1;
    const cd a = eta[K] / rho;
    int st = chain(op, x, nullptr, nullptr, dst, ChainCoef{a, eta[K - 1] - th[K - 1] * a, 0, 0},
                   s, prof);
    if (st) return st;
    cur = dst;
  }
  if (prof && K >= 3) FA_HIP(prof->begin(s));
  for (int j = K - 2; j >= 0; --j) {
    void* dst = (j == 0) ? out : (cur == t1 ? t2 : t1);
    int st = chain(op, cur, x, nullptr, dst, ChainCoef{1.0 / rho, -th[j] / rho, eta[j], 0}, s,
                   prof);
    if (st) return st;
    cur = dst;
    if (prof && K >= 3 && j == 1) FA_HIP(prof->end(s, K - 2, chain_bytes(op, true, false)));
  }
  *res = cur;
  return FA_OK;
}

int poly_apply_public(const Op& op, const void* x, void* y, void* ws, hipStream_t s) {
  const Layout L = make_layout(op, 1);
  void* t1 = at(ws, L.off_P);
  void* t2 = at(ws, L.off_Q);
  const void* res = nullptr;
  int64_t mv = 0;
  int st = poly_apply(op, op.poly, x, y, t1, t2, &res, s, nullptr, &mv);
  if (st) return st;
  if (res != y) FA_HIP(hipMemcpyAsync(y, res, op.n * elem_size(op.dtype), hipMemcpyDeviceToDevice, s));
  return FA_OK;
}

// --------------------------------------------------------------------------
// the preconditioned Arnoldi / Lanczos loop
// --------------------------------------------------------------------------
namespace {
struct HostH {
  int ldh = 0;
  int dtype = FA_F64;
  std::vector<double> buf;  // column-major, ldh rows, (complex interleaved)
  cd get(int i, int j) const {
    if (dtype == FA_C128) return cd(buf[2 * ((size_t)j * ldh + i)], buf[2 * ((size_t)j * ldh + i) + 1]);
    return cd(buf[(size_t)j * ldh + i], 0.0);
  }
};

// z = H_m^{-1/2} (beta e_1) from the host copy of H
int host_coeffs(const HostH& H, int m, bool lanczos, double beta, std::vector<cd>& z) {
  z.assign(m, cd(0.0));
  if (lanczos) {
    std::vector<double> al(m), of(std::max(m - 1, 1)), zr(m);
    for (int i = 0; i < m; ++i) al[i] = H.get(i, i).real();
    for (int i = 0; i + 1 < m; ++i) of[i] = H.get(i + 1, i).real();
    const int st = tridiag_invsqrt_e1(m, al.data(), of.data(), beta, zr.data());
    if (st != DENSE_OK) return FA_ERR_HESSENBERG;
    for (int i = 0; i < m; ++i) z[i] = zr[i];
    return FA_OK;
  }
  std::vector<cd> Hc((size_t)m * m);
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < m; ++i) Hc[(size_t)j * m + i] = (i <= j + 1) ? H.get(i, j) : cd(0.0);
  const int st = hess_invsqrt_e1(m, Hc.data(), m, beta, z.data());
  if (st != DENSE_OK) return FA_ERR_HESSENBERG;
  if (H.dtype == FA_F64)
    for (auto& v : z) v = cd(v.real(), 0.0);
  return FA_OK;
}

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}
}  // namespace

int apply(const Op& op, int kind, const void* d_b, void* d_x, int m_max, double tol,
          int check_every, void* ws, size_t ws_bytes, uint32_t flags, hipStream_t s,
          fa_stats* stats) {
  const double t0 = now_ms();
  fa_stats S;
  std::memset(&S, 0, sizeof(S));
  const Layout L = make_layout(op, m_max);
  if (!ws || ws_bytes < L.bytes || ((uintptr_t)ws & 255)) return FA_ERR_WORKSPACE;
  const size_t es = elem_size(op.dtype);
  const int64_t n = op.n;
  const bool lanczos = (op.flags & FA_HERMITIAN) && !(flags & FA_FORCE_ARNOLDI);
  const Poly& q = op.poly;
  const int K = (q.method < 0) ? 0 : q.degree;
  const int k_chk = check_every > 0 ? check_every : std::max(1, 64 / (K + 1));

  char* V = at(ws, L.off_V);
  void* U = at(ws, L.off_U);
  void* P = at(ws, L.off_P);
  void* Qb = at(ws, L.off_Q);
  void* part = at(ws, L.off_part);
  char* hcur = at(ws, L.off_h);
  char* Hd = at(ws, L.off_H);
  double* nrm = (double*)at(ws, L.off_nrm);
  void* zd = at(ws, L.off_z);
  auto Vc = [&](int j) -> char* { return V + (size_t)j * L.ldv * es; };
  auto Hcol = [&](int j) -> char* { return Hd + (size_t)j * L.ldh * es; };

  Prof prof;
  prof.on = (flags & FA_PROFILE) != 0;
  Prof* pp = prof.on ? &prof : nullptr;
  int64_t mvms = 0;
  int st = FA_OK;

  // Sec. 4: square root through the inverse square root, b' = A b
  const void* bsrc = d_b;
  if (kind == FA_SQRT) {
    st = chain(op, d_b, nullptr, nullptr, U, ChainCoef{1.0, 0.0, 0.0, 0.0}, s, pp);
    if (st) return st;
    ++mvms;
    bsrc = U;
  }
  // Algorithm 1: c = q(A) b', beta = ||c||, v_1 = c / beta
  {
    const void* res = nullptr;
    void* t1 = (bsrc == U) ? P : U;
    void* t2 = (bsrc == U) ? Qb : P;
    st = poly_apply(op, q, bsrc, Vc(0), t1, t2, &res, s, pp, &mvms);
    if (st) return st;
    if (res != Vc(0)) FA_HIP(launch_scale(op.dtype, n, cd(1.0), res, Vc(0), s));
    FA_HIP(launch_update(op.dtype, n, 0, V, L.ldv, hcur, Vc(0), part, nrm, s));
    FA_HIP(launch_normalize(op.dtype, n, Vc(0), nrm, Vc(0), nullptr, s));
  }
  double beta2 = 0.0;
  FA_HIP(hipMemcpyAsync(&beta2, nrm, sizeof(double), hipMemcpyDeviceToHost, s));
  FA_HIP(hipStreamSynchronize(s));
  if (!std::isfinite(beta2)) return FA_ERR_NONFINITE;
  const double beta = std::sqrt(beta2);
  if (beta == 0.0) {
    FA_HIP(launch_scale(op.dtype, n, cd(0.0), Vc(0), d_x, s));
    FA_HIP(hipStreamSynchronize(s));
    S.converged = 1;
    S.mvms = mvms;
    S.ms_total = now_ms() - t0;
    if (stats) *stats = S;
    return FA_OK;
  }

  HostH H;
  H.ldh = L.ldh;
  H.dtype = op.dtype;
  H.buf.assign((size_t)L.ldh * m_max * (op.dtype == FA_C128 ? 2 : 1), 0.0);
  int copied = 0;          // columns of H already on the host
  double colmax = 0.0;     // largest column norm of H seen (breakdown scale)
  std::vector<cd> z, zprev;
  int m = m_max;
  bool converged = false, breakdown = false;
  double est = 1.0;
  int64_t ips = 0;

  for (int j = 0; j < m_max; ++j) {
    char* vj = Vc(j);
    char* w = Vc(j + 1);
    // three-stage preconditioned product w = q(A) q(A) A v_j (Algorithm 1)
    if (K == 0) {
      st = chain(op, vj, nullptr, nullptr, w, ChainCoef{1.0, 0.0, 0.0, 0.0}, s, pp);
      if (st) return st;
      ++mvms;
    } else {
      st = chain(op, vj, nullptr, nullptr, U, ChainCoef{1.0, 0.0, 0.0, 0.0}, s, pp);
      if (st) return st;
      ++mvms;
      const void* y = nullptr;
      st = poly_apply(op, q, U, U, P, Qb, &y, s, pp, &mvms);
      if (st) return st;
      void* t1 = (y == P) ? U : P;
      const void* r2 = nullptr;
      st = poly_apply(op, q, y, w, t1, Qb, &r2, s, pp, &mvms);
      if (st) return st;
      if (r2 != w) FA_HIP(launch_scale(op.dtype, n, cd(1.0), r2, w, s));
    }
    // orthogonalization against v_1..v_j (h_ij = v_i^H w)
    if (lanczos) {
      if (j > 0)  // w -= beta_{j-1} v_{j-1}, beta_{j-1} = H(j, j-1)
        FA_HIP(launch_update(op.dtype, n, 1, Vc(j - 1), L.ldv, Hcol(j - 1) + (size_t)j * es, w,
                             part, nullptr, s));
      FA_HIP(launch_project(op.dtype, n, 1, vj, L.ldv, w, part, hcur, Hcol(j) + (size_t)j * es, 1,
                            s));
      FA_HIP(launch_update(op.dtype, n, 1, vj, L.ldv, hcur, w, part, nrm, s));
      ips += 2;
    } else {  // classical Gram-Schmidt, twice
      FA_HIP(launch_project(op.dtype, n, j + 1, V, L.ldv, w, part, hcur, Hcol(j), 1, s));
      FA_HIP(launch_update(op.dtype, n, j + 1, V, L.ldv, hcur, w, part, nullptr, s));
      FA_HIP(launch_project(op.dtype, n, j + 1, V, L.ldv, w, part, hcur, Hcol(j), 2, s));
      FA_HIP(launch_update(op.dtype, n, j + 1, V, L.ldv, hcur, w, part, nrm, s));
      ips += 2 * (j + 1) + 1;
    }
    // h_{j+1,j} = ||w||, v_{j+1} = w / h_{j+1,j}
    FA_HIP(launch_normalize(op.dtype, n, w, nrm, w, Hcol(j) + (size_t)(j + 1) * es, s));

    const int jj = j + 1;
    const bool check = (tol > 0.0) ? (jj % k_chk == 0 || jj == m_max) : (jj == m_max);
    if (!check) continue;
    // copy the new columns of H to the host
    FA_HIP(hipMemcpyAsync(H.buf.data() + (size_t)copied * L.ldh * (es / 8), Hcol(copied),
                          (size_t)(jj - copied) * L.ldh * es, hipMemcpyDeviceToHost, s));
    FA_HIP(hipStreamSynchronize(s));
    // scan new columns for a lucky breakdown / nonfinite entries
    int mb = -1;
    for (int c = copied; c < jj; ++c) {
      // Lanczos keeps only H(c, c) and H(c + 1, c) on the device; the entry
      // above the diagonal is the symmetric H(c, c - 1)
      double cn = 0.0;
      for (int i = lanczos ? c : 0; i <= c + 1; ++i) {
        const cd v = H.get(i, c);
        if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) return FA_ERR_NONFINITE;
        cn += std::norm(v);
      }
      if (lanczos && c > 0) cn += std::norm(H.get(c, c - 1));
      colmax = std::max(colmax, std::sqrt(cn));
      if (std::abs(H.get(c + 1, c)) <= 1e-12 * colmax) {
        mb = c + 1;
        break;
      }
    }
    copied = jj;
    if (mb > 0) {
      m = mb;
      breakdown = converged = true;
      break;
    }
    if (tol <= 0.0) break;
    const double th = now_ms();
    st = host_coeffs(H, jj, lanczos, beta, z);
    S.ms_host_fH += now_ms() - th;
    ++S.checks;
    if (st) return st;
    double dn = 0.0, zn = 0.0;
    for (int i = 0; i < jj; ++i) {
      const cd zp = (i < (int)zprev.size()) ? zprev[i] : cd(0.0);
      dn += std::norm(z[i] - zp);
      zn += std::norm(z[i]);
    }
    est = std::sqrt(dn / zn);
    zprev = z;
    if (est <= tol) {
      m = jj;
      converged = true;
      break;
    }
  }
  // final coefficients (if the loop did not end on a fresh check of size m)
  if ((int)z.size() != m || breakdown) {
    if (copied < m) {
      FA_HIP(hipMemcpyAsync(H.buf.data() + (size_t)copied * L.ldh * (es / 8), Hcol(copied),
                            (size_t)(m - copied) * L.ldh * es, hipMemcpyDeviceToHost, s));
      FA_HIP(hipStreamSynchronize(s));
    }
    const double th = now_ms();
    st = host_coeffs(H, m, lanczos, beta, z);
    S.ms_host_fH += now_ms() - th;
    if (st) return st;
  }
  // f_m = V_m z_m
  std::vector<double> zh((size_t)m * (es / 8));
  for (int i = 0; i < m; ++i) {
    if (op.dtype == FA_C128) {
      zh[2 * i] = z[i].real();
      zh[2 * i + 1] = z[i].imag();
    } else {
      zh[i] = z[i].real();
    }
  }
  FA_HIP(hipMemcpyAsync(zd, zh.data(), zh.size() * sizeof(double), hipMemcpyHostToDevice, s));
  FA_HIP(launch_combine(op.dtype, n, m, V, L.ldv, zd, d_x, s));
  FA_HIP(hipStreamSynchronize(s));

  S.iters = m;
  S.converged = converged ? 1 : 0;
  S.breakdown = breakdown ? 1 : 0;
  S.mvms = mvms;
  S.inner_products = ips;
  S.est_rel_change = est;
  S.h_last = (m <= (int)copied) ? std::abs(H.get(m, m - 1)) : 0.0;
  S.ms_total = now_ms() - t0;
  if (prof.on) {
    S.ms_chain = prof.total_ms();
    S.n_chain = prof.launches;
    S.chain_bytes = S.n_chain ? prof.bytes / (double)S.n_chain : 0.0;
  }
  if (stats) *stats = S;
  return converged ? FA_OK : FA_WARN_NOT_CONVERGED;
}

// --------------------------------------------------------------------------
// polynomial setup
// --------------------------------------------------------------------------
size_t poly_workspace_bytes(const Op& op, int degree, int method) {
  if (method == FA_POLY_CHEB || degree == 0) return 0;
  return make_layout(op, degree + 1).bytes;
}

int poly_setup(Op& op, int degree, int method, const void* d_start, void* ws, size_t ws_bytes,
               hipStream_t s, int64_t* mvms_setup) {
  if (degree < 0 || degree > 512) return FA_ERR_ARG;
  if (method == FA_POLY_AUTO) method = op.has_interval ? FA_POLY_CHEB : FA_POLY_RITZ;
  Poly q;
  *mvms_setup = 0;
  if (degree == 0) {
    q.method = -1;
    q.degree = 0;
    op.poly = q;
    op.poly_ready = true;
    return FA_OK;
  }
  if (method == FA_POLY_CHEB) {
    if (!op.has_interval) return FA_ERR_NO_INTERVAL;
    q.method = FA_POLY_CHEB;
    q.degree = degree;
    q.a = op.lo;
    q.b = op.hi;
    q.c.resize(degree + 1);
    cheb_coefficients(q.a, q.b, degree, q.c.data());
    // positivity of q on [a, b]: 10^4 equispaced points and the nodes
    const int npts = 10000;
    for (int i = 0; i < npts; ++i) {
      const double zz = q.a + (q.b - q.a) * i / (npts - 1);
      if (!(cheb_eval(q.c.data(), degree, q.a, q.b, zz) > 0.0)) return FA_ERR_BRANCH;
    }
    for (int k = 0; k <= degree; ++k) {
      const double zz = 0.5 * (q.a + q.b) + 0.5 * (q.b - q.a) * std::cos(M_PI * (k + 0.5) / (degree + 1));
      if (!(cheb_eval(q.c.data(), degree, q.a, q.b, zz) > 0.0)) return FA_ERR_BRANCH;
    }
    op.poly = q;
    op.poly_ready = true;
    return FA_OK;
  }
  if (method != FA_POLY_RITZ) return FA_ERR_ARG;
  if (!d_start) return FA_ERR_ARG;
  // d = degree + 1 Arnoldi steps on A itself (CGS2) from the given start vector
  const int d = degree + 1;
  const Layout L = make_layout(op, d);
  if (!ws || ws_bytes < L.bytes || ((uintptr_t)ws & 255)) return FA_ERR_WORKSPACE;
  const size_t es = elem_size(op.dtype);
  const int64_t n = op.n;
  char* V = at(ws, L.off_V);
  void* part = at(ws, L.off_part);
  char* hcur = at(ws, L.off_h);
  char* Hd = at(ws, L.off_H);
  double* nrm = (double*)at(ws, L.off_nrm);
  auto Vc = [&](int j) -> char* { return V + (size_t)j * L.ldv * es; };
  auto Hcol = [&](int j) -> char* { return Hd + (size_t)j * L.ldh * es; };
  FA_HIP(launch_update(op.dtype, n, 0, V, L.ldv, hcur, (void*)d_start, part, nrm, s));
  FA_HIP(launch_normalize(op.dtype, n, d_start, nrm, Vc(0), nullptr, s));
  for (int j = 0; j < d; ++j) {
    char* w = Vc(j + 1);
    int st = op_apply(op, Vc(j), w, s);
    if (st) return st;
    ++*mvms_setup;
    FA_HIP(launch_project(op.dtype, n, j + 1, V, L.ldv, w, part, hcur, Hcol(j), 1, s));
    FA_HIP(launch_update(op.dtype, n, j + 1, V, L.ldv, hcur, w, part, nullptr, s));
    FA_HIP(launch_project(op.dtype, n, j + 1, V, L.ldv, w, part, hcur, Hcol(j), 2, s));
    FA_HIP(launch_update(op.dtype, n, j + 1, V, L.ldv, hcur, w, part, nrm, s));
    FA_HIP(launch_normalize(op.dtype, n, w, nrm, w, Hcol(j) + (size_t)(j + 1) * es, s));
  }
  HostH H;
  H.ldh = L.ldh;
  H.dtype = op.dtype;
  H.buf.assign((size_t)L.ldh * d * (es / 8), 0.0);
  FA_HIP(hipMemcpyAsync(H.buf.data(), Hd, (size_t)L.ldh * d * es, hipMemcpyDeviceToHost, s));
  FA_HIP(hipStreamSynchronize(s));
  // steps completed before a lucky breakdown (same rule as in fa_apply)
  int steps = d;
  double colmax = 0.0;
  for (int c = 0; c < d; ++c) {
    double cn = 0.0;
    for (int i = 0; i <= c + 1; ++i) cn += std::norm(H.get(i, c));
    if (!std::isfinite(cn)) return FA_ERR_NONFINITE;
    colmax = std::max(colmax, std::sqrt(cn));
    if (std::abs(H.get(c + 1, c)) <= 1e-12 * colmax) {
      steps = c + 1;
      break;
    }
  }
  std::vector<cd> Hc((size_t)steps * steps), ev(steps);
  for (int j = 0; j < steps; ++j)
    for (int i = 0; i < steps; ++i) Hc[(size_t)j * steps + i] = (i <= j + 1) ? H.get(i, j) : cd(0.0);
  if (hess_eigenvalues(steps, Hc.data(), steps, ev.data()) != DENSE_OK) return FA_ERR_HESSENBERG;
  const bool real_op = op.dtype == FA_F64;
  for (auto& t : ev) {
    if (!(t.real() > 0.0)) return FA_ERR_BRANCH;  // Ritz value outside the right half-plane
    if (real_op) {
      if (std::fabs(t.imag()) > 1e-10 * std::abs(t)) return FA_ERR_UNSUPPORTED;
      t = cd(t.real(), 0.0);
    }
  }
  q.method = FA_POLY_RITZ;
  q.theta = leja_order(ev, real_op);
  q.degree = (int)q.theta.size() - 1;
  q.rho = leja_capacity(q.theta);
  q.eta = newton_invsqrt(q.theta, q.rho);
  if (real_op)
    for (auto& e : q.eta) e = cd(e.real(), 0.0);
  op.poly = q;
  op.poly_ready = true;
  return FA_OK;
}

}  // namespace fa
