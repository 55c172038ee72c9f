// Host runtime of the method: workspace layout, the polynomial chain, the
// preconditioned Arnoldi / Lanczos loop with host FP64 stopping checks, and
// the polynomial setup.  All device work is enqueued on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "dense.hpp"
#include "fa_internal.hpp"
#include "solver.hpp"

namespace fa {

uint64_t next_op_uid() {
  static std::atomic<uint64_t> counter{0};
  return ++counter;
}

// --------------------------------------------------------------------------
// workspace layout (every region 256-byte aligned)
// --------------------------------------------------------------------------
Layout make_layout(const Op& op, int m_max, uint32_t flags, bool with_poly) {
  Layout L;
  const size_t es = elem_size(op.dtype);
  L.ldv = round_up(op.n, 32);
  // Lanczos keeps only the diagonal and subdiagonal of H: column j holds
  // (H(j, j), H(j + 1, j)); Arnoldi keeps full columns of m_max + 1 rows
  L.band = (op.flags & FA_HERMITIAN) && !(flags & FA_FORCE_ARNOLDI);
  L.ldh = L.band ? 2 : m_max + 1;
  const RedPlan rp = red_plan(op.n);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (size_t)round_up((int64_t)bytes, 256);
    return o;
  };
  // two-pass Lanczos keeps a ring of three basis vectors; right
  // preconditioning also stores y_j = q(A) v_j (two-pass: only the latest)
  const bool two_pass = (flags & FA_TWO_PASS) != 0;
  const int nbasis = two_pass ? 3 : m_max + 1;
  L.off_V = take((size_t)nbasis * L.ldv * es);
  L.off_Y = (flags & FA_RIGHT_PREC) ? take((size_t)(two_pass ? 1 : m_max) * L.ldv * es) : 0;
  L.off_U = take((size_t)L.ldv * es);
  L.off_P = take((size_t)L.ldv * es);
  L.off_Q = take((size_t)L.ldv * es);
  L.off_R = take((size_t)L.ldv * es);
  L.off_S = take((size_t)L.ldv * es);
  // per-block partial sums of one projection (Lanczos projects on one
  // vector; the delayed-reorthogonalization step projects two vectors on
  // m_max + 1 columns)
  L.off_part = take((size_t)(L.band ? 3 : 2 * m_max + 4) *
                        std::max(rp.nblk, proj_nblk(op.n, op.dtype)) * es + 64);
  L.off_h = take((size_t)(2 * m_max + 4) * es);
  L.off_dc = take((size_t)(2 * m_max + 4) * es);
  L.off_H = take((size_t)L.ldh * m_max * es);
  L.off_nrm = take(8 * sizeof(double));
  L.off_z = take((size_t)(m_max + 1) * es);
  if (with_poly && op.poly_ready && op.poly.method == FA_POLY_LS)
    L.off_W = take((size_t)(op.poly.degree + 1) * L.ldv * es);
  L.scr_bytes = op_scratch_bytes(op);
  if (L.scr_bytes) L.off_scr = take(L.scr_bytes);
  L.bytes = off;
  return L;
}

// --------------------------------------------------------------------------
// profiling: HIP events around chain launches (thread-local pool)
// --------------------------------------------------------------------------
namespace {
thread_local std::vector<hipEvent_t> t_events;
// per device: an event (no timing) marking the end of a check's copies
thread_local std::vector<hipEvent_t> t_check_events;
hipError_t check_event(hipEvent_t* e) {
  int dev = 0;
  hipError_t err = hipGetDevice(&dev);
  if (err != hipSuccess) return err;
  if ((int)t_check_events.size() <= dev) t_check_events.resize(dev + 1, nullptr);
  if (!t_check_events[dev]) {
    err = hipEventCreateWithFlags(&t_check_events[dev], hipEventDisableTiming);
    if (err != hipSuccess) return err;
  }
  *e = t_check_events[dev];
  return hipSuccess;
}

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
  hipError_t reserve() {
    if (used + 2 > t_events.size()) {
      for (int i = 0; i < 64; ++i) {
        hipEvent_t e;
        hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) return err;
        t_events.push_back(e);
      }
    }
    return hipSuccess;
  }
  // a bracket of events around a run of launches (each event its own packet)
  hipError_t begin(hipStream_t s) {
    if (!on) return hipSuccess;
    hipError_t err = reserve();
    if (err != hipSuccess) return err;
    return hipEventRecord(t_events[used], s);
  }
  hipError_t end(hipStream_t s) {
    if (!on) return hipSuccess;
    hipError_t err = hipEventRecord(t_events[used + 1], s);
    used += 2;
    return err;
  }
  // the event pair one launch stamps with its own dispatch's start and end
  hipError_t pair(hipEvent_t* e0, hipEvent_t* e1) {
    hipError_t err = reserve();
    if (err != hipSuccess) return err;
    *e0 = t_events[used];
    *e1 = t_events[used + 1];
    used += 2;
    return hipSuccess;
  }
  int64_t terms = 0;  // recurrence terms of the timed launches
  void count(int nlaunch, double bytes_each, int terms_each = 1) {
    launches += nlaunch;
    bytes += nlaunch * bytes_each;
    terms += (int64_t)nlaunch * terms_each;
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
int op_apply(const Op& op, const void* x, void* y, void* ws, hipStream_t s) {
  void* sc = nullptr;
  if (ws) {
    const Layout L = make_layout(op, 1, 0);
    if (L.scr_bytes) sc = at(ws, L.off_scr);
  }
  if (!sc && op.kind == OP_WILSON && op.q2) return FA_ERR_WORKSPACE;  // Q x has to live somewhere
  OpScratchScope csr(op, sc, s);
  if (!csr.ok()) return FA_ERR_HIP;
  return chain(op, x, nullptr, nullptr, y, ChainCoef{1.0, 0.0, 0.0, 0.0}, s, nullptr);
}

// The terms of q(A) v (K products with A):
//   Chebyshev, Clenshaw (Sec. 5.1) with Ahat = sig A + tau I,
//     b_k = c_k v + 2 Ahat b_{k+1} - b_{k+2},  q(A) v = c_0 v + Ahat b_1 - b_2;
//     b_K = c_K v and b_{K+1} = 0 are folded into the first two terms.
//   Newton form on Leja points, Horner-type recurrence (Sec. 5.2),
//     r_K = eta_K v,  r_j = (A - theta_j) r_{j+1} / rho + eta_j v.
std::vector<Term> poly_terms(const Poly& q) {
  std::vector<Term> T;
  const int K = q.degree;
  if (q.method == FA_POLY_CHEB) {
    const std::vector<double>& c = q.c;
    const double sig = 2.0 / (q.b - q.a), tau = -(q.a + q.b) / (q.b - q.a);
    if (K == 1) {
      T.push_back({ChainCoef{sig * c[1], tau * c[1] + c[0], 0, 0}, false, false});
      return T;
    }
    T.push_back({ChainCoef{2 * sig * c[K], 2 * tau * c[K] + c[K - 1], 0, 0}, false, false});
    for (int i = 1; i < K; ++i) {
      const int k = K - 1 - i;  // the term produces b_k (k = 0: q(A) v)
      const double a = (k == 0) ? sig : 2 * sig, b = (k == 0) ? tau : 2 * tau;
      const double g0 = c[k] - (i == 1 ? c[K] : 0.0);
      T.push_back({ChainCoef{a, b, g0, i >= 2 ? -1.0 : 0.0}, true, i >= 2});
    }
    return T;
  }
  const std::vector<cd>& th = q.theta;
  const std::vector<cd>& eta = q.eta;
  const double rho = q.rho;
  const cd a = eta[K] / rho;
  T.push_back({ChainCoef{a, eta[K - 1] - th[K - 1] * a, 0, 0}, false, false});
  for (int j = K - 2; j >= 0; --j)
    T.push_back({ChainCoef{1.0 / rho, -th[j] / rho, eta[j], 0}, true, false});
  return T;
}

// q(A) x for a Ritz polynomial of a real operator in real blocks (Horner over
// the blocks, last to first):  R = a_L v + b_L u  (u = A v);  then for each
// block B:
//   real node theta:  R <- (A - theta) R / rho + a_B v
//   pair theta, conj(theta), c = Re theta, s = Im theta:
//     t  = (A - c) R / rho + d v,               d = -a_B rho / c
//     R <- (A - c) t / rho + (s/rho)^2 R + f u, f = b_B + a_B / c
// which adds ((A - c)^2 + s^2) R / rho^2 + a_B v + b_B u, two launches with at
// most two extra vectors each.
static int poly_apply_blocks(const Op& op, const Poly& q, const void* x, void* out,
                             void* const tmp[4], const void** res, hipStream_t s, int64_t* mvms) {
  const std::vector<Poly::Block>& B = q.blocks;
  const int L = (int)B.size();
  const double rho = q.rho;
  bool need_u = false;
  for (const auto& b : B) need_u |= b.pair;
  void* u = tmp[3];
  if (need_u) {
    FA_HIP(launch_chain(op, x, nullptr, nullptr, u, ChainCoef{1.0, 0.0, 0.0, 0.0}, s));
    *mvms += 1;
  }
  // R = a_L v + b_L u (no product with A: alpha = 0)
  void* R = tmp[0];
  FA_HIP(launch_chain(op, x, nullptr, need_u ? u : nullptr, R,
                      ChainCoef{0.0, B[L - 1].a, 0.0, B[L - 1].b}, s));
  void* spare[2] = {tmp[1], tmp[2]};
  for (int k = L - 2; k >= 0; --k) {
    const auto& b = B[k];
    const bool last = k == 0;
    void* dst = spare[0];
    if (!b.pair) {
      if (last && out != R) dst = out;
      FA_HIP(launch_chain(op, R, x, nullptr, dst, ChainCoef{1.0 / rho, -b.re / rho, b.a, 0.0}, s));
      *mvms += 1;
      spare[0] = R;
      R = dst;
    } else {
      const double c = b.re, e = (b.im / rho) * (b.im / rho);
      const double d = -b.a * rho / c, f = b.b + b.a / c;
      void* t = spare[0];
      FA_HIP(launch_chain(op, R, x, nullptr, t, ChainCoef{1.0 / rho, -c / rho, d, 0.0}, s));
      // R' may overwrite R (read pointwise) or go to out (never read here)
      void* d2 = (last && out != t) ? out : R;
      FA_HIP(launch_chain(op, t, R, u, d2, ChainCoef{1.0 / rho, -c / rho, e, f}, s));
      *mvms += 2;
      R = d2;
    }
  }
  *res = R;
  return FA_OK;
}

// q(A) x for the least-squares polynomial (Sec. 5.3) by the recurrence of
// its orthonormal basis polynomials with A in place of z:
//   w_0 = x / sqrt(N),
//   w_k = (A w_{k-1} - sum_{i<k} h_{i,k-1} w_i) / h_{k,k-1},  k = 1..K,
//   q(A) x = sum_k alpha_k w_k,
// K products with A and no inner products.  W holds the K + 1 vectors w_k
// (leading dimension round_up(n, 32), as the basis); the result goes to out
// (which may alias x: x is read only by the first launch).
static int poly_apply_ls(const Op& op, const Poly& q, const void* x, void* out, void* W,
                         const void** res, hipStream_t s, int64_t* mvms) {
  if (!W) return FA_ERR_WORKSPACE;
  const int K = q.degree, d = K + 1;
  const size_t es = elem_size(op.dtype);
  const int64_t ldv = round_up(op.n, 32);
  auto Wc = [&](int j) -> void* { return (char*)W + (size_t)j * ldv * es; };
  auto h = [&](int i, int j) { return q.hls[(size_t)j * d + i]; };
  FA_HIP(launch_scale(op.dtype, op.n, cd(1.0 / std::sqrt((double)q.npts)), x, Wc(0), s));
  for (int k = 1; k <= K; ++k) {
    const cd hk = h(k, k - 1);
    FA_HIP(launch_chain(op, Wc(k - 1), nullptr, nullptr, Wc(k),
                        ChainCoef{1.0 / hk, -h(k - 1, k - 1) / hk, 0.0, 0.0}, s));
    LsCoef g;
    for (int i = 0; i + 1 < k; ++i) {
      const cd gi = -h(i, k - 1) / hk;
      g.re[i] = gi.real();
      g.im[i] = gi.imag();
    }
    g.a0_re = q.alpha[0].real();
    g.a0_im = q.alpha[0].imag();
    g.ak_re = q.alpha[k].real();
    g.ak_im = q.alpha[k].imag();
    FA_HIP(launch_ls_step(op.dtype, op.n, k, W, ldv, g, k < K, out, s));
  }
  *mvms += K;
  *res = out;
  return FA_OK;
}

// q(A) x.  tmp holds 4 scratch vectors distinct from x and out.  The result
// goes to `out` when that is safe and to a scratch vector otherwise (a
// single-term launch may write over x pointwise, a two-term launch may not);
// *res names the buffer that holds q(A) x.  `fuse` is the most consecutive
// terms of the 7-point stencil one launch may take (1 to 4): groups of `fuse`
// terms while that many remain, then the largest group that fits, a pair or
// a single term.
// pm = P32 (mixed precision): x and every intermediate vector are FP32 and
// the last launch writes `out` in precision pout; pm = P64: everything FP64.
static int poly_apply(const Op& op, const Poly& q, const void* x, void* out, void* const tmp[4],
                      const void** res, hipStream_t s, Prof* prof, int64_t* mvms, int fuse,
                      Prec pm = P64, Prec pout = P64, void* wls = nullptr) {
  const int K = q.degree;
  if (q.method < 0 || K == 0) {
    *res = x;  // q == 1
    return FA_OK;
  }
  if (q.method == FA_POLY_LS) {
    if (pm != P64 || pout != P64) return FA_ERR_UNSUPPORTED;
    return poly_apply_ls(op, q, x, out, wls, res, s, mvms);
  }
  if (!q.blocks.empty()) {
    if (pm != P64) return FA_ERR_UNSUPPORTED;
    return poly_apply_blocks(op, q, x, out, tmp, res, s, mvms);
  }
  *mvms += K;
  const std::vector<Term> T = poly_terms(q);
  const int nT = (int)T.size();
  const bool pairs = fuse >= 2 && has_pair_kernel(op) && nT >= 2;
  if (!pairs) {
    // one launch per term; out_i may overwrite out_{i-2} in place (read pointwise)
    const void* xm1 = x;       // out_{i-1}
    const void* xm2 = nullptr; // out_{i-2}
    void* slot[2] = {tmp[0], tmp[1]};
    bool timing = false;
    for (int i = 0; i < nT; ++i) {
      const bool last = i == nT - 1;
      void* dst;
      if (last)
        dst = (out == xm1) ? (xm2 && xm2 != x ? (void*)xm2 : slot[i & 1]) : out;
      else
        dst = (i >= 2 && T[i].y1) ? (void*)xm2 : slot[i & 1];
      if (dst == xm1) dst = slot[(i + 1) & 1];
      const bool middle = !last && T[i].y0 && (q.method == FA_POLY_RITZ || T[i].y1);
      if (prof && middle && !timing) {
        FA_HIP(prof->begin(s));
        timing = true;
      }
      if (prof && timing && !middle) {
        FA_HIP(prof->end(s));
        timing = false;
      }
      FA_HIP(launch_chain(op, xm1, T[i].y0 ? x : nullptr, T[i].y1 ? xm2 : nullptr, dst, T[i].k, s,
                          pm, last ? pout : pm));
      if (prof && timing) prof->count(1, chain_bytes(op, T[i].y0, T[i].y1, pm));
      xm2 = xm1;
      xm1 = dst;
    }
    if (prof && timing) FA_HIP(prof->end(s));
    *res = xm1;
    return FA_OK;
  }
  // groups of g = 4, 3 or 2 terms per launch: the group (T[i], .., T[i+g-1])
  // reads out_{i-1}, out_{i-2} and x and writes out_{i+g-2}, out_{i+g-1} into
  // the buffer set not holding its inputs (the terms between stay on chip);
  // term i + 1 takes out_{i-1} and term i + 2 out_i as its y1
  const void* xm1 = x;
  const void* xm2 = nullptr;
  int set = 0;
  bool timing = false;
  int i = 0;
  for (;;) {
    const int g = (fuse >= 4 && i + 4 <= nT)   ? 4
                  : (fuse >= 3 && i + 3 <= nT) ? 3
                  : (i + 2 <= nT)              ? 2
                                               : 0;
    if (g == 0) break;
    const bool has_next = i + g < nT;  // someone reads out_{i+g-2} later
    void* o1 = has_next ? tmp[2 * set] : nullptr;
    void* o2 = tmp[2 * set + 1];
    if (!has_next && out != x && out != xm1 && out != xm2) o2 = out;
    bool middle = T[i].y0 && T[i].y1 && has_next;
    for (int t = 1; t < g; ++t) middle = middle && T[i + t].y1;
    // multi-term launches are timed by their own dispatch, pairs by a
    // bracket of events around each run of them
    const bool own = g >= 3;
    if (prof && timing && (!middle || own)) {
      FA_HIP(prof->end(s));
      timing = false;
    }
    if (prof && middle && !own && !timing) {
      FA_HIP(prof->begin(s));
      timing = true;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (prof && middle && own) FA_HIP(prof->pair(&e0, &e1));
    ChainCoef k[4];
    for (int t = 0; t < g; ++t) {
      k[t] = T[i + t].k;
      if (t > 0 && !T[i + t].y1) k[t].g1 = 0.0;
    }
    const Prec po = has_next ? pm : pout;
    if (g >= 3) {
      for (int t = 0; t < g; ++t)
        if (!T[i + t].y0) k[t].g0 = 0.0;
      FA_HIP(launch_chain_multi(op, g, xm1, x, T[i].y1 ? xm2 : nullptr, o1, o2, k, s, pm, po, 0,
                                e0, e1));
    } else {
      FA_HIP(launch_chain_pair(op, xm1, (T[i].y0 || T[i + 1].y0) ? x : nullptr,
                               T[i].y1 ? xm2 : nullptr, o1, o2, k[0], k[1], s, pm, po));
    }
    if (prof && middle)
      prof->count(1, chain_pair_bytes(op, true, true, o1 != nullptr, pm), g);
    xm2 = o1;
    xm1 = o2;
    set ^= 1;
    i += g;
  }
  if (prof && timing) FA_HIP(prof->end(s));
  if (i < nT) {  // odd number of terms: the last one alone (pointwise in out)
    void* dst = (out == xm1) ? tmp[2 * set] : out;
    FA_HIP(launch_chain(op, xm1, T[i].y0 ? x : nullptr, T[i].y1 ? xm2 : nullptr, dst, T[i].k, s,
                        pm, pout));
    xm1 = dst;
  }
  *res = xm1;
  return FA_OK;
}

int poly_apply_chain(const Op& op, const void* x, void* out, void* const tmp[4],
                     const void** res, hipStream_t s, int64_t* mvms, Prec p) {
  return poly_apply(op, op.poly, x, out, tmp, res, s, nullptr, mvms, 4, p, p);
}

int poly_apply_public(const Op& op, const void* x, void* y, void* ws, hipStream_t s) {
  const Layout L = make_layout(op, 1, 0);
  OpScratchScope csr(op, L.scr_bytes ? at(ws, L.off_scr) : nullptr, s);
  if (!csr.ok()) return FA_ERR_HIP;
  void* const tmp[4] = {at(ws, L.off_P), at(ws, L.off_Q), at(ws, L.off_R), at(ws, L.off_S)};
  const void* res = nullptr;
  int64_t mv = 0;
  int st = poly_apply(op, op.poly, x, y, tmp, &res, s, nullptr, &mv, 4, P64, P64,
                      L.off_W ? at(ws, L.off_W) : nullptr);
  if (st) return st;
  if (res != y) FA_HIP(hipMemcpyAsync(y, res, op.n * elem_size(op.dtype), hipMemcpyDeviceToDevice, s));
  return FA_OK;
}

// --------------------------------------------------------------------------
// the preconditioned Arnoldi / Lanczos loop
// --------------------------------------------------------------------------
namespace {
// Page-locked host memory for the iteration's small copies (columns of H,
// projections, norms, coefficients).  A copy into pageable memory is staged
// by the runtime through its own buffer and blocks the calling thread; one
// into page-locked memory queues on the stream like a kernel.  The memory is
// coherent (fine-grained), so a kernel can write the checks' data into it and
// the host can watch a flag there.  Buffers are pooled across calls and
// threads and kept for the life of the process.
class PinnedPool {
 public:
  void* take(size_t bytes) {
    {
      std::lock_guard<std::mutex> g(mu_);
      size_t best = free_.size();
      for (size_t i = 0; i < free_.size(); ++i)
        if (free_[i].second >= bytes && (best == free_.size() || free_[i].second < free_[best].second))
          best = i;
      if (best < free_.size()) {
        void* p = free_[best].first;
        free_.erase(free_.begin() + best);
        return p;
      }
    }
    void* p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocCoherent) != hipSuccess) return nullptr;
    std::lock_guard<std::mutex> g(mu_);
    size_of_[p] = bytes;
    return p;
  }
  void give(void* p) {
    std::lock_guard<std::mutex> g(mu_);
    free_.push_back({p, size_of_[p]});
  }

 private:
  std::mutex mu_;
  std::vector<std::pair<void*, size_t>> free_;
  std::unordered_map<void*, size_t> size_of_;
};
PinnedPool& pinned_pool() {
  static PinnedPool* pool = new PinnedPool;  // never destroyed (outlives the runtime's users)
  return *pool;
}
struct PinnedLease {
  void* p = nullptr;
  // bytes == 0: no area (the pool is not touched)
  explicit PinnedLease(size_t bytes) : p(bytes ? pinned_pool().take(bytes) : nullptr) {}
  ~PinnedLease() {
    if (p) pinned_pool().give(p);
  }
  PinnedLease(const PinnedLease&) = delete;
  PinnedLease& operator=(const PinnedLease&) = delete;
};

struct HostH {
  int ldh = 0;
  bool band = false;        // Lanczos: column j holds rows j and j + 1 only
  int dtype = FA_F64;
  double* buf = nullptr;    // column-major, ldh rows, (complex interleaved)
  std::vector<double> own;  // storage when buf is not given
  size_t off(int i, int j) const { return (size_t)j * ldh + (band ? i - j : i); }
  cd get(int i, int j) const {
    const size_t o = off(i, j);
    if (dtype == FA_C128) return cd(buf[2 * o], buf[2 * o + 1]);
    return cd(buf[o], 0.0);
  }
  void set(int i, int j, cd v) {
    const size_t o = off(i, j);
    if (dtype == FA_C128) {
      buf[2 * o] = v.real();
      buf[2 * o + 1] = v.imag();
    } else {
      buf[o] = v.real();
    }
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
  int st;
  if (H.dtype == FA_F64) {  // real Francis double-shift QR on the host copy
    st = real_hess_invsqrt_e1(m, H.buf, H.ldh, beta, z.data());
  } else {
    std::vector<cd> Hc((size_t)m * m);
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < m; ++i) Hc[(size_t)j * m + i] = (i <= j + 1) ? H.get(i, j) : cd(0.0);
    st = hess_invsqrt_e1(m, Hc.data(), m, beta, z.data());
  }
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
  const Layout L = make_layout(op, m_max, flags);
  if (!ws || ws_bytes < L.bytes || ((uintptr_t)ws & 255)) return FA_ERR_WORKSPACE;
  OpScratchScope csr(op, L.scr_bytes ? at(ws, L.off_scr) : nullptr, s);
  if (!csr.ok()) return FA_ERR_HIP;
  const size_t es = elem_size(op.dtype);
  const int64_t n = op.n;
  const bool lanczos = (op.flags & FA_HERMITIAN) && !(flags & FA_FORCE_ARNOLDI);
  const Poly& q = op.poly;
  const int K = (q.method < 0) ? 0 : q.degree;
  const int k_chk = check_every > 0 ? check_every : std::max(1, 64 / (K + 1));
  const bool two_pass = (flags & FA_TWO_PASS) != 0;
  // Algorithm 2 (right preconditioning); with q == 1 it is Algorithm 1
  const bool right = (flags & FA_RIGHT_PREC) && K > 0;
  // two-pass with Algorithm 2: fixed m only (its stopping estimate needs the
  // stored y_j, which the two-pass form does not keep)
  if (two_pass && (!lanczos || (right && tol > 0.0))) return FA_ERR_UNSUPPORTED;
  // Arnoldi: CGS2 with the reorthogonalization delayed by one step (one sweep
  // of projections and one of updates per step), unless FA_CGS2 asks for the
  // two classical passes in each step; the right-preconditioned variant keeps
  // CGS2 (its stored y_j would need the same delayed correction)
  const bool dcgs2 = !lanczos && !right && !(flags & FA_CGS2);
  void* const dcoef = at(ws, L.off_dc);

  char* V = at(ws, L.off_V);
  char* Y = right ? at(ws, L.off_Y) : nullptr;
  void* U = at(ws, L.off_U);
  void* const tmp[4] = {at(ws, L.off_P), at(ws, L.off_Q), at(ws, L.off_R), at(ws, L.off_S)};
  const int fuse = (flags & FA_NO_FUSION) ? 1 : (flags & FA_FUSE2) ? 2 : (flags & FA_FUSE3) ? 3 : 4;
  void* const wls = L.off_W ? at(ws, L.off_W) : nullptr;  // least-squares q
  // mixed precision: the polynomial chain in FP32 (stencil, Chebyshev q, K >= 1)
  const bool mixed = (flags & FA_MIXED) && K > 0;
  if (mixed && (op.kind != OP_STENCIL7 || q.method != FA_POLY_CHEB || right))
    return FA_ERR_UNSUPPORTED;
  const Prec pm = mixed ? P32 : P64;
  void* part = at(ws, L.off_part);
  char* hcur = at(ws, L.off_h);
  char* Hd = at(ws, L.off_H);
  double* nrm = (double*)at(ws, L.off_nrm);
  void* zd = at(ws, L.off_z);
  auto Vc = [&](int j) -> char* { return V + (size_t)(two_pass ? j % 3 : j) * L.ldv * es; };
  auto Yc = [&](int j) -> char* { return Y + (size_t)(two_pass ? 0 : j) * L.ldv * es; };
  auto Hcol = [&](int j) -> char* { return Hd + (size_t)j * L.ldh * es; };
  // entry H(i, j) (Lanczos: i in {j, j + 1})
  auto Hent = [&](int i, int j) -> char* {
    return Hcol(j) + (size_t)(L.band ? i - j : i) * es;
  };

  Prof prof;
  prof.on = (flags & FA_PROFILE) != 0;
  Prof* pp = prof.on ? &prof : nullptr;
  int64_t mvms = 0;
  int st = FA_OK;

  // Sec. 4: square root through the inverse square root, b' = A b
  // (two-pass: b' is kept in the output vector, which pass 1 does not touch
  // and which never aliases b)
  const void* bsrc = d_b;
  if (kind == FA_SQRT) {
    void* dst = two_pass ? d_x : U;
    st = chain(op, d_b, nullptr, nullptr, dst, ChainCoef{1.0, 0.0, 0.0, 0.0}, s, pp);
    if (st) return st;
    ++mvms;
    bsrc = dst;
  }
  // the first basis vector: Algorithm 1 c = q(A) b', v_1 = c / ||c||;
  // Algorithm 2 v_1 = b' / ||b'||
  auto start_vector = [&]() -> int {
    const void* res = nullptr;
    if (right) {
      res = bsrc;
    } else if (mixed) {  // b' to FP32 in the fifth scratch vector, then the FP32 chain
      void* b32 = tmp[3];
      FA_HIP(launch_to_f32(n, (const double*)bsrc, (float*)b32, s));
      void* const tmpm[4] = {tmp[0], tmp[1], tmp[2], U};
      const int r = poly_apply(op, q, b32, Vc(0), tmpm, &res, s, pp, &mvms, fuse, P32, P64);
      if (r) return r;
    } else {
      const int r = poly_apply(op, q, bsrc, Vc(0), tmp, &res, s, pp, &mvms, fuse, P64, P64, wls);
      if (r) return r;
    }
    if (res != Vc(0)) FA_HIP(launch_scale(op.dtype, n, cd(1.0), res, Vc(0), s));
    FA_HIP(launch_update(op.dtype, n, 0, V, L.ldv, hcur, Vc(0), part, nrm, s));
    FA_HIP(launch_normalize(op.dtype, n, Vc(0), nrm, Vc(0), nullptr, s));
    return FA_OK;
  };
  // one Krylov step: w = A q(A)^2 v_j in three stages, orthogonalized against
  // the basis (CGS2) or the two latest vectors (Lanczos), normalized into v_{j+1}.
  // phase 0: the whole step; phase 1: only u = A v_j and y = q(A) u
  // (Algorithm 1, K >= 1), y kept in half_y; phase 2: the rest of a step
  // begun by phase 1.  Delayed CGS2, j >= 1: phases 3 and 4 are phases 0
  // and 2 without the update of the basis (H's column j - 1 is final after
  // them), phase 5 is that update alone.
  int64_t ips = 0;
  const void* half_y = nullptr;
  auto step = [&](int j, int phase) -> int {
    char* vj = Vc(j);
    char* w = Vc(j + 1);
    if (phase == 5) {
      FA_HIP(launch_dcgs2(op.dtype, n, j, V, L.ldv, part, hcur, Hd, L.ldh, dcoef, s,
                          kDcgs2Update));
      return FA_OK;
    }
    const bool cont = phase == 2 || phase == 4;  // continues a step begun by phase 1
    const bool no_update = phase == 3 || phase == 4;
    if (K == 0) {
      const int r = chain(op, vj, nullptr, nullptr, w, ChainCoef{1.0, 0.0, 0.0, 0.0}, s, pp);
      if (r) return r;
      ++mvms;
    } else if (right) {  // Algorithm 2: y_j = q(A) v_j (stored), u = q(A) y_j, w = A u
      const void* y = nullptr;
      int r = poly_apply(op, q, vj, Yc(j), tmp, &y, s, pp, &mvms, fuse, P64, P64, wls);
      if (r) return r;
      if (y != Yc(j)) FA_HIP(launch_scale(op.dtype, n, cd(1.0), y, Yc(j), s));
      const void* u = nullptr;
      r = poly_apply(op, q, Yc(j), U, tmp, &u, s, pp, &mvms, fuse, P64, P64, wls);
      if (r) return r;
      r = chain(op, u, nullptr, nullptr, w, ChainCoef{1.0, 0.0, 0.0, 0.0}, s, pp);
      if (r) return r;
      ++mvms;
    } else {  // Algorithm 1: u = A v_j, y = q(A) u, w = q(A) y
      const void* y = half_y;
      if (!cont) {
        FA_HIP(launch_chain(op, vj, nullptr, nullptr, U, ChainCoef{1.0, 0.0, 0.0, 0.0}, s, P64,
                            pm));
        ++mvms;
        const int r = poly_apply(op, q, U, U, tmp, &y, s, pp, &mvms, fuse, pm, pm, wls);
        if (r) return r;
        if (phase == 1) {
          half_y = y;
          return FA_OK;
        }
      }
      int r = FA_OK;
      void* tmp2[4];  // the scratch vectors other than the one holding y
      {
        void* all[5] = {U, tmp[0], tmp[1], tmp[2], tmp[3]};
        int c = 0;
        for (void* b : all)
          if (b != y && c < 4) tmp2[c++] = b;
      }
      const void* r2 = nullptr;
      r = poly_apply(op, q, y, w, tmp2, &r2, s, pp, &mvms, fuse, pm, P64, wls);
      if (r) return r;
      if (r2 != w) FA_HIP(launch_scale(op.dtype, n, cd(1.0), r2, w, s));
    }
    // orthogonalization against v_1..v_j (h_ij = v_i^H w)
    if (dcgs2) {
      // column j + 1 stays unnormalized (u_{j+1}); step j also finishes q_j
      if (j == 0) {
        FA_HIP(launch_project(op.dtype, n, 1, V, L.ldv, w, part, hcur, Hcol(0), 1, s));
        FA_HIP(launch_update(op.dtype, n, 1, V, L.ldv, hcur, w, part, nullptr, s));
        ips += 1;
      } else {
        FA_HIP(launch_dcgs2(op.dtype, n, j, V, L.ldv, part, hcur, Hd, L.ldh, dcoef, s,
                            no_update ? kDcgs2Project : kDcgs2All));
        ips += 2 * (j + 1);
      }
      return FA_OK;
    }
    if (lanczos) {
      if (j > 0)  // w -= beta_{j-1} v_{j-1}, beta_{j-1} = H(j, j-1)
        FA_HIP(launch_update(op.dtype, n, 1, Vc(j - 1), L.ldv, Hent(j, j - 1), w, part, nullptr,
                             s));
      FA_HIP(launch_project(op.dtype, n, 1, vj, L.ldv, w, part, hcur, Hent(j, j), 1, s));
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
    FA_HIP(launch_normalize(op.dtype, n, w, nrm, w, Hent(j + 1, j), s));
    return FA_OK;
  };
  // host side of the small copies: page-locked when available (see
  // PinnedPool), else ordinary memory (the copies then block, same results)
  const size_t ed = es / 8;  // doubles per element
  const size_t n_h = (size_t)L.ldh * m_max * ed, n_sh = (size_t)(m_max + 2) * ed,
               n_z = (size_t)m_max * ed, n_sc = 4;
  const size_t n_pin = n_h + n_sh + 2 * n_z + n_sc;
  // kApplyNoAlloc: no page-locked area (it may have to be allocated)
  PinnedLease lease((flags & kApplyNoAlloc) ? 0 : n_pin * sizeof(double));
  std::vector<double> pageable(lease.p ? 0 : n_pin);
  double* const pin = lease.p ? (double*)lease.p : pageable.data();
  double* const h_host = pin;              // H, column-major with ldh rows
  double* const sh_host = pin + n_h;       // a projection of u_{j+1}
  double* const z_host = sh_host + n_sh;   // two coefficient vectors
  double* const sc_host = z_host + 2 * n_z;  // scalars
  // With page-locked memory, a check's data reaches the host through one
  // kernel that writes it there and then raises a flag (sc_host[3]) which the
  // host watches: no copy commands, no event, no wait for the stream.
  double* pin_dev = nullptr;  // the lease as the device addresses it
  if (lease.p) {
    void* dp = nullptr;
    if (hipHostGetDevicePointer(&dp, lease.p, 0) == hipSuccess) pin_dev = (double*)dp;
  }
  auto dev_of = [&](double* hp) { return pin_dev + (hp - pin); };
  int* const flag_host = reinterpret_cast<int*>(sc_host + 3);
  int chk_seq = 0;  // the value the next check raises the flag to (unique in the process,
                    // so a late write by an earlier user of this area never matches)
  auto next_seq = [] {
    static std::atomic<int> counter{0};
    return (counter.fetch_add(1) & 0x3fffffff) + 1;
  };
  // wait until the device has raised the flag to `seq` (the stream is
  // synchronized instead if that takes implausibly long)
  auto wait_flag = [&](int seq) -> int {
    const double t0 = now_ms();
    while (__atomic_load_n(flag_host, __ATOMIC_ACQUIRE) != seq) {
#if defined(__x86_64__)
      __builtin_ia32_pause();
#endif
      if (now_ms() - t0 > 2000.0) {
        FA_HIP(hipStreamSynchronize(s));
        return __atomic_load_n(flag_host, __ATOMIC_ACQUIRE) == seq ? FA_OK : FA_ERR_HIP;
      }
    }
    return FA_OK;
  };
  // coefficient vector z to the device (negated with `neg`) from host slot
  // `slot` (0 or 1); the slot must not be rewritten before the stream has
  // passed this copy (every caller synchronizes before the next use)
  auto z_to_device = [&](const std::vector<cd>& zz, int len, bool neg, void* dst,
                         int slot = 0) -> int {
    double* zh = z_host + (size_t)slot * n_z;
    const double sg = neg ? -1.0 : 1.0;
    for (int i = 0; i < len; ++i) {
      if (op.dtype == FA_C128) {
        zh[2 * i] = sg * zz[i].real();
        zh[2 * i + 1] = sg * zz[i].imag();
      } else {
        zh[i] = sg * zz[i].real();
      }
    }
    FA_HIP(hipMemcpyAsync(dst, zh, (size_t)len * ed * sizeof(double), hipMemcpyHostToDevice, s));
    if (!lease.p) FA_HIP(hipStreamSynchronize(s));
    return FA_OK;
  };

  st = start_vector();
  if (st) return st;
  const int64_t mvms_start = mvms;
  // ||c||^2 to the host.  With page-locked memory it goes through the flag
  // without a wait here: beta is first needed at the first check, whose
  // data arrive after it, so the steps are enqueued at once.  A zero or
  // nonfinite ||c|| is then handled at that check (the steps before it ran
  // on the zero vector the normalization leaves).
  bool beta_pending = false;
  if (pin_dev) {
    FA_HIP(launch_check_export(nrm, 1, dev_of(sc_host), nullptr, 0, nullptr,
                               (int*)dev_of(sc_host + 3), chk_seq = next_seq(), s));
    beta_pending = true;
  } else {
    FA_HIP(hipMemcpyAsync(sc_host, nrm, sizeof(double), hipMemcpyDeviceToHost, s));
    FA_HIP(hipStreamSynchronize(s));
  }
  double beta = 0.0;
  // beta from the host copy of ||c||^2; `done`: b' = 0 gave x = 0 (returned)
  auto take_beta = [&](bool& done) -> int {
    const double beta2 = sc_host[0];
    if (!std::isfinite(beta2)) return FA_ERR_NONFINITE;
    beta = std::sqrt(beta2);
    done = beta == 0.0;
    if (done) {
      FA_HIP(launch_scale(op.dtype, n, cd(0.0), Vc(0), d_x, s));
      FA_HIP(hipStreamSynchronize(s));
      S.converged = 1;
      S.mvms = mvms_start;
      S.ms_total = now_ms() - t0;
      if (stats) *stats = S;
    }
    return FA_OK;
  };
  if (!beta_pending) {
    bool done = false;
    st = take_beta(done);
    if (st || done) return st;
  }

  HostH H;
  H.ldh = L.ldh;
  H.band = L.band;
  H.dtype = op.dtype;
  H.buf = h_host;
  std::memset(h_host, 0, n_h * sizeof(double));
  int copied = 0;          // columns of H final on the host
  int refresh = 0;         // first column to copy again at the next check
  double colmax = 0.0;     // largest column norm of H seen (breakdown scale)
  std::vector<cd> z, zprev;
  int m = m_max;
  bool converged = false, breakdown = false;
  double est = 1.0;

  // When the host evaluation of H_j^{-1/2} e_1 at a check is expected to take
  // longer than a step, the next steps (as many as that time covers, fewer
  // than k) are enqueued before it, so the GPU works while the host does; if
  // the iteration stops at the check, their output is not used and their
  // counts are undone.  The host time is predicted from the previous check
  // (cubic in the order of H), the step time from the wall time between
  // checks.
  int ahead_until = 0;        // steps below this index are already enqueued
  double last_host_ms = 0.0;  // host time of the previous check's H^{-1/2} e_1
  int last_host_m = 0;
  double t_resume = now_ms();
  int j_resume = 0;
  // At a check the first half of the next step (u = A v_j, y = q(A) u) is
  // enqueued behind the copies before the host waits for them, so the GPU
  // works through the check's round trip (copies, host f(H), the next
  // launches); it is left out when the last two estimates, extrapolated
  // geometrically, predict convergence at this check.  If the iteration
  // stops there, its output is never read and its counts are undone.
  // (the half step's wait needs an event without page-locked memory, and
  // kApplyNoAlloc creates none)
  // Small Hermitian problems: the steps up to the next check in one launch
  // of one workgroup (kernels_small.hip; FA_NO_FUSION keeps one launch per
  // recurrence term)
  const bool small = lanczos && !right && !two_pass && !mixed && !(flags & FA_NO_FUSION) &&
                     small_lanczos_ok(op, q);
  std::vector<SmallTerm> small_terms;
  if (small && K > 0)
    for (const Term& t : poly_terms(q))
      small_terms.push_back(SmallTerm{t.k.alpha.real(), t.k.beta.real(), t.k.g0.real(),
                                      t.k.g1.real(), t.y0 ? 1 : 0, t.y1 ? 1 : 0});
  int small_until = 0;  // steps below this index are enqueued in a launch already
  const bool can_half =
      K > 0 && !right && !two_pass && tol > 0.0 && !(flags & kApplyNoAlloc) && !small;
  int half_j = -1;  // the step whose first half is enqueued
  // Delayed CGS2: at a check the iteration is expected to pass, the next
  // step is enqueued up to its projection before the check's data goes to
  // the host.  That projection finishes column j of H on the device (its
  // second pass), so no projection of u_{j+1} for the check is needed; the
  // step's update and the first half of the step after it follow, so the
  // GPU works through the check's round trip.  If the iteration stops there
  // after all, their output is never read and their counts are undone.
  const bool can_defer = dcgs2 && !two_pass && tol > 0.0 && !(flags & kApplyNoAlloc) && !small;
  int64_t pend_mvms = 0;  // counts and timings before the first half of a step
  Prof pend_prof = prof;  // that such a check enqueued (still pending at the next check)
  std::vector<double> est_hist;
  auto run_step = [&](int j) -> int {
    if (small) {
      if (j < small_until) return FA_OK;
      // to the next check (tol <= 0: to m_max)
      const int end = tol > 0.0 ? std::min(m_max, (j / k_chk + 1) * k_chk) : m_max;
      FA_HIP(launch_small_lanczos(op, small_terms, j, end, V, L.ldv, Hd, s));
      mvms += (int64_t)(end - j) * (2 * K + 1);
      ips += 2 * (int64_t)(end - j);
      small_until = end;
      return FA_OK;
    }
    if (half_j == j) {
      half_j = -1;
      return step(j, 2);
    }
    return step(j, 0);
  };
  for (int j = 0; j < m_max; ++j) {
    if (j >= ahead_until) {
      st = run_step(j);
      if (st) return st;
    }
    const int jj = j + 1;
    const bool check = (tol > 0.0) ? (jj % k_chk == 0 || jj == m_max) : (jj == m_max);
    if (!check) continue;
    // the new columns of H to the host
    const int from = std::min(copied, refresh);
    double* const h_dst = H.buf + (size_t)from * L.ldh * ed;
    const int64_t h_len = (int64_t)(jj - from) * L.ldh * ed;  // doubles
    bool predict_more = true;
    if (est_hist.size() >= 2 && est_hist[est_hist.size() - 2] > 0.0) {
      const double a = est_hist[est_hist.size() - 2], b = est_hist.back();
      predict_more = b * (b / a) > 10.0 * tol;
    }
    // counts and timings of the iteration so far, without the work enqueued
    // ahead (a first half of step jj from the previous check, or what this
    // check enqueues)
    const bool pend = half_j == jj;
    const int64_t mvms_base = pend ? mvms - pend_mvms : mvms, ips_base = ips;
    const Prof prof_base = pend ? pend_prof : prof;
    // (the first check cannot stop the iteration: its estimate is 1; the
    // second has no extrapolation, and a step thrown away costs far more
    // than the projection saved when the polynomial is long)
    const bool defer = can_defer && jj < m_max && jj >= ahead_until &&
                       ((est_hist.empty() && tol < 1.0) || (est_hist.size() >= 2 && predict_more));
    if (defer) {  // step jj up to its projection: column j of H final on the device
      st = step(jj, half_j == jj ? 4 : 3);
      if (st) return st;
      half_j = -1;
    }
    // without it, column j still lacks its second pass (done on the device in
    // the next step): project u_{j+1} on [q_0 .. q_j, u_{j+1}] and finish the
    // host copy: H(0:j, j) += s', H(j+1, j) = (||u_{j+1}||^2 - ||s'||^2)^{1/2}
    const bool fin_host = dcgs2 && !defer;
    if (fin_host)
      FA_HIP(launch_project(op.dtype, n, jj + 1, V, L.ldv, Vc(jj), part, hcur, nullptr, 0, s));
    const int64_t p_len = fin_host ? (int64_t)(jj + 1) * ed : 0;
    if (pin_dev) {
      FA_HIP(launch_check_export((const double*)Hcol(from), h_len, dev_of(h_dst),
                                 (const double*)hcur, p_len, dev_of(sh_host),
                                 (int*)dev_of(sc_host + 3), chk_seq = next_seq(), s));
    } else {
      FA_HIP(hipMemcpyAsync(h_dst, Hcol(from), (size_t)h_len * sizeof(double),
                            hipMemcpyDeviceToHost, s));
      if (p_len)
        FA_HIP(hipMemcpyAsync(sh_host, hcur, (size_t)p_len * sizeof(double),
                              hipMemcpyDeviceToHost, s));
    }
    if (defer) {
      // the rest of step jj and the first half of step jj + 1 (if any)
      st = step(jj, 5);
      if (st) return st;
      ahead_until = jj + 1;
      if (can_half && jj + 1 < m_max) {
        const int64_t m0 = mvms;
        const Prof p0 = prof;
        st = step(jj + 1, 1);
        if (st) return st;
        pend_mvms = mvms - m0;
        pend_prof = p0;
        half_j = jj + 1;
      }
      if (pin_dev) {
        st = wait_flag(chk_seq);
        if (st) return st;
      } else {
        FA_HIP(hipStreamSynchronize(s));
      }
    } else if (can_half && jj < m_max && predict_more && !pend) {  // (pend: enqueued already)
      hipEvent_t ev = nullptr;
      if (!pin_dev) {
        FA_HIP(check_event(&ev));
        FA_HIP(hipEventRecord(ev, s));
      }
      st = step(jj, 1);
      if (st) return st;
      half_j = jj;
      if (pin_dev) {
        st = wait_flag(chk_seq);
        if (st) return st;
      } else {
        FA_HIP(hipEventSynchronize(ev));
      }
    } else if (pin_dev) {
      st = wait_flag(chk_seq);
      if (st) return st;
    } else {
      FA_HIP(hipStreamSynchronize(s));
    }
    if (beta_pending) {  // ||c||^2 arrived with this check's data
      beta_pending = false;
      bool done = false;
      st = take_beta(done);
      if (st || done) return st;
    }
    // takes the counts and timings of what was enqueued ahead back out (the
    // iteration stops here); the second pass of column j counts as the
    // check's projection would
    auto undo_half = [&]() {
      mvms = mvms_base;
      if (defer) ips = ips_base + jj + 1;
      prof = prof_base;
      half_j = -1;
    };
    if (fin_host) {
      const double* sh = sh_host;
      auto sv = [&](int i) {
        return op.dtype == FA_C128 ? cd(sh[2 * i], sh[2 * i + 1]) : cd(sh[i], 0.0);
      };
      double ss = 0.0;
      for (int i = 0; i <= j; ++i) {
        H.set(i, j, H.get(i, j) + sv(i));
        ss += std::norm(sv(i));
      }
      const double nu2 = sv(jj).real() - ss;
      H.set(jj, j, cd(nu2 > 0.0 ? std::sqrt(nu2) : 0.0, 0.0));
      ips += jj + 1;
    }
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
    refresh = fin_host ? j : jj;
    if (mb > 0) {
      undo_half();
      m = mb;
      breakdown = converged = true;
      break;
    }
    if (tol <= 0.0) break;
    const int64_t mvms_here = mvms_base, ips_here = defer ? ips_base + jj + 1 : ips;
    const Prof prof_here = prof_base;
    {
      const double step_ms = (now_ms() - t_resume) / std::max(1, jj - j_resume);
      const double ratio = last_host_m > 0 ? (double)jj / last_host_m : 0.0;
      const double host_est = last_host_ms * ratio * ratio * ratio;
      int r = step_ms > 0.0 ? (int)(host_est / step_ms) : 0;
      r = std::min(r, std::min(k_chk - 1, m_max - jj));
      for (int a = std::max(jj, ahead_until); a < jj + r; ++a) {
        st = run_step(a);
        if (st) return st;
      }
      ahead_until = std::max(ahead_until, jj + std::max(r, 0));
    }
    const double th = now_ms();
    st = host_coeffs(H, jj, lanczos, beta, z);
    last_host_ms = now_ms() - th;
    last_host_m = jj;
    S.ms_host_fH += last_host_ms;
    ++S.checks;
    if (st) return st;
    if (right) {
      // Y is not orthonormal: est = ||Y_j (z_j - [z_{j-k}; 0])|| / ||Y_j z_j||
      std::vector<cd> dz(jj);
      for (int i = 0; i < jj; ++i) dz[i] = z[i] - ((i < (int)zprev.size()) ? zprev[i] : cd(0.0));
      st = z_to_device(dz, jj, false, zd);
      if (st) return st;
      FA_HIP(launch_combine(op.dtype, n, jj, Y, L.ldv, zd, tmp[0], s));
      FA_HIP(launch_update(op.dtype, n, 0, V, L.ldv, hcur, tmp[0], part, nrm, s));
      FA_HIP(hipMemcpyAsync(sc_host + 1, nrm, sizeof(double), hipMemcpyDeviceToHost, s));
      st = z_to_device(z, jj, false, zd, 1);
      if (st) return st;
      FA_HIP(launch_combine(op.dtype, n, jj, Y, L.ldv, zd, tmp[0], s));
      FA_HIP(launch_update(op.dtype, n, 0, V, L.ldv, hcur, tmp[0], part, nrm, s));
      FA_HIP(hipMemcpyAsync(sc_host + 2, nrm, sizeof(double), hipMemcpyDeviceToHost, s));
      FA_HIP(hipStreamSynchronize(s));
      est = std::sqrt(sc_host[1] / sc_host[2]);
    } else {  // V orthonormal: the iterates' difference from the coefficients
      double dn = 0.0, zn = 0.0;
      for (int i = 0; i < jj; ++i) {
        const cd zp = (i < (int)zprev.size()) ? zprev[i] : cd(0.0);
        dn += std::norm(z[i] - zp);
        zn += std::norm(z[i]);
      }
      est = std::sqrt(dn / zn);
    }
    zprev = z;
    est_hist.push_back(est);
    if (est <= tol) {
      m = jj;
      converged = true;
      mvms = mvms_here;  // steps enqueued ahead are not part of the result
      ips = ips_here;
      prof = prof_here;
      half_j = -1;
      break;
    }
    t_resume = now_ms();
    j_resume = std::max(jj, ahead_until);
  }
  if (beta_pending) {  // (no check ran)
    FA_HIP(hipStreamSynchronize(s));
    beta_pending = false;
    bool done = false;
    st = take_beta(done);
    if (st || done) return st;
  }
  // final coefficients (if the loop did not end on a fresh check of size m)
  if ((int)z.size() != m || breakdown) {
    if (copied < m) {
      FA_HIP(hipMemcpyAsync(H.buf + (size_t)copied * L.ldh * (es / 8), Hcol(copied),
                            (size_t)(m - copied) * L.ldh * es, hipMemcpyDeviceToHost, s));
      FA_HIP(hipStreamSynchronize(s));
    }
    const double th = now_ms();
    st = host_coeffs(H, m, lanczos, beta, z);
    S.ms_host_fH += now_ms() - th;
    if (st) return st;
  }
  if (two_pass) {
    // second pass: regenerate v_1..v_m with the same (deterministic) kernels
    // and accumulate x = sum_i z_i v_i, the basis never stored; Algorithm 2's
    // Y_m z_m = q(A) (V_m z_m) takes one more q(A) at the end
    st = z_to_device(z, m, true, zd);
    if (st) return st;
    st = start_vector();
    if (st) return st;
    FA_HIP(launch_scale(op.dtype, n, z[0], Vc(0), d_x, s));
    for (int j = 0; j + 1 < m; ++j) {
      st = step(j, 0);
      if (st) return st;
      FA_HIP(launch_update(op.dtype, n, 1, Vc(j + 1), L.ldv, (char*)zd + (size_t)(j + 1) * es,
                           d_x, part, nullptr, s));
    }
    if (right) {
      const void* r = nullptr;
      st = poly_apply(op, q, d_x, U, tmp, &r, s, pp, &mvms, fuse, P64, P64, wls);
      if (st) return st;
      if (r != d_x) FA_HIP(launch_scale(op.dtype, n, cd(1.0), r, d_x, s));
    }
  } else {
    // f_m = V_m z_m (Algorithm 1) or Y_m z_m (Algorithm 2)
    st = z_to_device(z, m, false, zd);
    if (st) return st;
    FA_HIP(launch_combine(op.dtype, n, m, right ? (const void*)Y : (const void*)V, L.ldv, zd, d_x,
                          s));
  }
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
    S.n_chain_terms = prof.terms;
  }
  if (stats) *stats = S;
  return converged ? FA_OK : FA_WARN_NOT_CONVERGED;
}

// --------------------------------------------------------------------------
// polynomial setup
// --------------------------------------------------------------------------
// Regroup the scaled Newton form of a real operator's Ritz polynomial into
// real blocks.  q(z) = sum_j eta_j w_j(z), w_j = prod_{i<j} (z - theta_i)/rho,
// with conjugate pairs adjacent.  At a block start the nodes before it form a
// conjugate-closed set, so w_j has real coefficients; q itself is real, so q
// equals the sum of w_{start(B)} times the real parts of the coefficients of
// each block's linear factor l_B(z) = eta_s + eta_{s+1} (z - theta_s)/rho
// (pair) or eta_s (real node).
static int real_blocks(Poly& q) {
  const std::vector<cd>& th = q.theta;
  const std::vector<cd>& eta = q.eta;
  const double rho = q.rho;
  q.blocks.clear();
  for (size_t j = 0; j < th.size();) {
    if (th[j].imag() == 0.0) {
      q.blocks.push_back({false, th[j].real(), 0.0, eta[j].real(), 0.0});
      j += 1;
      continue;
    }
    if (j + 1 >= th.size() || std::abs(th[j + 1] - std::conj(th[j])) > 1e-10 * std::abs(th[j]))
      return FA_ERR_UNSUPPORTED;  // a non-real node without its conjugate next to it
    // the evaluation divides by Re theta (see poly_apply): refuse nodes that
    // are nearly imaginary
    if (th[j].real() < 1e-3 * std::abs(th[j])) return FA_ERR_UNSUPPORTED;
    const cd e0 = eta[j], e1 = eta[j + 1];
    q.blocks.push_back({true, th[j].real(), std::fabs(th[j].imag()),
                        (e0 - e1 * th[j] / rho).real(), (e1 / rho).real()});
    j += 2;
  }
  return FA_OK;
}

size_t poly_workspace_bytes(const Op& op, int degree, int method) {
  if (method == FA_POLY_CHEB || degree == 0) return 0;
  // RITZ and HARMONIC: degree + 1 setup Arnoldi steps; LS: the default number
  const int steps = (method == FA_POLY_LS) ? LsParams().ritz_steps : degree + 1;
  return make_layout(op, steps, FA_FORCE_ARNOLDI, false).bytes;
}

namespace {
// `steps` Arnoldi steps on A (CGS2) from d_start; the eigenvalues of H (Ritz
// values) or of H + h^2 H^{-H} e e^T (harmonic Ritz values), fewer after a
// lucky breakdown.  Real operators: conjugate pairs made exact, real values
// made real.
int setup_ritz_values(const Op& op, int steps, bool harmonic, const void* d_start, void* ws,
                      size_t ws_bytes, hipStream_t s, int64_t* mvms_setup, std::vector<cd>& ev) {
  if (!d_start) return FA_ERR_ARG;
  const int d = steps;
  const Layout L = make_layout(op, d, FA_FORCE_ARNOLDI, false);
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
  OpScratchScope scr(op, L.scr_bytes ? at(ws, L.off_scr) : nullptr, s);
  if (!scr.ok()) return FA_ERR_HIP;
  FA_HIP(launch_update(op.dtype, n, 0, V, L.ldv, hcur, (void*)d_start, part, nrm, s));
  FA_HIP(launch_normalize(op.dtype, n, d_start, nrm, Vc(0), nullptr, s));
  for (int j = 0; j < d; ++j) {
    char* w = Vc(j + 1);
    int st = chain(op, Vc(j), nullptr, nullptr, w, ChainCoef{1.0, 0.0, 0.0, 0.0}, s, nullptr);
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
  H.own.assign((size_t)L.ldh * d * (es / 8), 0.0);
  H.buf = H.own.data();
  FA_HIP(hipMemcpyAsync(H.buf, Hd, (size_t)L.ldh * d * es, hipMemcpyDeviceToHost, s));
  FA_HIP(hipStreamSynchronize(s));
  // steps completed before a lucky breakdown (same rule as in fa_apply)
  int m = d;
  double colmax = 0.0;
  for (int c = 0; c < d; ++c) {
    double cn = 0.0;
    for (int i = 0; i <= c + 1; ++i) cn += std::norm(H.get(i, c));
    if (!std::isfinite(cn)) return FA_ERR_NONFINITE;
    colmax = std::max(colmax, std::sqrt(cn));
    if (std::abs(H.get(c + 1, c)) <= 1e-12 * colmax) {
      m = c + 1;
      break;
    }
  }
  std::vector<cd> Hc((size_t)m * m);
  ev.assign(m, cd(0.0));
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < m; ++i) Hc[(size_t)j * m + i] = (i <= j + 1) ? H.get(i, j) : cd(0.0);
  if (harmonic) {
    // harmonic Ritz values: eigenvalues of H_m + h_{m+1,m}^2 f e_m^T with
    // H_m^H f = e_m (Sec. 5.2); after a lucky breakdown h_{m+1,m} = 0
    const double hn = std::abs(H.get(m, m - 1));
    std::vector<cd> A((size_t)m * m), f(m, cd(0.0));
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < m; ++i) A[(size_t)j * m + i] = std::conj(Hc[(size_t)i * m + j]);
    f[m - 1] = 1.0;
    if (lu_solve(m, A.data(), f.data()) != DENSE_OK) return FA_ERR_HESSENBERG;
    for (int i = 0; i < m; ++i) Hc[(size_t)(m - 1) * m + i] += hn * hn * f[i];
  }
  if (hess_eigenvalues(m, Hc.data(), m, ev.data()) != DENSE_OK) return FA_ERR_HESSENBERG;
  for (auto& t : ev) {
    if (!(t.real() > 0.0)) return FA_ERR_BRANCH;  // outside the right half-plane
    // eigenvalues of a real H are real or come in conjugate pairs
    if (op.dtype == FA_F64 && std::fabs(t.imag()) <= 1e-10 * std::abs(t)) t = cd(t.real(), 0.0);
  }
  return FA_OK;
}
}  // namespace

int poly_setup(Op& op, int degree, int method, const void* d_start, void* ws, size_t ws_bytes,
               hipStream_t s, int64_t* mvms_setup, const LsParams& ls) {
  if (degree < 0 || degree > 512) return FA_ERR_ARG;
  if (method == FA_POLY_AUTO) method = op.has_interval ? FA_POLY_CHEB : FA_POLY_RITZ;
  Poly q;
  *mvms_setup = 0;
  if (degree == 0) {
    q.method = -1;
    q.degree = 0;
    op.poly = q;
    op.poly_ready = true;
    ++op.poly_version;
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
    ++op.poly_version;
    return FA_OK;
  }
  const bool real_op = op.dtype == FA_F64;
  if (method == FA_POLY_LS) {
    // Sec. 5.3: Ritz values from ls.ritz_steps Arnoldi steps, the contour
    // around them, the least-squares fit of z^{-1/2} on its points
    if (degree >= kLsMax || ls.ritz_steps < 2 || !(ls.r_min >= 0.0) || !(ls.step > 0.0))
      return FA_ERR_ARG;
    std::vector<cd> ev, pts;
    int st = setup_ritz_values(op, ls.ritz_steps, false, d_start, ws, ws_bytes, s, mvms_setup, ev);
    if (st) return st;
    st = ls_contour(ev, ls.r_min, ls.step, real_op, pts);
    if (st == DENSE_BRANCH) return FA_ERR_BRANCH;
    if (st != DENSE_OK) return FA_ERR_HESSENBERG;
    if ((long)pts.size() <= degree) return FA_ERR_ARG;
    st = ls_fit_invsqrt(pts, degree, real_op, q.hls, q.alpha);
    if (st == DENSE_BRANCH) return FA_ERR_BRANCH;
    if (st != DENSE_OK) return FA_ERR_HESSENBERG;
    q.method = FA_POLY_LS;
    q.degree = degree;
    q.npts = (long)pts.size();
    op.poly = q;
    op.poly_ready = true;
    ++op.poly_version;
    return FA_OK;
  }
  if (method != FA_POLY_RITZ && method != FA_POLY_HARMONIC) return FA_ERR_ARG;
  // d = degree + 1 Arnoldi steps on A itself (CGS2) from the given start vector
  std::vector<cd> ev;
  int st = setup_ritz_values(op, degree + 1, method == FA_POLY_HARMONIC, d_start, ws, ws_bytes, s,
                             mvms_setup, ev);
  if (st) return st;
  bool any_complex = false;
  for (const auto& t : ev) any_complex |= real_op && t.imag() != 0.0;
  q.method = FA_POLY_RITZ;
  q.harmonic = method == FA_POLY_HARMONIC;
  q.theta = leja_order(ev, real_op);
  q.degree = (int)q.theta.size() - 1;
  q.rho = leja_capacity(q.theta);
  q.eta = newton_invsqrt(q.theta, q.rho);
  if (real_op && any_complex) {
    const int st2 = real_blocks(q);
    if (st2) return st2;
  }
  op.poly = q;
  op.poly_ready = true;
  ++op.poly_version;
  return FA_OK;
}

}  // namespace fa
