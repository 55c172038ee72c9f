// Block (several right-hand sides) form of Algorithm 1: s right-hand sides
// sharing the operator run as one block Arnoldi process.
//
//   B' = B (or A B for the square root, Sec. 4);  C = q(A) B' = V_1 R_0
//   for j = 1, 2, ...:
//     W = q(A) (q(A) (A V_j))                     block stencil chain
//     twice: P = [V_1..V_j]^T W, W -= [V_1..V_j] P   FP64 MFMA, H(:, j) += P
//     W = V_{j+1} H_{j+1,j}                       CholQR2 (Gram matrix on MFMA,
//                                                 Cholesky in one workgroup)
//   every k steps: Z = H_j^{-1/2} E_1 R_0 by the coupled Newton-Schulz
//   iteration on the device (dense FP64 MFMA products), per-column estimate
//   ||Z_j e_c - [Z_{j-k} e_c; 0]|| / ||Z_j e_c||; stop when all <= tol
//   X = [V_1..V_m] Z.
//
// Blocks are row-major n x s (the s values of a grid point contiguous), the
// basis FP64, for the Gram-Schmidt products.  The stencil chain of a step
// runs on the s columns as a batch of s vectors: V_j is moved to column-major
// order, A and q(A) twice run as the single-vector chain launches (up to four
// Clenshaw terms per launch, the intermediate terms on chip) over the whole
// batch, and the result is moved back into the row-major W.  With FA_MIXED
// the chain runs in FP32 storage with FP32 arithmetic; everything else stays
// FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "fa_internal.hpp"
#include "solver.hpp"

// workgroups the multi-term chain launches aim at over the batch of columns
#ifndef FA_BLK_MULTI_BLOCKS
#define FA_BLK_MULTI_BLOCKS 1536
#endif

namespace fa {

namespace {

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

constexpr int kNsplitMax = 256;  // split-K chunks of the projections

struct BlkLayout {
  int64_t bstride = 0;  // elements per basis block (n * s rounded up)
  int M = 0;            // m_max * s (the largest Hessenberg order)
  int64_t ldh = 0;      // leading dimension of H (row-major)
  size_t off_V = 0, off_C[5] = {0, 0, 0, 0, 0}, off_part = 0, off_H = 0, off_G = 0, off_R = 0,
         off_Ri = 0, off_R0 = 0, off_Rt = 0, off_P2 = 0, off_NS[4] = {0, 0, 0, 0}, off_Zc = 0,
         off_nrm = 0, off_flag = 0, off_rows = 0;
  size_t bytes = 0;
};

BlkLayout blk_layout(const Op& op, int s, int m_max, bool mixed) {
  BlkLayout L;
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off += (size_t)round_up((int64_t)b, 256);
    return o;
  };
  L.bstride = round_up(op.n * s, 32);
  L.M = m_max * s;
  L.ldh = L.M;
  const size_t ce = mixed ? 4 : 8;
  L.off_V = take((size_t)(m_max + 1) * L.bstride * 8);
  for (int i = 0; i < 5; ++i) L.off_C[i] = take((size_t)L.bstride * ce);
  L.off_part = take((size_t)kNsplitMax * (m_max + 1) * s * s * 8);
  L.off_H = take((size_t)(L.M + s) * L.ldh * 8);
  L.off_G = take((size_t)s * s * 8);
  L.off_R = take((size_t)s * s * 8);
  L.off_Ri = take((size_t)s * s * 8);
  L.off_R0 = take((size_t)s * s * 8);
  L.off_Rt = take((size_t)s * s * 8);
  L.off_P2 = take((size_t)(L.M + s) * s * 8);
  for (int i = 0; i < 4; ++i) L.off_NS[i] = take((size_t)L.M * L.M * 8);
  L.off_Zc = take((size_t)L.M * s * 8);
  L.off_nrm = take(8 * sizeof(double));
  L.off_flag = take((size_t)(m_max + 2) * sizeof(int));
  L.off_rows = take((size_t)2 * L.M * 8);
  L.bytes = off;
  return L;
}

char* at(void* ws, size_t off) { return (char*)ws + off; }

#define BLK_HIP(x)                              \
  do {                                          \
    if ((x) != hipSuccess) return FA_ERR_HIP;   \
  } while (0)

// Autotuner.  A launch parameter with several candidates is timed on the
// caller's stream the first time its problem shape occurs in the process
// (one warm-up and one timed run per candidate, HIP events); the fastest is
// kept for every later launch of that shape, and run once more so that the
// results of the current call are the chosen candidate's.  Only launches
// that may be repeated without changing their result are tuned.
struct Tuner {
  std::mutex mu;
  std::map<std::vector<int64_t>, int> best;
};
Tuner& tuner() {
  static Tuner t;
  return t;
}

template <class F>
int tune_pick(const std::vector<int64_t>& key, const std::vector<int>& cands, hipStream_t st,
              F&& run, int* chosen, double* ms_tune) {
  {
    std::lock_guard<std::mutex> g(tuner().mu);
    auto it = tuner().best.find(key);
    if (it != tuner().best.end()) {
      *chosen = it->second;
      BLK_HIP(run(*chosen));
      return FA_OK;
    }
  }
  const double t0 = now_ms();
  hipEvent_t a, b;
  BLK_HIP(hipEventCreate(&a));
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return FA_ERR_HIP;
  }
  float best_ms = 1e30f;
  int best_c = cands[0];
  int st_code = FA_OK;
  for (int c : cands) {
    float ms = 0.0f;
    if (run(c) != hipSuccess || hipEventRecord(a, st) != hipSuccess || run(c) != hipSuccess ||
        hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
        hipEventElapsedTime(&ms, a, b) != hipSuccess) {
      st_code = FA_ERR_HIP;
      break;
    }
    if (ms < best_ms) {
      best_ms = ms;
      best_c = c;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (st_code) return st_code;
  {
    std::lock_guard<std::mutex> g(tuner().mu);
    *chosen = tuner().best.emplace(key, best_c).first->second;
  }
  BLK_HIP(run(*chosen));
  *ms_tune += now_ms() - t0;
  return FA_OK;
}

bool is_tuned(const std::vector<int64_t>& key) {
  std::lock_guard<std::mutex> g(tuner().mu);
  return tuner().best.count(key) != 0;
}

// Executable graphs of block steps, keyed by everything their kernel
// arguments depend on (op identity and polynomial version, workspace address,
// block size, Krylov dimension bound, precision mode, step index, tuned
// parameters).  Freed with the op (release_op_graphs) or at process end.
struct GraphCache {
  std::mutex mu;
  std::map<std::vector<int64_t>, hipGraphExec_t> execs;
};
GraphCache& graphs() {
  static GraphCache c;
  return c;
}

}  // namespace

void release_op_graphs(uint64_t uid) {
  std::lock_guard<std::mutex> g(graphs().mu);
  for (auto it = graphs().execs.begin(); it != graphs().execs.end();) {
    if ((uint64_t)it->first[0] == uid) {
      (void)hipGraphExecDestroy(it->second);
      it = graphs().execs.erase(it);
    } else {
      ++it;
    }
  }
}

size_t block_workspace_bytes(const Op& op, int s, int m_max, uint32_t flags) {
  return blk_layout(op, s, m_max, (flags & FA_MIXED) != 0).bytes;
}

int block_apply(const Op& op, int kind, int s, const void* d_B, void* d_X, int m_max, double tol,
                int check_every, void* ws, size_t ws_bytes, uint32_t flags, hipStream_t st,
                fa_block_stats* stats) {
  const double t0 = now_ms();
  fa_block_stats S;
  std::memset(&S, 0, sizeof(S));
  if (op.kind != OP_STENCIL7 || op.dtype != FA_F64) return FA_ERR_UNSUPPORTED;
  const Poly& q = op.poly;
  const int K = (q.method < 0) ? 0 : q.degree;
  if (K > 0 && q.method != FA_POLY_CHEB) return FA_ERR_UNSUPPORTED;
  const bool mixed = (flags & FA_MIXED) && K > 0;
  const BlkLayout L = blk_layout(op, s, m_max, (flags & FA_MIXED) != 0);
  if (!ws || ws_bytes < L.bytes || ((uintptr_t)ws & 255)) return FA_ERR_WORKSPACE;
  if ((flags & FA_GRAPH) && !st) return FA_ERR_ARG;  // the null stream cannot be captured
  const int k_chk = check_every > 0 ? check_every : std::max(1, 64 / (K + 1));
  const Prec pc = mixed ? P32 : P64;
  const int64_t n = op.n;

  double* V = (double*)at(ws, L.off_V);
  auto Vb = [&](int j) { return V + (size_t)j * L.bstride; };
  void* C[5];
  for (int i = 0; i < 5; ++i) C[i] = at(ws, L.off_C[i]);
  double* part = (double*)at(ws, L.off_part);
  double* H = (double*)at(ws, L.off_H);
  double* G = (double*)at(ws, L.off_G);
  double* R = (double*)at(ws, L.off_R);
  double* Ri = (double*)at(ws, L.off_Ri);
  double* R0 = (double*)at(ws, L.off_R0);
  double* Rt = (double*)at(ws, L.off_Rt);
  double* P2 = (double*)at(ws, L.off_P2);
  double* NS[4];
  for (int i = 0; i < 4; ++i) NS[i] = (double*)at(ws, L.off_NS[i]);
  double* Zc = (double*)at(ws, L.off_Zc);
  double* nrm = (double*)at(ws, L.off_nrm);
  int* flag = (int*)at(ws, L.off_flag);
  double* rowsc = (double*)at(ws, L.off_rows);
  int64_t mvms = 0;

  // H and the per-step flags start at zero (the projections add into H)
  BLK_HIP(hipMemsetAsync(H, 0, (size_t)(L.M + s) * L.ldh * 8, st));
  BLK_HIP(hipMemsetAsync(flag, 0, (size_t)(m_max + 2) * sizeof(int), st));

  // z-planes per workgroup of the row-major block stencil launches (A B for
  // the square root, A V_j without a polynomial)
  const int zc = 8;
  hipStream_t cur = st;  // the stream the step launches go to (captured with FA_GRAPH)
  // the op as a batch of s column vectors of n (the chain scratch blocks hold
  // s * n values of the chain precision)
  Op opb = op;
  opb.nbatch = s;
  opb.bstride = n;
  opb.multi_blocks = FA_BLK_MULTI_BLOCKS;
  // q(A) on the batch in column-major x (chain precision; x is overwritten):
  // the result is x or one of tmp
  auto qcols = [&](void* x, void* const tmp[4], void** res) -> int {
    const void* r = nullptr;
    int64_t mv = 0;
    const int e = poly_apply_chain(opb, x, x, tmp, &r, cur, &mv, pc);
    if (e) return e;
    mvms += mv * s;
    *res = const_cast<void*>(r);
    return FA_OK;
  };
  // the four of C[0..4] that are not `y`
  auto others = [&](const void* y, void* (&t)[4]) {
    int c = 0;
    for (int i = 0; i < 5; ++i)
      if (C[i] != y && c < 4) t[c++] = C[i];
  };
  // P (ldp) = [V_1..V_nb]^T W with the split-K chunk count tuned per shape
  auto proj = [&](int nb, const double* Vp, int64_t vb, const double* W, double* P,
                  int ldp) -> int {
    std::vector<int> cands;
    for (int c : {64, 128, 256})
      if (c <= kNsplitMax && c <= std::max<int64_t>(1, n / 64)) cands.push_back(c);
    if (cands.empty()) cands.push_back(1);
    int chosen = 0;
    return tune_pick({0, n, s, nb}, cands, cur,
                     [&](int c) {
                       return launch_blk_proj(n, s, nb, Vp, vb, W, part, c, P, ldp, false, cur);
                     },
                     &chosen, &S.ms_tune);
  };

  // CholQR2 of the block W in place; H_sub (ldsub) = R2 R1
  auto cholqr2 = [&](double* W, double* Hsub, int64_t ldsub, int step) -> int {
    for (int pass = 0; pass < 2; ++pass) {
      {
        const int r = proj(1, W, 0, W, G, s);
        if (r) return r;
      }
      BLK_HIP(launch_chol(s, G, pass == 0 ? Rt : R, Ri, flag + step, cur));
      BLK_HIP(launch_gemm(n, s, s, 1.0, W, 0, s, s, Ri, s, 0.0, W, s, cur));
    }
    // Hsub = R (second) * Rt (first)
    BLK_HIP(launch_gemm(s, s, s, 1.0, R, 0, s, s, Rt, s, 0.0, Hsub, ldsub, cur));
    return FA_OK;
  };

  // Z = H_m^{-1/2} E_1 R_0 on the device (coupled Newton-Schulz), m blocks
  auto invsqrt_E1R = [&](int m, int* iters) -> int {
    const int Mm = m * s;
    double hn[2] = {0.0, 0.0};
    BLK_HIP(launch_mat_norms(Mm, H, L.ldh, nrm, rowsc, st));
    BLK_HIP(hipMemcpyAsync(hn, nrm, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    BLK_HIP(hipStreamSynchronize(st));
    const double c = hn[0];
    if (!(c > 0.0) || !std::isfinite(c)) return FA_ERR_NONFINITE;
    double *Y = NS[0], *Z = NS[1], *Tm = NS[2], *Tmp = NS[3];
    BLK_HIP(launch_scale_mat(Mm, Mm, 1.0 / c, H, L.ldh, Y, Mm, st));
    BLK_HIP(launch_set_diag(Mm, Mm, 1.0, Z, Mm, st));
    int it = 0;
    double prev = 1e300;
    for (;; ++it) {
      // T = (3 I - Z Y) / 2
      BLK_HIP(launch_set_diag(Mm, Mm, 1.5, Tm, Mm, st));
      BLK_HIP(launch_gemm(Mm, Mm, Mm, -0.5, Z, 0, Mm, Mm, Y, Mm, 1.0, Tm, Mm, st));
      BLK_HIP(launch_mat_norms(Mm, Tm, Mm, nrm, rowsc, st));
      BLK_HIP(hipMemcpyAsync(hn, nrm, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
      BLK_HIP(hipStreamSynchronize(st));
      const double dev = hn[1];  // max |T - I|
      if (!std::isfinite(dev) || it > 200 || (it > 20 && dev > 4.0 * prev))
        return FA_ERR_HESSENBERG;  // no convergence
      prev = dev;
      if (dev == 0.0) break;
      // Y <- Y T, Z <- T Z
      BLK_HIP(launch_gemm(Mm, Mm, Mm, 1.0, Y, 0, Mm, Mm, Tm, Mm, 0.0, Tmp, Mm, st));
      std::swap(Y, Tmp);
      BLK_HIP(launch_gemm(Mm, Mm, Mm, 1.0, Tm, 0, Mm, Mm, Z, Mm, 0.0, Tmp, Mm, st));
      std::swap(Z, Tmp);
      if (dev < 1e-14) {
        ++it;
        break;
      }
    }
    *iters = it;
    // Zc = (Z / sqrt(c))[:, 0:s] R_0
    BLK_HIP(launch_gemm(Mm, s, s, 1.0 / std::sqrt(c), Z, 0, Mm, s, R0, s, 0.0, Zc, s, st));
    return FA_OK;
  };

  // ---- start block -------------------------------------------------------
  const double* Bp = (const double*)d_B;
  if (kind == FA_SQRT) {  // B' = A B into the slot of V_2 (free until step 1)
    BLK_HIP(launch_blk_chain(op, s, d_B, nullptr, nullptr, Vb(1), ChainCoef{1.0, 0.0, 0.0, 0.0},
                             P64, P64, P64, st));
    mvms += s;
    Bp = Vb(1);
  }
  if (K == 0) {
    BLK_HIP(hipMemcpyAsync(Vb(0), Bp, (size_t)n * s * 8, hipMemcpyDeviceToDevice, st));
  } else {  // C = q(A) B' on the columns
    BLK_HIP(launch_blk_rows_to_cols(n, s, Bp, C[0], pc, st));
    void* const tq[4] = {C[1], C[2], C[3], C[4]};
    void* res = nullptr;
    int r = qcols(C[0], tq, &res);
    if (r) return r;
    BLK_HIP(launch_blk_cols_to_rows(n, s, res, pc, Vb(0), st));
  }
  {
    int r = cholqr2(Vb(0), R0, s, m_max + 1);
    if (r) return r;
  }

  // ---- block Arnoldi loop --------------------------------------------------
  std::vector<double> Hh;      // host copy of H columns (row-major, ldh), for checks
  std::vector<double> zprev, zcur((size_t)L.M * s);
  int m = m_max;
  bool converged = false, breakdown = false;
  double colmax = 0.0, est_max = 1.0;
  int ns_iters = 0;
  // one block step: W = A q(A)^2 V_j, block CGS2, CholQR2 (all launches on `cur`)
  auto do_step = [&](int j) -> int {
    double* W = Vb(j + 1);
    if (K == 0) {
      BLK_HIP(launch_blk_chain(op, s, Vb(j), nullptr, nullptr, W, ChainCoef{1.0, 0.0, 0.0, 0.0},
                               P64, P64, P64, cur, zc));
      mvms += s;
    } else {
      // V_j to columns (FP64, in W, free until the end of the step), U = A V_j
      // in the chain precision, then q(A) twice on the batch, and the result
      // back to rows in W
      BLK_HIP(launch_blk_rows_to_cols(n, s, Vb(j), W, P64, cur));
      BLK_HIP(launch_chain(opb, W, nullptr, nullptr, C[0], ChainCoef{1.0, 0.0, 0.0, 0.0}, cur,
                           P64, pc));
      mvms += s;
      void* y = nullptr;
      {
        void* const t1[4] = {C[1], C[2], C[3], C[4]};
        const int r = qcols(C[0], t1, &y);
        if (r) return r;
      }
      void* w = nullptr;
      {
        void* t2[4];
        others(y, t2);
        const int r = qcols(y, t2, &w);
        if (r) return r;
      }
      BLK_HIP(launch_blk_cols_to_rows(n, s, w, pc, W, cur));
    }
    // block CGS2: H(0:(j+1)s, js:(j+1)s) = P1 + P2
    const int nb = j + 1;
    double* Hcol = H + (size_t)j * s;
    {
      int r = proj(nb, V, L.bstride, W, Hcol, (int)L.ldh);
      if (r) return r;
      BLK_HIP(launch_gemm(n, s, nb * s, -1.0, V, L.bstride, s, s, Hcol, L.ldh, 1.0, W, s, cur));
      r = proj(nb, V, L.bstride, W, P2, s);
      if (r) return r;
    }
    BLK_HIP(launch_gemm(n, s, nb * s, -1.0, V, L.bstride, s, s, P2, s, 1.0, W, s, cur));
    BLK_HIP(launch_add_mat(nb * s, s, P2, s, Hcol, L.ldh, cur));
    // W = V_{j+1} H_{j+1,j}
    {
      int r = cholqr2(W, H + (size_t)(j + 1) * s * L.ldh + (size_t)j * s, L.ldh, j);
      if (r) return r;
    }
    return FA_OK;
  };
  const bool use_graph = (flags & FA_GRAPH) != 0;
  const int64_t step_mvms = (int64_t)(K > 0 ? 2 * K + 1 : 1) * s;
  // run step j: replayed from a captured graph when FA_GRAPH is set and its
  // launch parameters are tuned already, else launched one by one
  auto run_step = [&](int j) -> int {
    const bool tuned = is_tuned({0, n, s, j + 1}) && is_tuned({0, n, s, 1});
    if (!use_graph || !tuned) return do_step(j);
    const std::vector<int64_t> key{(int64_t)op.uid, (int64_t)op.poly_version, (int64_t)(uintptr_t)ws,
                                   s, m_max, mixed ? 1 : 0, j, zc, n};
    hipGraphExec_t exec = nullptr;
    {
      std::lock_guard<std::mutex> g(graphs().mu);
      auto it = graphs().execs.find(key);
      if (it != graphs().execs.end()) exec = it->second;
    }
    if (exec) {
      mvms += step_mvms;
      ++S.graph_steps;
      BLK_HIP(hipGraphLaunch(exec, st));
      return FA_OK;
    }
    // captured on the caller's stream (not the null stream: checked at entry)
    BLK_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const int r = do_step(j);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &graph);
    if (r) {
      if (graph) (void)hipGraphDestroy(graph);
      return r;
    }
    if (e != hipSuccess) return FA_ERR_HIP;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return FA_ERR_HIP;
    {
      std::lock_guard<std::mutex> g(graphs().mu);
      auto ins = graphs().execs.emplace(key, exec);
      if (!ins.second) {  // another thread stored one meanwhile
        (void)hipGraphExecDestroy(exec);
        exec = ins.first->second;
      }
    }
    ++S.graph_steps;
    BLK_HIP(hipGraphLaunch(exec, st));
    return FA_OK;
  };

  for (int j = 0; j < m_max; ++j) {
    {
      const int r = run_step(j);
      if (r) return r;
    }
    const int jj = j + 1;
    const bool check = (tol > 0.0) ? (jj % k_chk == 0 || jj == m_max) : (jj == m_max);
    if (!check) continue;
    // breakdown scan on the host copy of the new columns and the flags
    const int rows = (jj + 1) * s;
    Hh.assign((size_t)rows * L.ldh, 0.0);
    std::vector<int> fl(m_max + 2, 0);
    BLK_HIP(hipMemcpyAsync(Hh.data(), H, (size_t)rows * L.ldh * 8, hipMemcpyDeviceToHost, st));
    BLK_HIP(hipMemcpyAsync(fl.data(), flag, (size_t)(m_max + 2) * sizeof(int),
                           hipMemcpyDeviceToHost, st));
    BLK_HIP(hipStreamSynchronize(st));
    if (fl[m_max + 1]) return FA_ERR_HESSENBERG;  // rank-deficient start block
    int mb = -1;
    for (int c = 0; c < jj && mb < 0; ++c) {
      for (int b = 0; b < s; ++b) {
        double cn = 0.0;
        for (int r = 0; r < (c + 2) * s; ++r) {
          const double v = Hh[(size_t)r * L.ldh + c * s + b];
          if (!std::isfinite(v)) return FA_ERR_NONFINITE;
          cn += v * v;
        }
        colmax = std::max(colmax, std::sqrt(cn));
      }
      int small = 0;
      for (int b = 0; b < s; ++b)
        if (std::fabs(Hh[(size_t)((c + 1) * s + b) * L.ldh + c * s + b]) <= 1e-12 * colmax) ++small;
      if (small == s) {
        mb = c + 1;  // the block Krylov space is invariant
      } else if (small > 0 || fl[c]) {
        return FA_ERR_HESSENBERG;  // partial rank loss: would need deflation
      }
    }
    if (mb > 0) {
      m = mb;
      breakdown = converged = true;
      break;
    }
    if (tol <= 0.0) break;
    const double th = now_ms();
    int it = 0;
    int r = invsqrt_E1R(jj, &it);
    if (r) return r;
    ns_iters = it;
    ++S.checks;
    BLK_HIP(hipMemcpyAsync(zcur.data(), Zc, (size_t)jj * s * s * 8, hipMemcpyDeviceToHost, st));
    BLK_HIP(hipStreamSynchronize(st));
    S.ms_fH += now_ms() - th;
    // per-column relative change of the coefficient block
    est_max = 0.0;
    for (int b = 0; b < s; ++b) {
      double dn = 0.0, zn = 0.0;
      for (int i = 0; i < jj * s; ++i) {
        const double z = zcur[(size_t)i * s + b];
        const double zp = (i < (int)(zprev.size() / s)) ? zprev[(size_t)i * s + b] : 0.0;
        dn += (z - zp) * (z - zp);
        zn += z * z;
      }
      est_max = std::max(est_max, std::sqrt(dn / zn));
    }
    zprev.assign(zcur.begin(), zcur.begin() + (size_t)jj * s * s);
    if (est_max <= tol) {
      m = jj;
      converged = true;
      break;
    }
  }
  // final coefficients unless the loop ended on a fresh check of size m
  if ((int)(zprev.size() / s) != m * s || breakdown) {
    const double th = now_ms();
    int it = 0;
    int r = invsqrt_E1R(m, &it);
    if (r) return r;
    ns_iters = it;
    S.ms_fH += now_ms() - th;
  }
  // X = [V_1 .. V_m] Z
  BLK_HIP(launch_gemm(n, s, m * s, 1.0, V, L.bstride, s, s, Zc, s, 0.0, (double*)d_X, s, st));
  BLK_HIP(hipStreamSynchronize(st));
  S.iters = m;
  S.converged = converged ? 1 : 0;
  S.breakdown = breakdown ? 1 : 0;
  S.ns_iters = ns_iters;
  S.zc = zc;
  S.mvms = mvms;
  S.est_max = est_max;
  S.ms_total = now_ms() - t0;
  if (stats) *stats = S;
  return converged ? FA_OK : FA_WARN_NOT_CONVERGED;
}

}  // namespace fa
