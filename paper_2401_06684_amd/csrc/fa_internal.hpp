// Internal declarations shared by the runtime (host) and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <memory>
#include <vector>

#include "../../include/fa.h"

namespace fa {

using cd = std::complex<double>;

// complex FP64 on the device: interleaved (re, im), 16-byte aligned
struct __attribute__((aligned(16))) cplx {
  double x, y;
};

enum OpKind { OP_CSR = 0, OP_STENCIL7 = 1, OP_WILSON = 2 };

// the preconditioning polynomial, in the representation the chain kernels use
struct Poly {
  int method = -1;  // -1: q == 1; FA_POLY_CHEB; FA_POLY_RITZ (Newton form); FA_POLY_LS
  bool harmonic = false;  // RITZ nodes are harmonic Ritz values
  // LS (Sec. 5.3): recurrence of the orthonormal polynomials (d x (d - 1),
  // column-major), coefficients alpha (d), number of contour points
  std::vector<cd> hls, alpha;
  long npts = 0;
  int degree = 0;   // K
  double a = 0, b = 0;        // CHEB interval
  std::vector<double> c;      // CHEB coefficients c_0..c_K
  std::vector<cd> theta;      // RITZ Leja-ordered nodes
  std::vector<cd> eta;        // RITZ scaled Newton coefficients
  double rho = 1.0;           // RITZ scaling
  // Real operators whose Ritz values include conjugate pairs: the Newton form
  // regrouped into real blocks (a real node, or a conjugate pair kept adjacent
  // by the Leja order).  With w_B the real product of the factors of the
  // blocks before B, q(z) = sum_B w_B(z) (a_B + b_B z).
  struct Block {
    bool pair;
    double re, im;  // the node (pair: theta = re + i im, im > 0)
    double a, b;    // real linear part a_B + b_B z
  };
  std::vector<Block> blocks;  // empty unless a real op has non-real nodes
};

struct Op {
  OpKind kind;
  int dtype;  // FA_F64 / FA_C128
  int64_t n;
  uint32_t flags;
  // CSR
  const int32_t* rowptr = nullptr;
  const int32_t* colind = nullptr;
  const void* vals = nullptr;
  int64_t nnz = 0;
  // work split, in the caller's operator memory: csr_nblk blocks of
  // consecutive rows with at most kCsrBlockEntries entries and kCsrBlockRows
  // rows each ({r0, r1, rowptr[r0], rowptr[r1]}), and csr_nlong rows with
  // more than kCsrBlockEntries entries ({row, first chunk, chunks}), cut into
  // csr_nchunk chunks of at most kCsrBlockEntries ({row, begin, end, long
  // index})
  int csr_nblk = 0, csr_nlong = 0, csr_nchunk = 0;
  int csr_maxrow = 0;  // entries of the longest row
  const int32_t* csr_blk_dev = nullptr;
  const int32_t* csr_chunk_dev = nullptr;
  const int32_t* csr_long_dev = nullptr;
  // stencil
  int dims[4] = {1, 1, 1, 1};
  double coef[7] = {0, 0, 0, 0, 0, 0, 0};
  // a batch of nbatch vectors, bstride elements apart, in each stencil chain
  // launch (set on a copy of the op by the block solver); multi_blocks: the
  // workgroup count the multi-term launches aim at (0: the default)
  int nbatch = 1;
  int64_t bstride = 0;
  int multi_blocks = 0;
  // Wilson: the links in the structure-of-arrays order Us[mu][e][s] (e the
  // row-major 3x3 element), in the caller's operator memory
  const void* links = nullptr;
  int links_rows = 3;  // rows of each link stored (2: special unitary, row 2 rebuilt)
  double m0 = 0.0;
  double mu = 0.0;     // chemical potential (temporal hops scaled by e^{+-mu})
  bool q2 = false;     // the op is (Gamma_5 D)^2
  // spectral interval
  bool has_interval = false;
  double lo = 0, hi = 0;
  Poly poly;
  bool poly_ready = false;
  // identity for caches that hold launch parameters of this op: a process-
  // wide unique id set at creation, and a counter bumped by every setup of q
  uint64_t uid = 0;
  uint64_t poly_version = 0;
};
// a fresh process-wide unique id (thread-safe)
uint64_t next_op_uid();

// CSR work split: a row block is at most kCsrBlockRows rows with at most
// kCsrBlockEntries entries, one workgroup of kCsrThreads threads with
// kCsrPer entries each; longer rows are cut into chunks of that size
#ifndef FA_CSR_THREADS
#define FA_CSR_THREADS 512
#endif
#ifndef FA_CSR_PER
#define FA_CSR_PER 8
#endif
constexpr int kCsrThreads = FA_CSR_THREADS;
constexpr int kCsrPer = FA_CSR_PER;
constexpr int kCsrBlockEntries = kCsrThreads * kCsrPer;
constexpr int kCsrBlockRows = kCsrThreads;

// storage precision of the vectors of one chain launch
enum Prec { P64 = 0, P32 = 1 };

// One fused chain launch: out = alpha A x + beta x + g0 y0 + g1 y1, with y0 /
// y1 optional (nullptr).  out may alias y1 (each point reads its own y1 entry
// before writing), never x.  Coefficients are complex; real ops use .real().
struct ChainCoef {
  cd alpha, beta, g0, g1;
};

// Two consecutive terms in one launch (7-point stencil only):
//   s = t1.alpha A x + t1.beta x + t1.g0 y0 + t1.g1 y1,  out1 = s (if out1),
//   out2 = t2.alpha A s + t2.beta s + t2.g0 y0 + t2.g1 x.
// out1 / out2 must not alias x, y0 or y1.
hipError_t launch_chain_pair(const Op& op, const void* x, const void* y0, const void* y1,
                             void* out1, void* out2, const ChainCoef& t1, const ChainCoef& t2,
                             hipStream_t s, Prec pin = P64, Prec pout = P64);
inline bool has_pair_kernel(const Op& op) { return op.kind == OP_STENCIL7; }
// nt = 3 or 4 consecutive terms s_t = a_t A s_{t-1} + b_t s_{t-1} + g0_t v +
// g1_t s_{t-2} (s_0 = x, s_{-1} = y1 or zero when y1 is null) on a 7-point
// stencil; writes s_{nt-1} to out1 (if not null) and s_nt to out2; k holds nt
// terms; blocks = target workgroup count (0: default); ev0 / ev1, if not
// null, receive the start and end time of the launch's own dispatch
hipError_t launch_chain_multi(const Op& op, int nt, const void* x, const void* v, const void* y1,
                              void* out1, void* out2, const ChainCoef* k, hipStream_t s,
                              Prec pin, Prec pout, int blocks = 0, hipEvent_t ev0 = nullptr,
                              hipEvent_t ev1 = nullptr);

// Operator scratch, from the caller's workspace: for a CSR op whose long
// rows are split over several workgroups, their partial sums and one counter
// per long row (nullptr: each long row summed by one workgroup, the same
// bits); for a Wilson op with q2, the intermediate vector Q x of a product
// with Q^2 (required).  The bytes a call needs (0: none), clearing the
// counters before the first launch of a call, and the scratch the chain
// launches of the calling thread use; set_op_scratch returns the previous
// one.
size_t op_scratch_bytes(const Op& op);
hipError_t op_scratch_clear(const Op& op, void* scratch, hipStream_t s);
void* set_op_scratch(void* p);

// Small Hermitian problems: the Lanczos steps j0 .. j1 - 1 of Algorithm 1 in
// one workgroup (kernels_small.hip).  Real FP64, n <= kSmallMaxN, a 7-point
// stencil or a CSR matrix with rows of at most kSmallRow entries, q == 1 or
// a Chebyshev q of at most kSmallMaxTerms terms.
constexpr int kSmallMaxN = 2048, kSmallRow = 8, kSmallMaxTerms = 32;
struct SmallTerm {  // out = a A x + b x + g0 v (if y0) + g1 out_{-2} (if y1)
  double a, b, g0, g1;
  int y0, y1;
};
struct SmallLanczosArgs {
  int n, j0, j1, nterms;
  int64_t ldv;
  double* V;  // basis, column-major, ldv
  double* H;  // banded H: column j = (H(j, j), H(j + 1, j))
  const int32_t* rowptr;
  const int32_t* colind;
  const double* vals;
  int nx, ny, nz;
  double c[7];
  SmallTerm t[kSmallMaxTerms];
};
bool small_lanczos_ok(const Op& op, const Poly& q);
hipError_t launch_small_lanczos(const Op& op, const std::vector<SmallTerm>& terms, int j0,
                                int j1, void* V, int64_t ldv, void* H, hipStream_t s);

// algorithmic bytes moved by one chain launch (x read once, y0, y1 read,
// out written, plus the operator's own data); p = storage of the vectors
double chain_bytes(const Op& op, bool has_y0, bool has_y1, Prec p = P64);
// algorithmic bytes of one two-term launch (x, y0, y1 read once; out1, out2 written)
double chain_pair_bytes(const Op& op, bool has_y0, bool has_y1, bool has_out1, Prec p = P64);
// y (FP32) = x (FP64), n entries
hipError_t launch_to_f32(int64_t n, const double* x, float* y, hipStream_t s);

// ---- kernel launchers (kernels_*.hip) ----
// pin: storage of x, y0, y1; pout: storage of out.  FP32 storage (with FP32
// arithmetic) is available for the 7-point stencil only.
// Us[mu][e][s] = U[mu][s][e] (complex FP64, 4 directions, the first ne = 9 or
// 6 elements of each row-major 3x3 link, V sites)
hipError_t launch_wilson_links_soa(int64_t V, int ne, const void* U, void* Us, hipStream_t s);
hipError_t launch_chain(const Op& op, const void* x, const void* y0, const void* y1, void* out,
                        const ChainCoef& k, hipStream_t s, Prec pin = P64, Prec pout = P64);

// Gram-Schmidt building blocks on a column-major basis V (ld = ldv elements).
// Partial sums go to `part` (ncols x nblk), the second stage writes `h`.
struct RedPlan {
  int nblk;     // blocks of the first stage
  int rows;     // rows per block
  int threads;  // threads per block
};
RedPlan red_plan(int64_t n);
// first-stage blocks of the projections on vectors of `dtype`
int proj_nblk(int64_t n, int dtype);
// h[c] = sum_r conj(V[r, c]) w[r], c < ncols (h may be null); hsum_mode 1 also
// stores hsum[c] = h[c], mode 2 adds it (CGS2: H(:, j) = h1 + h2), 0 ignores hsum
hipError_t launch_project(int dtype, int64_t n, int ncols, const void* V, int64_t ldv,
                          const void* w, void* part, void* h, void* hsum, int hsum_mode,
                          hipStream_t s);
// w[r] -= sum_c V[r, c] h[c]; if nrm2 != null also nrm2 = ||w_new||^2 (double)
hipError_t launch_update(int dtype, int64_t n, int ncols, const void* V, int64_t ldv,
                         const void* h, void* w, void* part, double* nrm2, hipStream_t s);
// x[r] = sum_c V[r, c] z[c]
hipError_t launch_combine(int dtype, int64_t n, int ncols, const void* V, int64_t ldv,
                          const void* z, void* x, hipStream_t s);
// out = w / sqrt(nrm2) (nrm2 on device); hout (if not null) = sqrt(nrm2) as a T
hipError_t launch_normalize(int dtype, int64_t n, const void* w, const double* nrm2,
                            void* out, void* hout, hipStream_t s);
// One step of CGS2 with delayed reorthogonalization, j >= 1: V columns
// 0..j-1 hold q_0..q_{j-1}, column j the once-orthogonalized u_j and column
// j + 1 the new z = Op u_j.  Finishes column j - 1 of H (column-major, ldh),
// forms the first-pass column j, and leaves q_j in column j and u_{j+1} in
// column j + 1.  part: 2 (j + 1) x nblk partials; S: 2 (j + 1) values;
// coef: 2 j + 2 values.  stage: kDcgs2All; kDcgs2Project, the projection
// and H (column j - 1 final, first-pass column j) only; kDcgs2Update, the
// update of columns j and j + 1 only (after a kDcgs2Project of the same j).
enum { kDcgs2All = 0, kDcgs2Project = 1, kDcgs2Update = 2 };
hipError_t launch_dcgs2(int dtype, int64_t n, int j, const void* V, int64_t ldv, void* part,
                        void* S, void* H, int64_t ldh, void* coef, hipStream_t s,
                        int stage = kDcgs2All);
// y = a * x for a scalar on the host
hipError_t launch_scale(int dtype, int64_t n, cd a, const void* x, void* y, hipStream_t s);

// least-squares polynomial step (kernel arguments by value; degree <= kLsMax)
constexpr int kLsMax = 64;
struct LsCoef {
  double re[kLsMax], im[kLsMax];  // g_i, i < k - 1
  double a0_re, a0_im, ak_re, ak_im;
};
hipError_t launch_ls_step(int dtype, int64_t n, int k, void* W, int64_t ldv, const LsCoef& g,
                          bool keep, void* out, hipStream_t s);

// ---- block (several right-hand sides) kernels, row-major n x s blocks ----
// one recurrence term on a block, 7-point stencil; s in {16, 32, 64}; storage
// of x (px), y0/y1 (py) and out (po): all FP64, all FP32, FP64 x -> FP32 out
// (no y), or FP32 x, y -> FP64 out; zc: z-planes per workgroup
hipError_t launch_blk_chain(const Op& op, int s, const void* x, const void* y0, const void* y1,
                            void* out, const ChainCoef& k, Prec px, Prec py, Prec po,
                            hipStream_t st, int zc = 8);
// a row-major n x s FP64 block to s vectors of n (column c at c * n; FP64 or
// FP32: py) and back; s in {16, 32, 64}; no aliasing
hipError_t launch_blk_rows_to_cols(int64_t n, int s, const double* X, void* Y, Prec py,
                                   hipStream_t st);
hipError_t launch_blk_cols_to_rows(int64_t n, int s, const void* Y, Prec py, double* X,
                                   hipStream_t st);
// one workgroup: ha[0:na) = a, hb[0:nb) = b (ha, hb, flag in page-locked
// coherent host memory, device-accessible), then *flag = seq once the copies
// are visible to the host
hipError_t launch_check_export(const double* a, int64_t na, double* ha, const double* b,
                               int64_t nb, double* hb, int* flag, int seq, hipStream_t s);
// P (row i*s + a, column b; leading dimension ldp) = (or +=) V_i^T W, i < nb,
// V_i = V + i * v_blk; split-K over nsplit chunks of rows (part holds
// nsplit * nb * s * s doubles)
hipError_t launch_blk_proj(int64_t n, int s, int nb, const double* V, int64_t v_blk,
                           const double* W, double* part, int nsplit, double* P, int ldp, bool acc,
                           hipStream_t st);
// C = alpha A B + beta C; A (r, k) at A[(k / kb) * a_blk + r * lda + k % kb]
hipError_t launch_gemm(int64_t M, int N, int K, double alpha, const double* A, int64_t a_blk,
                       int64_t lda, int kb, const double* B, int64_t ldb, double beta, double* C,
                       int64_t ldc, hipStream_t st);
// Cholesky G = R^T R and R^{-1} (s <= 64, row-major); *flag = 1 if G is not PD
hipError_t launch_chol(int s, const double* G, double* R, double* Rinv, int* flag,
                       hipStream_t st);
hipError_t launch_set_diag(int M, int N, double d, double* C, int64_t ldc, hipStream_t st);
hipError_t launch_scale_mat(int M, int N, double a, const double* X, int64_t ldx, double* Y,
                            int64_t ldy, hipStream_t st);
hipError_t launch_add_mat(int M, int N, const double* X, int64_t ldx, double* Y, int64_t ldy,
                          hipStream_t st);
// out[0] = max row sum of |X|, out[1] = max |X - I| (X square M x M);
// scratch holds 2 M doubles
hipError_t launch_mat_norms(int M, const double* X, int64_t ldx, double* out, double* scratch,
                            hipStream_t st);

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }
inline size_t elem_size(int dtype) { return dtype == FA_C128 ? 16 : 8; }

}  // namespace fa

// the opaque handle of the C ABI
struct fa_op_s {
  fa::Op op;
};
