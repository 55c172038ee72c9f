// Host runtime entry points used by the C ABI layer.
#pragma once
#include <vector>

#include "fa_internal.hpp"

namespace fa {

// device workspace layout of fa_apply for Krylov dimension m_max (offsets in
// bytes, every region 256-byte aligned)
struct Layout {
  int64_t ldv = 0;  // leading dimension of the basis (elements)
  int ldh = 0;      // leading dimension of H (elements)
  bool band = false;  // H stored as (diagonal, subdiagonal) pairs (Lanczos)
  size_t off_V = 0, off_Y = 0, off_U = 0, off_P = 0, off_Q = 0, off_R = 0, off_S = 0, off_part = 0, off_h = 0, off_H = 0,
         off_nrm = 0, off_z = 0;
  size_t off_W = 0;  // least-squares polynomial: its d basis vectors (0: none)
  size_t off_dc = 0; // coefficients of the delayed-reorthogonalization step
  size_t off_scr = 0, scr_bytes = 0;  // operator scratch (split CSR rows, Q x of Q^2; 0: none)
  size_t bytes = 0;
};
// with_poly: include the storage the op's polynomial needs (least squares)
Layout make_layout(const Op& op, int m_max, uint32_t flags, bool with_poly = true);

// One term of a polynomial recurrence: out_i = alpha A x_i + beta x_i + g0 v
// + g1 out_{i-2}, where x_i = out_{i-1} (x_0 = v, the vector q(A) acts on).
struct Term {
  ChainCoef k;
  bool y0, y1;
};
// the terms of q(A) v for a Chebyshev or (complex) Newton-form q (K terms)
std::vector<Term> poly_terms(const Poly& q);

// internal fa_apply flag (outside the public flag bits): allocate nothing,
// i.e. no page-locked check area (pageable copies instead) and no events
// (no half steps across the checks); profiling is refused by the caller
constexpr uint32_t kApplyNoAlloc = 1u << 30;

// the calling thread's chain launches use the operator scratch `scratch`
// (may be null) while this lives; its counters are cleared on construction
// (check ok())
class OpScratchScope {
 public:
  OpScratchScope(const Op& op, void* scratch, hipStream_t s)
      : err_(op_scratch_clear(op, scratch, s)), prev_(set_op_scratch(scratch)) {}
  ~OpScratchScope() { set_op_scratch(prev_); }
  bool ok() const { return err_ == hipSuccess; }
  OpScratchScope(const OpScratchScope&) = delete;
  OpScratchScope& operator=(const OpScratchScope&) = delete;

 private:
  hipError_t err_;
  void* prev_;
};

// q(A) x for the op's polynomial (and its batch settings), the chain in
// precision p, fused up to four terms per launch on a stencil: the result is
// left in *res, which is x, out or one of tmp (four vectors, none of them x or
// out); x may be overwritten when out == x.  *mvms += the degree.
int poly_apply_chain(const Op& op, const void* x, void* out, void* const tmp[4],
                     const void** res, hipStream_t s, int64_t* mvms, Prec p);
// y = A x; ws (may be null) of make_layout(op, 1, 0).bytes splits long CSR rows
int op_apply(const Op& op, const void* x, void* y, void* ws, hipStream_t s);
int poly_apply_public(const Op& op, const void* x, void* y, void* ws, hipStream_t s);
int apply(const Op& op, int kind, const void* d_b, void* d_x, int m_max, double tol,
          int check_every, void* ws, size_t ws_bytes, uint32_t flags, hipStream_t s,
          fa_stats* stats);
// parameters of the Sec. 5.3 least-squares polynomial (defaults: the choices
// of Sec. 6, Example 3)
struct LsParams {
  int ritz_steps = 60;
  double r_min = 0.1;
  double step = 0.005;
};
size_t block_workspace_bytes(const Op& op, int s, int m_max, uint32_t flags);
// destroy the block-step graphs cached for an op (fa_destroy)
void release_op_graphs(uint64_t uid);
int block_apply(const Op& op, int kind, int s, const void* d_B, void* d_X, int m_max, double tol,
                int check_every, void* ws, size_t ws_bytes, uint32_t flags, hipStream_t st,
                fa_block_stats* stats);
size_t poly_workspace_bytes(const Op& op, int degree, int method);
int poly_setup(Op& op, int degree, int method, const void* d_start, void* ws, size_t ws_bytes,
               hipStream_t s, int64_t* mvms_setup, const LsParams& ls = LsParams());

}  // namespace fa
