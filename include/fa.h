/*
 * fa.h -- polynomially preconditioned Krylov approximation of A^{-1/2} b and
 * A^{1/2} b on an MI355X (gfx950), behind a plain C ABI.
 *
 * Method (Frommer, Ramirez-Hidalgo, Schweitzer, Tsolakis, "Polynomial
 * preconditioning for the action of the matrix square root and inverse square
 * root", arXiv 2401.06684):
 *
 *   Problem (Sec. 1): given A in C^{n x n} and b, approximate f(A) b for
 *   f(z) = z^{-1/2} or z^{1/2} (principal branch, cut on (-inf, 0], Sec. 3)
 *   with a polynomial Krylov method, without shifted linear solves.
 *
 *   Identity (Sec. 3, eq. prec_identity): with q ~ z^{-1/2} a polynomial whose
 *   values on spec(A) lie in the open right half-plane,
 *       A^{-1/2} b = (A q(A)^2)^{-1/2} q(A) b.
 *   Left preconditioning (Algorithm 1): Arnoldi on A q(A)^2 from c = q(A) b,
 *   f_m = V_m H_m^{-1/2} e_1 ||c||.  Each step applies A once and q(A) twice
 *   (the three-stage product of Algorithm 1; q^2 is never formed).
 *   Square root (Sec. 4): A^{1/2} b = A^{-1/2} (A b).
 *   Stopping (Sec. 3.1, Sec. 6): every k steps the relative change of the
 *   iterate ||f_j - f_{j-k}|| / ||f_j||, computed from the coefficient vectors
 *   because V is orthonormal; k = max(1, 64 / (degree + 1)) by default.
 *
 * Everything on the path runs on the device (the operator, the polynomial
 * chain, Gram-Schmidt, the final combination) except the small dense
 * H_m^{-1/2} e_1, evaluated in FP64 on the host (Schur method, Sec. 3.1).
 *
 * Conventions for every entry point:
 *   - Return value: 0 = FA_OK, > 0 = warning (outputs valid), < 0 = error
 *     (outputs undefined).  fa_status_string() names each code.
 *   - "d_" arguments are device pointers (memory of the current HIP device),
 *     "h_" arguments host pointers.  All device memory is owned by the caller;
 *     the library never allocates device memory (it calls no hipMalloc): the
 *     Krylov basis and scratch come in a caller workspace (fa_workspace_bytes),
 *     an operator's own device data (the reordered Wilson links, the CSR list
 *     of long rows) in caller "operator memory" (fa_op_device_bytes).  It
 *     borrows operator arrays and operator memory given to fa_create_* until
 *     fa_destroy.  The only memory it allocates is page-locked host memory
 *     for the small copies at the stopping checks (pooled for the process).
 *   - The library creates no streams: all device work goes to the caller's
 *     streams (hip_stream arguments; fa_server_create takes one per worker).
 *   - hip_stream is a hipStream_t (NULL = the default stream).  All device
 *     work of a call is enqueued on it; calls that return host results
 *     synchronize that stream before returning.
 *   - FP64 vectors are contiguous double[n]; complex vectors (FA_C128) are
 *     contiguous interleaved (re, im) double pairs, i.e. C99 double complex,
 *     same layout as torch.complex128.
 *   - An fa_op is immutable after fa_poly_setup; concurrent fa_apply calls on
 *     one op are allowed with distinct workspaces and streams.
 */
#ifndef FA_H
#define FA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fa_op_s* fa_op;

/* status codes */
enum {
  FA_OK = 0,
  FA_WARN_NOT_CONVERGED = 1, /* m_max reached; x = f_{m_max} is returned           */
  FA_ERR_ARG = -1,           /* invalid argument (null pointer, size, kind, ...)    */
  FA_ERR_NO_POLY = -2,       /* fa_apply before fa_poly_setup                        */
  FA_ERR_BRANCH = -3,        /* q not positive on the spectral interval, or a Ritz
                                value with Re <= 0: the principal root is not
                                guaranteed (Sec. 3, Sec. 5.1, Sec. 5.2)              */
  FA_ERR_HESSENBERG = -4,    /* H_m has an eigenvalue on (-inf, 0]: no principal
                                H_m^{-1/2}                                            */
  FA_ERR_WORKSPACE = -5,     /* workspace null, misaligned or too small              */
  FA_ERR_HIP = -6,           /* a HIP runtime call failed                            */
  FA_ERR_NONFINITE = -7,     /* NaN or Inf met in b or in the iteration              */
  FA_ERR_NO_INTERVAL = -8,   /* Chebyshev setup without a spectral interval          */
  FA_ERR_UNSUPPORTED = -9    /* combination not available for this operator          */
};

/* value types */
enum { FA_F64 = 0, FA_C128 = 1 };

/* functions */
enum { FA_INVSQRT = 0, FA_SQRT = 1 };

/* matrix-free operators for fa_create_stencil; FA_CSR names fa_create_csr's
 * operators in fa_op_device_bytes */
enum {
  FA_STENCIL7 = 0, /* real 7-point (3D) or 5-point (nz = 1) stencil, zero Dirichlet  */
  FA_WILSON4D = 1, /* Wilson-Dirac-like operator, periodic 4D lattice, complex       */
  FA_CSR = 2       /* sparse matrix in CSR form (fa_create_csr)                       */
};

/* polynomial constructions for fa_poly_setup */
enum {
  FA_POLY_AUTO = 0, /* CHEB when the op has a real spectral interval, else RITZ     */
  FA_POLY_CHEB = 1, /* Chebyshev interpolant of z^{-1/2} on [lo, hi], Sec. 5.1      */
  FA_POLY_RITZ = 2, /* interpolant at Ritz values, Newton form, Leja order, Sec. 5.2 */
  FA_POLY_HARMONIC = 3, /* as RITZ at the harmonic Ritz values (the eigenvalues of
                          H_d + h_{d+1,d}^2 H_d^{-H} e_d e_d^T), Sec. 5.2           */
  FA_POLY_LS = 4       /* least-squares fit of z^{-1/2} on a contour around the Ritz
                          values, Sec. 5.3 (fa_poly_setup_ls)                     */
};

/* flags */
enum {
  FA_HERMITIAN = 1u,     /* create: A is Hermitian; apply uses Lanczos (3-term)        */
  FA_FORCE_ARNOLDI = 4u, /* apply: Gram-Schmidt (CGS2) even for a Hermitian op          */
  FA_PROFILE = 8u,       /* apply: time the middle terms of every q(A) application      */
  FA_NO_FUSION = 16u,    /* apply: one launch per recurrence term (no multi-term launches) */
  FA_FUSE2 = 1024u,      /* apply: at most two recurrence terms per launch (default on a
                            7-point stencil: four per launch, then the largest
                            group that fits: three, a pair or a single term)    */
  FA_FUSE3 = 2048u,      /* apply: at most three recurrence terms per launch        */
  FA_TWO_PASS = 64u,     /* apply: two-pass Lanczos (Hermitian op, not with
                            FA_FORCE_ARNOLDI, else FA_ERR_UNSUPPORTED): pass 1
                            keeps three basis vectors and computes H_m and
                            z_m = H_m^{-1/2} e_1 ||c||; pass 2 regenerates
                            v_1..v_m with the same kernels and accumulates
                            x = sum_i z_i v_i.  Workspace O(n), about twice the
                            products with A.  With FA_RIGHT_PREC (Algorithm 2)
                            x = q(A) (V_m z_m), one more q(A) at the end, and
                            only a fixed m (tol <= 0; else FA_ERR_UNSUPPORTED:
                            the right variant's stopping estimate needs the
                            stored y_j).                                         */
  FA_RIGHT_PREC = 128u,  /* apply: right preconditioning (Algorithm 2): the basis of
                            K_m(A q(A)^2, b), y_j = q(A) v_j stored, x = Y_m z_m with
                            z_m = H_m^{-1/2} e_1 ||b||.  The stopping estimate is
                            ||Y_j (z_j - [z_{j-k}; 0])|| / ||Y_j z_j||.  Not with
                            FA_MIXED.  With q == 1 it is the plain method.         */
  FA_CGS2 = 512u,        /* apply: classical Gram-Schmidt applied twice in every
                            Arnoldi step.  Default: the second pass of step j is
                            delayed to step j + 1 and merged with its first
                            (one sweep of projections on two vectors and one
                            of updates per step instead of two of each); the
                            same Arnoldi relation up to rounding.  Lanczos and
                            FA_RIGHT_PREC always use their own scheme. */
  FA_GRAPH = 256u,       /* fa_block_apply: run each block step from a HIP graph,
                            captured at the step's first use once its launch
                            parameters are tuned and replayed afterwards (per op,
                            polynomial, workspace address, block size, m_max,
                            precision and step index; released by fa_destroy) */
  FA_Q2 = 4096u,         /* create (FA_WILSON4D): the operator is A = Q^2, Q = Gamma_5 D
                            (Sec. 6, Example 2: the sign function of Q through
                            (Q^2)^{-1/2}); each product with A is two products with
                            Q, Q^2 is never formed.  Applying it needs one
                            vector of scratch from the workspace (see
                            fa_workspace_bytes, fa_op_apply).                    */
  FA_MIXED = 32u         /* apply: the polynomial chain (A and q(A) in the three-stage
                            product, and c = q(A) b) in FP32 storage with FP32
                            accumulation; Gram-Schmidt, H, H^{-1/2} e_1, the basis and
                            x = V z stay FP64.  7-point stencil with a Chebyshev q of
                            degree >= 1 (degree 0: the flag is ignored); other
                            operators or polynomials: FA_ERR_UNSUPPORTED             */
};

typedef struct {
  int32_t iters;          /* m: Krylov dimension of the returned iterate               */
  int32_t converged;      /* 1 if est <= tol or a lucky breakdown occurred              */
  int32_t breakdown;      /* 1 if h_{m+1,m} vanished (Krylov space invariant)           */
  int32_t checks;         /* number of host evaluations of H_j^{-1/2} e_1               */
  int64_t mvms;           /* products with A in fa_apply: m (2K + 1) + K (+1 for sqrt)  */
  int64_t mvms_setup;     /* products with A in fa_poly_setup (Ritz: d)                 */
  int64_t inner_products; /* length-n inner products in the iteration (FA_CGS2: 2j + 1
                             at step j of m; delayed CGS2: 2j at step j, its second
                             pass taken in step j + 1, plus j + 1 for a check that
                             projects u_{j+1} itself; Lanczos: 2 per step)              */
  double est_rel_change;  /* last ||f_j - f_{j-k}|| / ||f_j||                           */
  double h_last;          /* h_{m+1,m}                                                  */
  double ms_total;        /* wall time of fa_apply                                      */
  double ms_host_fH;      /* host time spent in H_j^{-1/2} e_1                          */
  double ms_chain;        /* FA_PROFILE: device time of the timed chain launches, the
                             launches of the middle of a q(A) recurrence (the Clenshaw
                             terms that read x, v, b_{k+2}; the Newton terms that read
                             r, v).  A stencil launch of three or four terms carries
                             its own start and end event (the dispatch's own time);
                             other launches are timed by HIP events bracketing each
                             run of consecutive ones, which includes the short gaps
                             between them.  Each event pair adds a few microseconds
                             to the solve.                                             */
  int64_t n_chain;        /* FA_PROFILE: number of chain launches timed                 */
  double chain_bytes;     /* FA_PROFILE: algorithmic bytes of one timed launch: x, each
                             combined vector and each output once, plus the operator's
                             own arrays (Wilson links, CSR arrays)                      */
  int64_t n_chain_terms;  /* FA_PROFILE: recurrence terms in the timed launches        */
} fa_stats;

/*
 * fa_op_device_bytes -- bytes of caller "operator memory" (d_opmem) that
 * fa_create_csr / fa_create_stencil may need for an operator of this kind and
 * size (an upper bound: the op uses what it needs of it).
 *   FA_STENCIL7: 0 (the op is its 7 coefficients).
 *   FA_CSR     : the work split of the n rows and nnz entries, bounded by
 *                16 n bytes of row blocks, 16 c bytes of chunks of long rows
 *                and 12 l bytes of long rows, each rounded up to a multiple
 *                of 256, where l = nnz / 4097 + 1, c = 2 l + nnz / 4096.
 *   FA_WILSON4D: 576 V bytes (V = Lx Ly Lz Lt from dims): the links in the
 *                kernels' order, whole; special unitary links use 384 V of it
 *                (with FA_Q2 too: its scratch vector is workspace, per call).
 * Returns 0 for an unknown kind or invalid dims.  Needs no GPU.
 */
size_t fa_op_device_bytes(int kind, const int32_t dims[4], int64_t n, int64_t nnz);

/*
 * fa_create_csr -- borrow a CSR matrix (the sparse matrix-vector product of
 * Sec. 6, Examples 1 and 3).
 *   n, nnz       : order and stored entries (n >= 1, nnz >= 0, < 2^31)
 *   d_rowptr     : int32[n + 1], d_rowptr[0] = 0, nondecreasing, d_rowptr[n] = nnz
 *   d_colind     : int32[nnz], column indices in [0, n)
 *   d_vals       : double[nnz] (FA_F64) or double complex[nnz] (FA_C128)
 *   dtype        : FA_F64 or FA_C128 (vectors passed to fa_apply use the same type)
 *   flags        : FA_HERMITIAN to select Lanczos in fa_apply
 *   d_opmem      : operator memory, opmem_bytes bytes, 256-byte aligned,
 *                  fa_op_device_bytes(FA_CSR, NULL, n, nnz) bytes suffice;
 *                  borrowed until fa_destroy.
 * The arrays are not copied; they must stay alive and unchanged until
 * fa_destroy.  hip_stream is synchronized first (the arrays may be written
 * on it); then the row pointers and column indices are read once to the host
 * to check them and to pick the work split, written to d_opmem: blocks of
 * consecutive rows with at most 4096 entries and 512 rows each (one
 * 512-thread workgroup streams a block's entries through LDS and sums each
 * row with a lane group sized to the block), and rows of more than 4096
 * entries, a workgroup each, in the same launch.  A CSR op has no spectral
 * interval until fa_set_spectral_interval is called.
 * Errors: FA_ERR_ARG (row pointers that do not start at 0, end at nnz and
 * never decrease, or a column index outside [0, n)), FA_ERR_WORKSPACE
 * (d_opmem NULL, misaligned or too small for the split), FA_ERR_HIP.
 */
int fa_create_csr(fa_op* out, int64_t n, int64_t nnz, const int32_t* d_rowptr,
                  const int32_t* d_colind, const void* d_vals, int dtype, uint32_t flags,
                  void* d_opmem, size_t opmem_bytes, void* hip_stream);

/*
 * fa_create_stencil -- a matrix-free operator.
 *   FA_STENCIL7: dims = {nx, ny, nz, 1}, x fastest (index i + nx (j + ny k));
 *     params = 7 doubles {c0, c_xm, c_xp, c_ym, c_yp, c_zm, c_zp}:
 *       (A u)_p = c0 u_p + c_xm u_{p-ex} + c_xp u_{p+ex} + c_ym u_{p-ey} + ...
 *     neighbours outside the grid are zero.  Real (FA_F64) vectors.  When
 *     c_dm c_dp > 0 in every direction the spectrum is real and the op gets the
 *     exact interval c0 -+ sum_d 2 sqrt(c_dm c_dp) cos(pi / (N_d + 1)) (for the
 *     Laplacian, the interval stated in Sec. 6, Example 1).
 *   FA_WILSON4D: dims = {Lx, Ly, Lz, Lt} (each >= 2), params = {m0} or
 *     {m0, mu} (1 or 2 doubles):
 *       (D psi)(x) = (4 + m0) psi(x) - 1/2 sum_nu [e^{mu d_nu,t} (I - g_nu) U_nu(x) psi(x + nu)
 *                                    + e^{-mu d_nu,t} (I + g_nu) U_nu(x - nu)^H psi(x - nu)]
 *     (mu: chemical potential on the temporal hops, 0 by default; m0 < 0 is
 *     allowed, e.g. the shift m_w = -1.4 of Example 2); with flags FA_Q2 the
 *     op is A = (Gamma_5 D)^2, Gamma_5 = diag(1, 1, -1, -1) on spin;
 *     periodic, chiral-basis Euclidean gamma matrices; 12 complex per site,
 *     vectors [t][z][y][x][spin 4][colour 3] (FA_C128).  d_links: device
 *     double complex[4][Lt][Lz][Ly][Lx][3][3] (direction mu = x, y, z, t, row
 *     major 3x3), read once on hip_stream (which is synchronized) into the
 *     operator memory d_opmem, reordered so that one link element of
 *     consecutive sites is contiguous; the caller's link array may be freed
 *     after the call, d_opmem must live until fa_destroy.  When every link is
 *     special unitary (row 2 equals conj(row 0 x row 1) to within 1e-13,
 *     checked on the host at creation) only rows 0 and 1 are kept (24 V
 *     complex doubles) and the kernels rebuild row 2; otherwise all of it
 *     (36 V).  The Wilson-Dirac operator is the matrix of Sec. 6, Example 2
 *     without its clover term.
 *   flags: FA_HERMITIAN allowed only for symmetric stencils and for FA_Q2
 *     with mu = 0 (then Gamma_5 D is Hermitian); FA_Q2 only for FA_WILSON4D.
 *   d_opmem, opmem_bytes: operator memory (256-byte aligned), at least
 *     fa_op_device_bytes(kind, dims, 0, 0) bytes; NULL for FA_STENCIL7.
 * Errors: FA_ERR_ARG, FA_ERR_WORKSPACE (Wilson: d_opmem NULL, misaligned or
 * smaller than the links kept), FA_ERR_HIP (Wilson: the link copy failed).
 */
int fa_create_stencil(fa_op* out, int kind, const int32_t dims[4], const double* params,
                      int nparams, const void* d_links, uint32_t flags, void* d_opmem,
                      size_t opmem_bytes, void* hip_stream);

/* Set (or replace) the real interval [lo, hi], 0 < lo < hi, assumed to hold
 * spec(A); used by FA_POLY_CHEB (Sec. 5.1).  Errors: FA_ERR_ARG. */
int fa_set_spectral_interval(fa_op op, double lo, double hi);

/* Query the interval; returns FA_ERR_NO_INTERVAL if the op has none. */
int fa_get_spectral_interval(fa_op op, double* lo, double* hi);

/* Bytes of device workspace fa_poly_setup needs for `degree` (0 for CHEB;
 * for FA_POLY_LS: its default 60 setup Arnoldi steps, whatever the degree;
 * with ritz_steps s given to fa_poly_setup_ls, the figure for degree s - 1
 * and FA_POLY_RITZ). */
size_t fa_poly_workspace_bytes(fa_op op, int degree, int method);

/*
 * fa_poly_setup -- choose the preconditioning polynomial q of degree K
 * (K + 1 = the paper's d coefficients; K = 0 means q == 1, the plain method).
 *   FA_POLY_CHEB (Sec. 5.1): Chebyshev interpolant of z^{-1/2} at the K + 1
 *     first-kind Chebyshev points of [lo, hi]; q is checked positive on 10^4
 *     points of [lo, hi] plus the nodes (else FA_ERR_BRANCH).
 *   FA_POLY_RITZ (Sec. 5.2): K + 1 Arnoldi steps on A from d_start (a device
 *     vector of length n, the caller's random start vector; it is normalized
 *     internally and not modified); the Ritz values (eigenvalues of H_{K+1})
 *     are the interpolation nodes of z^{-1/2}, stored in Newton form on the
 *     Leja ordering with capacity scaling.  A Ritz value with Re <= 0 gives
 *     FA_ERR_BRANCH.  For real operators, conjugate pairs of Ritz values are
 *     evaluated in real arithmetic (quadratic factors); a pair with
 *     Re theta < 1e-3 |theta| gives FA_ERR_UNSUPPORTED.  If Arnoldi breaks down
 *     after j < K + 1 steps the degree becomes j - 1.  Needs d_workspace of
 *     fa_poly_workspace_bytes.
 *   FA_POLY_HARMONIC (Sec. 5.2): as RITZ with the harmonic Ritz values.
 *   FA_POLY_LS (Sec. 5.3): as fa_poly_setup_ls with ritz_steps 60, r_min 0.1
 *     and step 0.005 (the choices of Sec. 6, Example 3).
 * Runs on hip_stream and synchronizes it.  Errors: FA_ERR_ARG, FA_ERR_BRANCH,
 * FA_ERR_NO_INTERVAL, FA_ERR_WORKSPACE, FA_ERR_UNSUPPORTED, FA_ERR_HIP.
 */
int fa_poly_setup(fa_op op, int degree, int method, const void* d_start, void* d_workspace,
                  size_t ws_bytes, void* hip_stream);

/*
 * fa_poly_setup_ls -- the least-squares polynomial of Sec. 5.3, degree K
 * (1 <= K <= 63):
 *   1. ritz_steps (>= 2) Arnoldi steps on A from d_start give Ritz values
 *      (any with Re <= 0: FA_ERR_BRANCH);
 *   2. the contour is the boundary of their convex hull minus the disk
 *      |z| < r_min (the part of the hull boundary inside the disk replaced by
 *      the arc |z| = r_min), discretized at equal arc length with spacing at
 *      most `step`; for real operators the mirror images are added, so the
 *      point set is conjugate-symmetric and q has real coefficients;
 *   3. Arnoldi on diag(z_1..z_N) from [1..1]/sqrt(N) gives the orthonormal
 *      polynomials p_j of the discrete inner product and their recurrence;
 *      alpha = P^H z^{-1/2} (the least-squares solution); Re q(z_i) <= 0 at a
 *      point gives FA_ERR_BRANCH.
 *   q(A) v is then evaluated by the recurrence with A in place of z (K
 *   products with A, O(K^2) vector updates, no inner products); fa_apply's
 *   workspace then also holds K + 1 vectors for it (query fa_workspace_bytes
 *   after the setup).  Not with FA_MIXED.
 *   d_workspace: fa_poly_workspace_bytes(op, ritz_steps - 1, FA_POLY_RITZ)
 *   bytes.  Errors: FA_ERR_ARG, FA_ERR_BRANCH, FA_ERR_HESSENBERG (degenerate
 *   contour), FA_ERR_WORKSPACE, FA_ERR_HIP.
 */
int fa_poly_setup_ls(fa_op op, int degree, int ritz_steps, double r_min, double step,
                     const void* d_start, void* d_workspace, size_t ws_bytes, void* hip_stream);

/*
 * fa_poly_get -- read back the polynomial (host arrays of at least degree + 1
 * entries each; any pointer may be NULL).
 *   method: FA_POLY_CHEB / FA_POLY_RITZ / FA_POLY_HARMONIC / FA_POLY_LS, or -1
 *   for q == 1.
 *   CHEB: coef[i] = c_i, interval = {lo, hi}.
 *   RITZ: nodes_re/im = Leja-ordered Ritz values, coef_re/im = scaled Newton
 *         coefficients eta_j, *rho = scaling: q(z) = sum_j eta_j prod_{i<j} (z - theta_i)/rho.
 */
int fa_poly_get(fa_op op, int* degree, int* method, double* coef_re, double* coef_im,
                double* nodes_re, double* nodes_im, double* interval, double* rho);
/*   LS:   coef_re/im = alpha_j, *rho = N (number of contour points); the
 *         recurrence through fa_poly_get_ls. */

/* fa_poly_get_ls -- the recurrence of an FA_POLY_LS polynomial: *npts = N and
 * h_re/h_im (host, (K + 1) x K, column-major) = the Hessenberg matrix with
 * z p_{j-1} = sum_{i<=j} h_{i,j-1} p_i, p_0 = N^{-1/2}.  Errors: FA_ERR_ARG
 * (another kind of polynomial), FA_ERR_NO_POLY. */
int fa_poly_get_ls(fa_op op, int64_t* npts, double* h_re, double* h_im);

/* Bytes of device workspace fa_apply needs for Krylov dimension m_max:
 * (m_max + 1) basis vectors + 5 chain vectors + reduction scratch + H. */
size_t fa_workspace_bytes(fa_op op, int m_max, uint32_t flags);

/*
 * fa_apply -- x ~ A^{-1/2} b (kind FA_INVSQRT) or A^{1/2} b (FA_SQRT) by
 * left polynomially preconditioned Arnoldi (Algorithm 1) with classical
 * Gram-Schmidt applied twice (the second pass delayed by one step unless
 * FA_CGS2), or Lanczos for FA_HERMITIAN ops.
 *   d_b, d_x     : device vectors of length n (d_x must not alias d_b)
 *   m_max        : maximal Krylov dimension (>= 1)
 *   tol          : stop when ||f_j - f_{j-k}|| / ||f_j|| <= tol; tol <= 0 runs
 *                  exactly m_max steps
 *   check_every  : k; 0 selects max(1, 64 / (degree + 1))
 *   d_workspace  : >= fa_workspace_bytes(op, m_max, flags) bytes, 256-byte aligned
 *   stats        : filled if not NULL
 * A zero b returns x = 0.  A lucky breakdown returns the exact iterate of the
 * invariant Krylov space.  Returns FA_WARN_NOT_CONVERGED if m_max is reached
 * with est > tol (x = f_{m_max}).
 * Errors: FA_ERR_ARG, FA_ERR_NO_POLY, FA_ERR_WORKSPACE, FA_ERR_HESSENBERG,
 * FA_ERR_NONFINITE, FA_ERR_HIP.
 */
int fa_apply(fa_op op, int kind, const void* d_b, void* d_x, int m_max, double tol,
             int check_every, void* d_workspace, size_t ws_bytes, uint32_t flags,
             void* hip_stream, fa_stats* stats);

/*
 * fa_apply_noalloc -- fa_apply for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Arguments, flags and results as fa_apply, without the
 * workspace: the library keeps one static device array of
 * FA_NOALLOC_MAX_BYTES (64 MiB) per device, held from the library's first
 * use on that device until the process ends, and runs the solve in it.
 *   - The call allocates nothing: no device or page-locked memory, no HIP
 *     events (so no FA_PROFILE: FA_ERR_ARG; the stopping checks copy through
 *     pageable memory and the next step is not overlapped with them).
 *   - fa_workspace_bytes(op, m_max, flags) must not exceed
 *     FA_NOALLOC_MAX_BYTES, else FA_ERR_WORKSPACE (nothing runs).
 *   - All calls on one device share the array: the library serializes them
 *     (a host lock, held until the call's device work has finished), so
 *     concurrent calls from several threads wait for each other; the array
 *     keeps the last call's contents, and no call relies on them.
 * Errors: as fa_apply.
 */
#define FA_NOALLOC_MAX_BYTES ((size_t)64 << 20)
int fa_apply_noalloc(fa_op op, int kind, const void* d_b, void* d_x, int m_max, double tol,
                     int check_every, uint32_t flags, void* hip_stream, fa_stats* stats);

/* y = A x on the device (one operator application, the "mvm" of the paper's
 * tables).  x, y: device vectors of length n, not aliased.  d_workspace
 * (optional, >= fa_workspace_bytes(op, 1, 0) bytes, 256-byte aligned) lets a
 * CSR op split rows of more than 4096 entries over several workgroups; with
 * NULL each such row is summed by one workgroup (same result, bit for bit).
 * Errors: FA_ERR_ARG, FA_ERR_WORKSPACE, FA_ERR_HIP. */
int fa_op_apply(fa_op op, const void* d_x, void* d_y, void* d_workspace, size_t ws_bytes,
                void* hip_stream);

/* y = q(A) x by the polynomial's recurrence (Clenshaw for CHEB, Horner for
 * RITZ), K products with A.  d_workspace: >= fa_workspace_bytes(op, 1, 0). */
int fa_poly_apply(fa_op op, const void* d_x, void* d_y, void* d_workspace, size_t ws_bytes,
                  void* hip_stream);

/* Order n of the operator and its value type (FA_F64 / FA_C128). */
int fa_op_info(fa_op op, int64_t* n, int* dtype);

int fa_destroy(fa_op op);
const char* fa_status_string(int status);

/*
 * fa_dense_invsqrt_e1 -- host-only FP64 routine used at every stopping check:
 * z = H^{-1/2} (beta e_1) for an m x m upper Hessenberg H (column-major, leading
 * dimension ldh >= m), by reduction to complex Schur form with shifted QR,
 * the principal square root of the triangular factor (Bjorck-Hammarling
 * recurrence) and a triangular solve (Sec. 3.1).  dtype FA_F64: h and z are
 * double arrays; FA_C128: interleaved complex.  Needs no GPU.
 * Errors: FA_ERR_ARG, FA_ERR_HESSENBERG (eigenvalue on (-inf, 0] or QR did not
 * converge).
 */
int fa_dense_invsqrt_e1(int m, int dtype, const double* h_H, int ldh, double beta, double* h_z);

/* Host-only: z = T^{-1/2} (beta e_1) for the symmetric tridiagonal T with
 * diagonal alpha[m] and off-diagonal offd[m-1] (Lanczos).  Errors as above. */
int fa_dense_tridiag_invsqrt_e1(int m, const double* alpha, const double* offd, double beta,
                                double* z);

/* ------------------------------------------------------------------------
 * Several right-hand sides sharing the operator: block Arnoldi.
 *
 * The block form of Algorithm 1 (an extension: the paper treats one
 * right-hand side): C = q(A) B' = V_1 R_0 (B' = B, or A B for FA_SQRT);
 * each step W = q(A) (q(A) (A V_j)) on the s columns as one batch (the
 * single-vector stencil launches, up to four recurrence terms each, over all
 * columns at once), classical block Gram-Schmidt twice as
 * FP64 matrix-core products (H(:, j) = [V_1..V_j]^T W summed over both
 * passes), W = V_{j+1} H_{j+1,j} by Cholesky QR twice; every k steps
 * Z_j = H_j^{-1/2} E_1 R_0 (coupled Newton-Schulz iteration on the device, FP64)
 * and the per-column estimate ||Z_j e_c - [Z_{j-k} e_c; 0]|| / ||Z_j e_c||;
 * stop when every column is <= tol; X = [V_1..V_m] Z_m.
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t iters;       /* m: block steps                                     */
  int32_t converged;   /* every column's estimate <= tol, or lucky breakdown  */
  int32_t breakdown;   /* the new block vanished (invariant block space)      */
  int32_t checks;
  int32_t ns_iters;    /* Newton-Schulz iterations of the last H^{-1/2}       */
  int32_t zc;          /* z-planes per workgroup of the row-major block
                          stencil launches (A B for FA_SQRT, A V_j with q = 1) */
  int32_t graph_steps; /* block steps replayed from (or captured into) graphs */
  int32_t reserved;
  int64_t mvms;        /* products of A with single vectors (s per block)    */
  double est_max;      /* largest per-column estimate at the last check       */
  double ms_total;
  double ms_fH;        /* time in H^{-1/2} E_1 R_0 (device, incl. syncs)     */
  double ms_tune;      /* autotuning in this call (first use of a shape)     */
} fa_block_stats;

/* Workspace of fa_block_apply: (m_max + 1) FP64 basis blocks of n x s, five
 * chain blocks (FP32 with FA_MIXED), split-K partials, H ((m_max + 1) s x
 * m_max s) and four (m_max s)^2 matrices for the Newton-Schulz iteration. */
size_t fa_block_workspace_bytes(fa_op op, int s, int m_max, uint32_t flags);

/*
 * fa_block_apply -- X ~ A^{-1/2} B or A^{1/2} B for s right-hand sides.
 *   op       : a real 7-point stencil (fa_create_stencil FA_STENCIL7) with a
 *              Chebyshev q or q == 1; others: FA_ERR_UNSUPPORTED
 *   s        : 16, 32 or 64
 *   d_B, d_X : device, n x s FP64, ROW-MAJOR (entry (i, c) at i * s + c: the s
 *              values of grid point i contiguous); d_X must not alias d_B
 *   m_max    : maximal number of block steps; tol, check_every as fa_apply
 *   flags    : FA_MIXED (the stencil chain in FP32 storage and arithmetic;
 *              Gram-Schmidt, Cholesky QR, H^{-1/2} and X = V Z in FP64),
 *              FA_GRAPH (block steps from HIP graphs captured on hip_stream,
 *              which must not be the null stream; the same launches, so the
 *              same results)
 * d_B and d_X must be 32-byte aligned.  Launch parameters (the split-K chunk
 * count of the projections per basis size, the z-march length of the
 * stencil) are autotuned at the first use of a problem shape in the process
 * (timed on hip_stream, then cached).
 * Returns FA_OK, FA_WARN_NOT_CONVERGED, or FA_ERR_ARG, FA_ERR_NO_POLY,
 * FA_ERR_WORKSPACE, FA_ERR_UNSUPPORTED, FA_ERR_HESSENBERG (a new block lost
 * rank partially -- block Arnoldi without deflation cannot continue -- or the
 * Newton-Schulz iteration did not converge), FA_ERR_NONFINITE, FA_ERR_HIP.
 * Blocks the host at checks and at return.
 */
int fa_block_apply(fa_op op, int kind, int s, const void* d_B, void* d_X, int m_max, double tol,
                   int check_every, void* d_workspace, size_t ws_bytes, uint32_t flags,
                   void* hip_stream, fa_block_stats* stats);

/* ------------------------------------------------------------------------
 * Serving: a request loop of f(A)b solves with continuous admission.
 *
 * Requests (fa_apply arguments) are queued in arrival order.  The oldest
 * request is admitted as soon as a worker is idle and the device pool has
 * room for its workspace (fa_workspace_bytes(op, m_max, flags): the Krylov
 * basis of m_max + 1 vectors of n entries plus scratch), so basis memory
 * bounds the solves in flight.  Each worker runs on a stream of the caller
 * (fa_server_create); admitted solves run concurrently on the device and a finished
 * solve frees its memory and worker at once, whatever step the others are
 * at.  Operators and polynomials stay on the device between requests (the
 * caller creates and sets them up once).  Results do not depend on what else
 * runs (the kernels are deterministic): a solve gives the same bits alone
 * and in the mix.
 * ------------------------------------------------------------------------ */
typedef struct fa_server_s* fa_server;

typedef struct {
  int32_t status;       /* fa_apply's return value                          */
  int32_t worker;       /* index of the worker that ran it                  */
  fa_stats stats;       /* fa_apply's statistics                            */
  double t_submit_ms;   /* host steady clock at submit, admission, and end  */
  double t_start_ms;
  double t_done_ms;
  size_t ws_bytes;      /* pool bytes the request held                      */
} fa_request_info;

typedef struct {
  int32_t pending, inflight, peak_inflight;
  uint64_t completed;
  size_t pool_bytes, bytes_inflight, peak_bytes_inflight, largest_free;
} fa_server_info;

/* Create a server on the current device.  d_pool: device memory of
 * pool_bytes (256-byte aligned), borrowed for the server's lifetime, from
 * which request workspaces are carved.  n_workers (1..64): concurrent solves
 * at most.  hip_streams: n_workers hipStream_t of the caller (worker w runs
 * its solves on hip_streams[w]; distinct streams let the solves overlap, HIP
 * maps them onto the device's hardware queues), borrowed until
 * fa_server_destroy returns.  Errors: FA_ERR_ARG, FA_ERR_HIP. */
int fa_server_create(fa_server* out, void* d_pool, size_t pool_bytes, int n_workers,
                     void* const* hip_streams);

/* Queue one solve (arguments as fa_apply; FA_PROFILE not allowed).  d_b and
 * d_x must stay valid and untouched until the request is done; op must
 * outlive it.  Returns at once with *ticket.  Errors: FA_ERR_ARG,
 * FA_ERR_WORKSPACE (the workspace exceeds the whole pool). */
int fa_server_submit(fa_server srv, fa_op op, int kind, const void* d_b, void* d_x, int m_max,
                     double tol, int check_every, uint32_t flags, uint64_t* ticket);

/* *done = 1 once the request finished (its x is complete on the device). */
int fa_server_poll(fa_server srv, uint64_t ticket, int* done);

/* Block until the request finished, fill *info (may be NULL), forget the
 * ticket and return the request's fa_apply status.  One wait per ticket.
 * FA_ERR_ARG for an unknown ticket. */
int fa_server_wait(fa_server srv, uint64_t ticket, fa_request_info* info);

/* Queue depth, solves in flight, completed count and pool occupancy. */
int fa_server_status(fa_server srv, fa_server_info* info);

/* Finish every queued request and stop the workers.  No fa_server_wait may
 * be pending.  The pool and the streams stay the caller's. */
int fa_server_destroy(fa_server srv);

#ifdef __cplusplus
}
#endif
#endif /* FA_H */
