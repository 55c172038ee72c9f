// Host FP64 dense linear algebra for the small problems of the method:
//   - H_m^{-1/2} e_1 for an upper Hessenberg H_m (Sec. 3.1: Schur form, principal
//     square root of the triangular factor, then a solve),
//   - T_m^{-1/2} e_1 for a symmetric tridiagonal T_m (Lanczos),
//   - eigenvalues of H_d (Ritz values, Sec. 5.2),
//   - Chebyshev interpolation coefficients (Sec. 5.1), Leja ordering and Newton
//     divided differences (Sec. 5.2).
// No LAPACK: everything is written here so the library has no host BLAS/LAPACK
// dependency.
#pragma once
#include <complex>
#include <vector>

namespace fa {

using cd = std::complex<double>;

enum DenseStatus { DENSE_OK = 0, DENSE_BRANCH = 1, DENSE_NOCONV = 2 };

// Complex Schur form of an upper Hessenberg matrix by the single-shift QR
// algorithm with Wilkinson shifts.  T (m x m, column-major, ld m) is
// overwritten by the upper triangular factor; the plane rotations are kept so
// that Q^H v and Q v can be applied to vectors afterwards (H = Q T Q^H).
struct Schur {
  int m = 0;
  std::vector<cd> T;
  struct Rot { int k; double c; cd s; };
  std::vector<Rot> rots;
  int compute(int m, const cd* H, int ldh);  // DENSE_OK or DENSE_NOCONV
  void apply_QH(cd* v) const;                // v <- Q^H v
  void apply_Q(cd* v) const;                 // v <- Q v
  cd t(int i, int j) const { return T[(size_t)j * m + i]; }
};

// z = H^{-1/2} (beta e_1); H complex upper Hessenberg (column-major, ldh).
int hess_invsqrt_e1(int m, const cd* H, int ldh, double beta, cd* z);

// Real Schur form of a real upper Hessenberg matrix by the Francis
// double-shift QR algorithm (3x3 Householder reflectors chasing the bulge),
// then each 2x2 diagonal block triangularized by a unitary 2x2 transform, so
// that H = Q T Q^H with T complex upper triangular.  About a quarter of the
// arithmetic of the complex single-shift algorithm.
struct RealSchur {
  int m = 0;
  std::vector<double> Tr;  // real quasi-triangular factor (column-major)
  std::vector<cd> T;       // complex triangular factor (column-major)
  struct Refl { int k, len; double v[3]; double tau; };  // I - tau v v^T on rows k..k+len-1
  struct Rot2 { int k; cd g1, g2; };                    // columns (g1, g2), (-conj g2, conj g1)
  std::vector<Refl> refl;
  std::vector<Rot2> rot;
  int compute(int m, const double* H, int ldh);
  void apply_QH(cd* v) const;
  void apply_Q(cd* v) const;
  cd t(int i, int j) const { return T[(size_t)j * m + i]; }
};

// z = H^{-1/2} (beta e_1) for a real upper Hessenberg H (z real up to rounding)
int real_hess_invsqrt_e1(int m, const double* H, int ldh, double beta, cd* z);

// z = T^{-1/2} (beta e_1); T symmetric tridiagonal.
int tridiag_invsqrt_e1(int m, const double* alpha, const double* offd, double beta,
                       double* z);

// eigenvalues of an upper Hessenberg matrix
int hess_eigenvalues(int m, const cd* H, int ldh, cd* ev);

// x = A^{-1} x for a general complex m x m matrix (column-major, ld m; A is
// overwritten by its LU factors).  Gaussian elimination with partial
// pivoting; DENSE_NOCONV if a pivot vanishes.
int lu_solve(int m, cd* A, cd* x);

// c_0..c_K of the Chebyshev interpolant of z^{-1/2} on [a, b] at K+1
// first-kind Chebyshev points.
void cheb_coefficients(double a, double b, int K, double* c);
// value of sum_i c_i T_i((2z - a - b)/(b - a)) at a real point (Clenshaw)
double cheb_eval(const double* c, int K, double a, double b, double z);

// Leja ordering (largest modulus first, then maximal product of distances;
// with pair_conjugates a non-real node is followed by its conjugate).
std::vector<cd> leja_order(const std::vector<cd>& nodes, bool pair_conjugates);
// capacity estimate rho = (prod_{i<d-1} |t_{d-1} - t_i|)^{1/(d-1)}
double leja_capacity(const std::vector<cd>& t);
// scaled Newton divided differences of z^{-1/2}: eta_j = f[t_0..t_j] rho^j
std::vector<cd> newton_invsqrt(const std::vector<cd>& t, double rho);

// Sec. 5.3 least-squares polynomial (lspoly.cpp).
// Convex hull of the points, counter-clockwise, collinear points dropped.
std::vector<cd> convex_hull(const std::vector<cd>& pts);
// Discretized boundary of (convex hull of theta) minus the disk |z| < r_min,
// equal arc-length spacing <= step; with `symmetric` the mirror images are
// appended.  DENSE_BRANCH if a hull vertex has Re <= 0; DENSE_NOCONV for a
// degenerate hull or one within r_min of 0.
int ls_contour(const std::vector<cd>& theta, double r_min, double step, bool symmetric,
               std::vector<cd>& out);
// Least-squares fit of z^{-1/2} of the given degree on the points: recurrence
// hls (d x (d - 1), column-major, ld d) of the orthonormal polynomials and
// their coefficients alpha (d = degree + 1).  DENSE_BRANCH if Re q <= 0 at a
// point; real_op: hls and alpha made real (the point set conjugate-symmetric).
int ls_fit_invsqrt(const std::vector<cd>& z, int degree, bool real_op, std::vector<cd>& hls,
                   std::vector<cd>& alpha);

}  // namespace fa
