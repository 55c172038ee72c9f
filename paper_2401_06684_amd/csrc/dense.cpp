// Host FP64 dense routines; see dense.hpp.
#include "dense.hpp"

#include <algorithm>
#include <cmath>
#include <limits>

namespace fa {

namespace {
constexpr double kEps = 2.220446049250313e-16;

// Plane rotation G = [[c, s], [-conj(s), c]] (c real) with G [x; y] = [r; 0].
inline void givens(cd x, cd y, double& c, cd& s) {
  const double ax = std::abs(x), ay = std::abs(y);
  if (ay == 0.0) { c = 1.0; s = 0.0; return; }
  if (ax == 0.0) { c = 0.0; s = 1.0; return; }
  const double r = std::hypot(ax, ay);
  c = ax / r;
  s = (x / ax) * std::conj(y) / r;
}
}  // namespace

int Schur::compute(int m_, const cd* H, int ldh) {
  m = m_;
  T.assign((size_t)m * m, cd(0.0));
  rots.clear();
  for (int j = 0; j < m; ++j)
    for (int i = 0; i <= std::min(j + 1, m - 1); ++i) T[(size_t)j * m + i] = H[(size_t)j * ldh + i];
  auto at = [&](int i, int j) -> cd& { return T[(size_t)j * m + i]; };
  double hnorm = 0.0;
  for (const cd& v : T) hnorm = std::max(hnorm, std::abs(v));
  if (hnorm == 0.0) hnorm = 1.0;

  int hi = m - 1;
  int its = 0;
  while (hi > 0) {
    // active block [l, hi]: the last negligible subdiagonal entry above hi
    int l = hi;
    for (; l > 0; --l) {
      double s = std::abs(at(l, l)) + std::abs(at(l - 1, l - 1));
      if (s == 0.0) s = hnorm;
      if (std::abs(at(l, l - 1)) <= kEps * s) {
        at(l, l - 1) = 0.0;
        break;
      }
    }
    if (l == hi) {  // 1x1 block converged
      --hi;
      its = 0;
      continue;
    }
    if (++its > 100) return DENSE_NOCONV;
    cd mu;
    if (its % 12 == 11) {  // exceptional shift against cycling
      mu = at(hi, hi) + 0.75 * std::abs(at(hi, hi - 1));
    } else {  // Wilkinson shift: eigenvalue of the trailing 2x2 closer to T(hi, hi)
      const cd a = at(hi - 1, hi - 1), b = at(hi - 1, hi), c = at(hi, hi - 1), d = at(hi, hi);
      const cd half = 0.5 * (a + d);
      const cd disc = std::sqrt(0.25 * (a - d) * (a - d) + b * c);
      const cd m1 = half + disc, m2 = half - disc;
      mu = (std::abs(m1 - d) < std::abs(m2 - d)) ? m1 : m2;
    }
    // implicit single-shift sweep: the first rotation comes from the shifted
    // first column, the others chase the bulge down the subdiagonal
    cd x = at(l, l) - mu, y = at(l + 1, l);
    for (int k = l; k < hi; ++k) {
      double c;
      cd s;
      givens(x, y, c, s);
      const int c0 = (k == l) ? l : k - 1;
      for (int col = c0; col < m; ++col) {  // rows k, k+1 from the left
        const cd a = at(k, col), b = at(k + 1, col);
        at(k, col) = c * a + s * b;
        at(k + 1, col) = -std::conj(s) * a + c * b;
      }
      const int r1 = std::min(k + 2, hi);
      cd* ck = &T[(size_t)k * m];
      cd* ck1 = &T[(size_t)(k + 1) * m];
      const cd sc = std::conj(s);
      for (int row = 0; row <= r1; ++row) {  // columns k, k+1 from the right
        const cd a = ck[row], b = ck1[row];
        ck[row] = a * c + b * sc;
        ck1[row] = -a * s + b * c;
      }
      rots.push_back({k, c, s});
      if (k < hi - 1) {
        x = at(k + 1, k);
        y = at(k + 2, k);
      }
    }
  }
  for (int j = 0; j < m; ++j)
    for (int i = j + 1; i < m; ++i) at(i, j) = 0.0;
  return DENSE_OK;
}

void Schur::apply_QH(cd* v) const {
  // H = Q T Q^H with Q = G_1^H G_2^H ... G_N^H, so Q^H v = G_N ... G_1 v
  for (const Rot& r : rots) {
    const cd a = v[r.k], b = v[r.k + 1];
    v[r.k] = r.c * a + r.s * b;
    v[r.k + 1] = -std::conj(r.s) * a + r.c * b;
  }
}

void Schur::apply_Q(cd* v) const {
  for (auto it = rots.rbegin(); it != rots.rend(); ++it) {
    const cd a = v[it->k], b = v[it->k + 1];
    v[it->k] = it->c * a - it->s * b;
    v[it->k + 1] = std::conj(it->s) * a + it->c * b;
  }
}

int hess_eigenvalues(int m, const cd* H, int ldh, cd* ev) {
  Schur S;
  const int st = S.compute(m, H, ldh);
  if (st != DENSE_OK) return st;
  for (int i = 0; i < m; ++i) ev[i] = S.t(i, i);
  return DENSE_OK;
}

// principal square root of a complex upper triangular T (Bjorck-Hammarling)
// applied as z = Q R^{-1} Q^H (beta e_1); shared by both Schur variants
template <typename S>
static int triangular_invsqrt_e1(const S& sch, int m, double beta, cd* z) {
  double scale = 1.0;
  for (int i = 0; i < m; ++i) scale = std::max(scale, std::abs(sch.t(i, i)));
  for (int i = 0; i < m; ++i) {
    const cd t = sch.t(i, i);
    if (t.real() <= 0.0 && std::fabs(t.imag()) <= 1e-12 * scale) return DENSE_BRANCH;
  }
  std::vector<cd> R((size_t)m * m, cd(0.0));
  auto r = [&](int i, int j) -> cd& { return R[(size_t)j * m + i]; };
  for (int j = 0; j < m; ++j) {
    r(j, j) = std::sqrt(sch.t(j, j));
    for (int i = j - 1; i >= 0; --i) {
      cd s = sch.t(i, j);
      for (int k = i + 1; k < j; ++k) s -= r(i, k) * r(k, j);
      r(i, j) = s / (r(i, i) + r(j, j));
    }
  }
  std::vector<cd> u(m, cd(0.0));
  u[0] = beta;
  sch.apply_QH(u.data());
  for (int i = m - 1; i >= 0; --i) {
    cd s = u[i];
    for (int k = i + 1; k < m; ++k) s -= r(i, k) * u[k];
    u[i] = s / r(i, i);
  }
  sch.apply_Q(u.data());
  for (int i = 0; i < m; ++i) z[i] = u[i];
  return DENSE_OK;
}

int lu_solve(int m, cd* A, cd* x) {
  auto a = [&](int i, int j) -> cd& { return A[(size_t)j * m + i]; };
  for (int k = 0; k < m; ++k) {
    int p = k;
    for (int i = k + 1; i < m; ++i)
      if (std::abs(a(i, k)) > std::abs(a(p, k))) p = i;
    if (a(p, k) == cd(0.0)) return DENSE_NOCONV;
    if (p != k) {
      for (int j = 0; j < m; ++j) std::swap(a(k, j), a(p, j));
      std::swap(x[k], x[p]);
    }
    for (int i = k + 1; i < m; ++i) {
      const cd l = a(i, k) / a(k, k);
      a(i, k) = l;
      for (int j = k + 1; j < m; ++j) a(i, j) -= l * a(k, j);
      x[i] -= l * x[k];
    }
  }
  for (int k = m - 1; k >= 0; --k) {
    cd t = x[k];
    for (int j = k + 1; j < m; ++j) t -= a(k, j) * x[j];
    x[k] = t / a(k, k);
  }
  return DENSE_OK;
}

int hess_invsqrt_e1(int m, const cd* H, int ldh, double beta, cd* z) {
  Schur S;
  const int st = S.compute(m, H, ldh);
  if (st != DENSE_OK) return st;
  return triangular_invsqrt_e1(S, m, beta, z);
}

// ---- real Francis double-shift QR ----------------------------------------
namespace {
// Householder reflector I - tau v v^T (v[0] = 1) with (I - tau v v^T) x = (beta, 0, ...)
inline void house(int len, const double* x, double* v, double& tau) {
  double sig = 0.0;
  for (int i = 1; i < len; ++i) sig += x[i] * x[i];
  v[0] = 1.0;
  for (int i = 1; i < len; ++i) v[i] = x[i];
  if (sig == 0.0) {
    tau = 0.0;
    return;
  }
  const double mu = std::sqrt(x[0] * x[0] + sig);
  const double v0 = (x[0] <= 0.0) ? x[0] - mu : -sig / (x[0] + mu);
  tau = 2.0 * v0 * v0 / (sig + v0 * v0);
  for (int i = 1; i < len; ++i) v[i] /= v0;
}
}  // namespace

int RealSchur::compute(int m_, const double* H, int ldh) {
  m = m_;
  Tr.assign((size_t)m * m, 0.0);
  refl.clear();
  rot.clear();
  for (int j = 0; j < m; ++j)
    for (int i = 0; i <= std::min(j + 1, m - 1); ++i) Tr[(size_t)j * m + i] = H[(size_t)j * ldh + i];
  auto a = [&](int i, int j) -> double& { return Tr[(size_t)j * m + i]; };
  double hnorm = 0.0;
  for (double v : Tr) hnorm = std::max(hnorm, std::fabs(v));
  if (hnorm == 0.0) hnorm = 1.0;

  auto reflect = [&](int k, int len, const double* v, double tau, int ilo, int ihi) {
    // left: rows k..k+len-1, columns from max(ilo, k-1) to m-1
    for (int c = std::max(ilo, k - 1); c < m; ++c) {
      double sdot = 0.0;
      for (int r = 0; r < len; ++r) sdot += v[r] * a(k + r, c);
      sdot *= tau;
      for (int r = 0; r < len; ++r) a(k + r, c) -= sdot * v[r];
    }
    // right: columns k..k+len-1, rows 0..min(k+len, ihi)
    const int rmax = std::min(k + len, ihi);
    for (int r = 0; r <= rmax; ++r) {
      double sdot = 0.0;
      for (int c = 0; c < len; ++c) sdot += a(r, k + c) * v[c];
      sdot *= tau;
      for (int c = 0; c < len; ++c) a(r, k + c) -= sdot * v[c];
    }
    Refl R;
    R.k = k;
    R.len = len;
    R.tau = tau;
    for (int i = 0; i < 3; ++i) R.v[i] = (i < len) ? v[i] : 0.0;
    refl.push_back(R);
  };

  int hi = m - 1, its = 0, total = 0;
  while (hi >= 0) {
    int l = hi;
    for (; l > 0; --l) {
      double sc = std::fabs(a(l, l)) + std::fabs(a(l - 1, l - 1));
      if (sc == 0.0) sc = hnorm;
      if (std::fabs(a(l, l - 1)) <= kEps * sc) {
        a(l, l - 1) = 0.0;
        break;
      }
    }
    if (l >= hi - 1) {  // a 1x1 or 2x2 block has split off
      hi = l - 1;
      its = 0;
      continue;
    }
    if (++its > 100 || ++total > 100 * m) return DENSE_NOCONV;
    // double shift: the eigenvalues of the trailing 2x2 block (sum s, product t)
    double sh, th;
    if (its % 11 == 10) {  // exceptional shift
      const double w = std::fabs(a(hi, hi - 1)) + std::fabs(a(hi - 1, hi - 2));
      sh = 1.5 * w + a(hi, hi);
      th = w * w;
    } else {
      sh = a(hi - 1, hi - 1) + a(hi, hi);
      th = a(hi - 1, hi - 1) * a(hi, hi) - a(hi - 1, hi) * a(hi, hi - 1);
    }
    // first column of (H - mu1)(H - mu2) restricted to rows l..l+2
    double x[3];
    x[0] = a(l, l) * a(l, l) + a(l, l + 1) * a(l + 1, l) - sh * a(l, l) + th;
    x[1] = a(l + 1, l) * (a(l, l) + a(l + 1, l + 1) - sh);
    x[2] = a(l + 1, l) * a(l + 2, l + 1);
    for (int k = l; k <= hi - 2; ++k) {
      double v[3], tau;
      house(3, x, v, tau);
      if (tau != 0.0) reflect(k, 3, v, tau, l, hi);
      x[0] = a(k + 1, k);
      x[1] = a(k + 2, k);
      if (k < hi - 2) x[2] = a(k + 3, k);
      if (k > l) {  // the reflector annihilated the bulge in column k - 1
        a(k + 1, k - 1) = 0.0;
        a(k + 2, k - 1) = 0.0;
      }
    }
    {
      double v[3], tau;
      house(2, x, v, tau);
      if (tau != 0.0) reflect(hi - 1, 2, v, tau, l, hi);
      if (hi - 2 >= l) a(hi, hi - 2) = 0.0;
    }
  }
  // complex triangular T: triangularize each remaining 2x2 diagonal block
  T.assign((size_t)m * m, cd(0.0));
  for (int j = 0; j < m; ++j)
    for (int i = 0; i <= std::min(j + 1, m - 1); ++i) T[(size_t)j * m + i] = a(i, j);
  auto t_ = [&](int i, int j) -> cd& { return T[(size_t)j * m + i]; };
  for (int i = 0; i + 1 < m; ++i) {
    if (t_(i + 1, i) == 0.0) continue;
    const cd A = t_(i, i), B = t_(i, i + 1), Cc = t_(i + 1, i), D = t_(i + 1, i + 1);
    const cd half = 0.5 * (A + D);
    const cd disc = std::sqrt(0.25 * (A - D) * (A - D) + B * Cc);
    // eigenvector (lam - D, C) of the block for the eigenvalue farther from D
    // (the nearer one makes lam - D a cancellation when C is small)
    const cd l1 = half + disc, l2 = half - disc;
    const cd lam = (std::abs(l1 - D) >= std::abs(l2 - D)) ? l1 : l2;
    // normalized, it is the first column of G
    cd g1 = lam - D, g2 = Cc;
    const double nr = std::sqrt(std::norm(g1) + std::norm(g2));
    g1 /= nr;
    g2 /= nr;
    // T <- G^H T G on rows / columns i, i+1;  G = [[g1, -conj g2], [g2, conj g1]]
    for (int c = i; c < m; ++c) {
      const cd r0 = t_(i, c), r1 = t_(i + 1, c);
      t_(i, c) = std::conj(g1) * r0 + std::conj(g2) * r1;
      t_(i + 1, c) = -g2 * r0 + g1 * r1;
    }
    for (int r = 0; r <= i + 1; ++r) {
      const cd c0 = t_(r, i), c1 = t_(r, i + 1);
      t_(r, i) = c0 * g1 + c1 * g2;
      t_(r, i + 1) = -c0 * std::conj(g2) + c1 * std::conj(g1);
    }
    t_(i + 1, i) = 0.0;
    rot.push_back({i, g1, g2});
    ++i;  // the next block starts after this one
  }
  return DENSE_OK;
}

void RealSchur::apply_QH(cd* v) const {
  // H = (P_1 ... P_N G_1 ... G_R) T (...)^H with symmetric reflectors P
  for (const Refl& r : refl) {
    cd sdot = 0.0;
    for (int i = 0; i < r.len; ++i) sdot += r.v[i] * v[r.k + i];
    sdot *= r.tau;
    for (int i = 0; i < r.len; ++i) v[r.k + i] -= sdot * r.v[i];
  }
  for (const Rot2& g : rot) {
    const cd a0 = v[g.k], a1 = v[g.k + 1];
    v[g.k] = std::conj(g.g1) * a0 + std::conj(g.g2) * a1;
    v[g.k + 1] = -g.g2 * a0 + g.g1 * a1;
  }
}

void RealSchur::apply_Q(cd* v) const {
  for (auto it = rot.rbegin(); it != rot.rend(); ++it) {
    const cd a0 = v[it->k], a1 = v[it->k + 1];
    v[it->k] = it->g1 * a0 - std::conj(it->g2) * a1;
    v[it->k + 1] = it->g2 * a0 + std::conj(it->g1) * a1;
  }
  for (auto it = refl.rbegin(); it != refl.rend(); ++it) {
    cd sdot = 0.0;
    for (int i = 0; i < it->len; ++i) sdot += it->v[i] * v[it->k + i];
    sdot *= it->tau;
    for (int i = 0; i < it->len; ++i) v[it->k + i] -= sdot * it->v[i];
  }
}

int real_hess_invsqrt_e1(int m, const double* H, int ldh, double beta, cd* z) {
  RealSchur S;
  const int st = S.compute(m, H, ldh);
  if (st != DENSE_OK) return st;
  return triangular_invsqrt_e1(S, m, beta, z);
}

int tridiag_invsqrt_e1(int m, const double* alpha, const double* offd, double beta,
                       double* z) {
  // Symmetric QR algorithm: T = Q diag(d) Q^T by implicit single-shift QR
  // sweeps with the Wilkinson shift on the bottom unreduced block (Golub and
  // Van Loan, Matrix Computations, Sec. 8.3).  A sweep on rows lo..hi is a
  // chain of plane rotations P_k (rows k, k+1): the first is chosen from the
  // shifted first column (d_lo - mu, e_lo), each later one annihilates the
  // bulge T(k-1, k+1) the previous one created; T <- P_k T P_k^T, and
  // Q = P_1^T P_2^T ... P_N^T.  Only Q^T e_1 and one product Q w are needed,
  // so the rotations are recorded and applied to those two vectors (O(m^2)
  // work instead of O(m^3) for Q itself).
  struct Rot {
    int k;
    double c, s;
  };
  std::vector<double> d(alpha, alpha + m), e(std::max(m - 1, 1), 0.0);
  for (int i = 0; i + 1 < m; ++i) e[i] = offd[i];
  std::vector<Rot> rot;
  // about m^2 rotations in all (two sweeps per eigenvalue, each over about
  // half of T); the record grows beyond this if it has to
  rot.reserve(std::min<size_t>((size_t)m * m + 64, (size_t)1 << 20));
  int hi = m - 1;
  long sweeps = 0;
  while (hi > 0) {
    // negligible couplings split T into independent blocks
    for (int i = 0; i < hi; ++i)
      if (std::fabs(e[i]) <= kEps * (std::fabs(d[i]) + std::fabs(d[i + 1]))) e[i] = 0.0;
    if (e[hi - 1] == 0.0) {  // d[hi] is an eigenvalue
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && e[lo - 1] != 0.0) --lo;
    if (++sweeps > 40L * m) return DENSE_NOCONV;
    // Wilkinson shift: the eigenvalue of the trailing 2 x 2 block nearer d[hi]
    const double t = 0.5 * (d[hi - 1] - d[hi]), eh = e[hi - 1];
    // (sqrt of sums of squares: the entries are far from overflow here)
    const double mu = d[hi] - eh * eh / (t + (t >= 0.0 ? 1.0 : -1.0) * std::sqrt(t * t + eh * eh));
    double x = d[lo] - mu, y = e[lo];  // the vector the next rotation acts on
    for (int k = lo; k < hi; ++k) {
      const double r = std::sqrt(x * x + y * y);
      const double ir = r == 0.0 ? 0.0 : 1.0 / r;  // one division per rotation
      const double c = r == 0.0 ? 1.0 : x * ir, s = y * ir;
      if (k > lo) e[k - 1] = r;  // the bulge T(k-1, k+1) is now zero
      // the 2 x 2 block on rows and columns k, k+1
      const double a = d[k], bb = d[k + 1], f = e[k];
      const double cs = c * s, cc = c * c, ss = s * s;
      d[k] = cc * a + 2.0 * cs * f + ss * bb;
      d[k + 1] = ss * a - 2.0 * cs * f + cc * bb;
      e[k] = cs * (bb - a) + (cc - ss) * f;
      rot.push_back({k, c, s});
      if (k + 1 < hi) {  // the coupling to row k + 2 moves the bulge down
        x = e[k];
        y = s * e[k + 1];
        e[k + 1] *= c;
      }
    }
  }
  for (int k = 0; k < m; ++k)
    if (!(d[k] > 0.0)) return DENSE_BRANCH;
  // u = Q^T e_1 = P_N ... P_1 e_1
  std::vector<double> u(m, 0.0);
  u[0] = 1.0;
  for (const Rot& g : rot) {
    const double p = u[g.k], q = u[g.k + 1];
    u[g.k] = g.c * p + g.s * q;
    u[g.k + 1] = g.c * q - g.s * p;
  }
  // z = Q diag(d)^{-1/2} (beta u) = P_1^T ... P_N^T w
  for (int k = 0; k < m; ++k) z[k] = u[k] * beta / std::sqrt(d[k]);
  for (auto it = rot.rbegin(); it != rot.rend(); ++it) {
    const double p = z[it->k], q = z[it->k + 1];
    z[it->k] = it->c * p - it->s * q;
    z[it->k + 1] = it->s * p + it->c * q;
  }
  return DENSE_OK;
}

void cheb_coefficients(double a, double b, int K, double* c) {
  // c_i = (2/d) sum_k f(x_k) cos(i t_k), t_k = pi (k + 1/2)/d, x_k on [a, b];
  // c_0 halved: the d-point Gauss-Chebyshev rule for the projection integral
  const int d = K + 1;
  std::vector<double> t(d), fx(d);
  for (int k = 0; k < d; ++k) {
    t[k] = M_PI * (k + 0.5) / d;
    const double x = 0.5 * (a + b) + 0.5 * (b - a) * std::cos(t[k]);
    fx[k] = 1.0 / std::sqrt(x);
  }
  for (int i = 0; i < d; ++i) {
    double s = 0.0;
    for (int k = 0; k < d; ++k) s += fx[k] * std::cos(i * t[k]);
    c[i] = 2.0 / d * s;
  }
  c[0] *= 0.5;
}

double cheb_eval(const double* c, int K, double a, double b, double z) {
  const double zh = (2.0 * z - (a + b)) / (b - a);
  double b1 = 0.0, b2 = 0.0;
  for (int k = K; k >= 1; --k) {
    const double t = c[k] + 2.0 * zh * b1 - b2;
    b2 = b1;
    b1 = t;
  }
  return c[0] + zh * b1 - b2;
}

std::vector<cd> leja_order(const std::vector<cd>& nodes, bool pair_conjugates) {
  std::vector<cd> rest(nodes), out;
  if (rest.empty()) return out;
  auto take = [&](size_t i) {
    out.push_back(rest[i]);
    rest.erase(rest.begin() + (long)i);
  };
  auto take_partner = [&]() {
    const cd z = out.back();
    if (!pair_conjugates || z.imag() == 0.0 || rest.empty()) return;
    size_t best = 0;
    for (size_t i = 1; i < rest.size(); ++i)
      if (std::abs(rest[i] - std::conj(z)) < std::abs(rest[best] - std::conj(z))) best = i;
    if (std::abs(rest[best] - std::conj(z)) <= 1e-10 * std::max(1.0, std::abs(z))) take(best);
  };
  // first: largest modulus, ties to larger real part, then Im >= 0
  size_t first = 0;
  for (size_t i = 1; i < rest.size(); ++i) {
    const cd a = rest[i], b = rest[first];
    if (std::abs(a) > std::abs(b) ||
        (std::abs(a) == std::abs(b) &&
         (a.real() > b.real() || (a.real() == b.real() && a.imag() >= 0 && b.imag() < 0))))
      first = i;
  }
  take(first);
  take_partner();
  while (!rest.empty()) {
    size_t best = 0;
    double best_score = -std::numeric_limits<double>::infinity();
    bool best_up = false;
    for (size_t i = 0; i < rest.size(); ++i) {
      double sc = 0.0;
      for (const cd& s : out) {
        const double dd = std::abs(rest[i] - s);
        sc += (dd > 0.0) ? std::log(dd) : -std::numeric_limits<double>::infinity();
      }
      const bool up = rest[i].imag() >= 0.0;
      if (sc > best_score || (sc == best_score && up && !best_up)) {
        best = i;
        best_score = sc;
        best_up = up;
      }
    }
    take(best);
    take_partner();
  }
  return out;
}

double leja_capacity(const std::vector<cd>& t) {
  const size_t d = t.size();
  if (d < 2) return 1.0;
  double s = 0.0;
  for (size_t i = 0; i + 1 < d; ++i) s += std::log(std::abs(t[d - 1] - t[i]));
  return std::exp(s / double(d - 1));
}

std::vector<cd> newton_invsqrt(const std::vector<cd>& t, double rho) {
  const size_t d = t.size();
  std::vector<cd> dd(d);
  for (size_t i = 0; i < d; ++i) dd[i] = 1.0 / std::sqrt(t[i]);
  for (size_t j = 1; j < d; ++j)
    for (size_t i = d - 1; i >= j; --i) dd[i] = (dd[i] - dd[i - 1]) / ((t[i] - t[i - j]) / rho);
  return dd;
}

}  // namespace fa
