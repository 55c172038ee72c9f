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

int hess_invsqrt_e1(int m, const cd* H, int ldh, double beta, cd* z) {
  Schur S;
  const int st = S.compute(m, H, ldh);
  if (st != DENSE_OK) return st;
  double scale = 1.0;
  for (int i = 0; i < m; ++i) scale = std::max(scale, std::abs(S.t(i, i)));
  for (int i = 0; i < m; ++i) {
    const cd t = S.t(i, i);
    if (t.real() <= 0.0 && std::fabs(t.imag()) <= 1e-12 * scale) return DENSE_BRANCH;
  }
  // R = T^{1/2}: principal roots on the diagonal, then column by column
  // R_ij (R_ii + R_jj) = T_ij - sum_{i<k<j} R_ik R_kj (Bjorck-Hammarling)
  std::vector<cd> R((size_t)m * m, cd(0.0));
  auto r = [&](int i, int j) -> cd& { return R[(size_t)j * m + i]; };
  for (int j = 0; j < m; ++j) {
    r(j, j) = std::sqrt(S.t(j, j));
    for (int i = j - 1; i >= 0; --i) {
      cd s = S.t(i, j);
      for (int k = i + 1; k < j; ++k) s -= r(i, k) * r(k, j);
      r(i, j) = s / (r(i, i) + r(j, j));
    }
  }
  std::vector<cd> u(m, cd(0.0));
  u[0] = beta;
  S.apply_QH(u.data());
  for (int i = m - 1; i >= 0; --i) {  // R y = u
    cd s = u[i];
    for (int k = i + 1; k < m; ++k) s -= r(i, k) * u[k];
    u[i] = s / r(i, i);
  }
  S.apply_Q(u.data());
  for (int i = 0; i < m; ++i) z[i] = u[i];
  return DENSE_OK;
}

int tridiag_invsqrt_e1(int m, const double* alpha, const double* offd, double beta,
                       double* z) {
  // eigendecomposition T = Z diag(d) Z^T by implicit QL iterations with
  // Wilkinson shifts, accumulating the rotations into Z
  std::vector<double> d(alpha, alpha + m), e(m, 0.0), Z((size_t)m * m, 0.0);
  for (int i = 0; i + 1 < m; ++i) e[i] = offd[i];
  for (int i = 0; i < m; ++i) Z[(size_t)i * m + i] = 1.0;
  auto zz = [&](int i, int j) -> double& { return Z[(size_t)j * m + i]; };
  for (int l = 0; l < m; ++l) {
    int its = 0;
    while (true) {
      int mm = l;
      for (; mm < m - 1; ++mm) {
        const double dd = std::fabs(d[mm]) + std::fabs(d[mm + 1]);
        if (std::fabs(e[mm]) <= kEps * dd) break;
      }
      if (mm == l) break;
      if (++its > 100) return DENSE_NOCONV;
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[mm] - d[l] + e[l] / (g + std::copysign(r, g));
      double s = 1.0, c = 1.0, p = 0.0;
      int i = mm - 1;
      bool early = false;
      for (; i >= l; --i) {
        const double f = s * e[i], b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= p;
          e[mm] = 0.0;
          early = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        for (int k = 0; k < m; ++k) {
          const double t = zz(k, i + 1);
          zz(k, i + 1) = s * zz(k, i) + c * t;
          zz(k, i) = c * zz(k, i) - s * t;
        }
      }
      if (early) continue;
      d[l] -= p;
      e[l] = g;
      e[mm] = 0.0;
    }
  }
  for (int k = 0; k < m; ++k)
    if (!(d[k] > 0.0)) return DENSE_BRANCH;
  std::vector<double> w(m);
  for (int k = 0; k < m; ++k) w[k] = zz(0, k) * beta / std::sqrt(d[k]);
  for (int i = 0; i < m; ++i) {
    double s = 0.0;
    for (int k = 0; k < m; ++k) s += zz(i, k) * w[k];
    z[i] = s;
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
