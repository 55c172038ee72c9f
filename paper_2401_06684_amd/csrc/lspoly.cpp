// Least-squares preconditioning polynomial on a contour (Sec. 5.3), host FP64.
//
// The contour is the boundary of the convex hull of the Ritz values with the
// part closer to 0 than r_min cut away by the circle |z| = r_min (so the
// region is hull minus the open disk), discretized at equal arc length with
// spacing at most `step` (the choices of Sec. 6, Example 3).  For a real
// operator the point set is made conjugate-symmetric by adding the mirror
// images, which keeps the fitted polynomial real.
//
// The fit runs Arnoldi on diag(z_1..z_N) from the constant vector N^{-1/2}:
// its vectors are the values of the orthonormal polynomials p_0..p_{d-1} of
// the discrete inner product, its Hessenberg matrix the (full) recurrence
// that generates them, and alpha_j = <z^{-1/2}, p_j> gives the best
// approximation q = sum_j alpha_j p_j.
#include <algorithm>
#include <cmath>

#include "dense.hpp"

namespace fa {

std::vector<cd> convex_hull(const std::vector<cd>& pts_in) {
  std::vector<cd> p(pts_in);
  std::sort(p.begin(), p.end(), [](const cd& a, const cd& b) {
    return a.real() < b.real() || (a.real() == b.real() && a.imag() < b.imag());
  });
  p.erase(std::unique(p.begin(), p.end()), p.end());
  if (p.size() <= 2) return p;
  auto cross = [](const cd& o, const cd& a, const cd& b) {
    return (a.real() - o.real()) * (b.imag() - o.imag()) -
           (a.imag() - o.imag()) * (b.real() - o.real());
  };
  std::vector<cd> h(2 * p.size());
  size_t k = 0;
  for (size_t i = 0; i < p.size(); ++i) {  // lower chain
    while (k >= 2 && cross(h[k - 2], h[k - 1], p[i]) <= 0) --k;
    h[k++] = p[i];
  }
  for (size_t i = p.size() - 1, t = k + 1; i-- > 0;) {  // upper chain
    while (k >= t && cross(h[k - 2], h[k - 1], p[i]) <= 0) --k;
    h[k++] = p[i];
  }
  h.resize(k - 1);  // the last point repeats the first
  return h;
}

int ls_contour(const std::vector<cd>& theta, double r_min, double step, bool symmetric,
               std::vector<cd>& out) {
  out.clear();
  const std::vector<cd> hull = convex_hull(theta);
  if (hull.size() < 2 || !(step > 0.0) || !(r_min >= 0.0)) return DENSE_NOCONV;
  for (const cd& v : hull)
    if (!(v.real() > 0.0)) return DENSE_BRANCH;
  // walk the hull counter-clockwise, keep the parts of the edges outside the
  // disk, and bridge each excursion into the disk by an arc
  struct Piece {
    bool arc;
    cd a, b;        // segment end points / arc entry and exit points
    double a0, da;  // arc: start angle and (signed) angle span
    double len;
  };
  std::vector<Piece> pcs;
  bool inside = false;
  cd entry;
  const size_t nv = hull.size();
  for (size_t i = 0; i < nv; ++i) {
    const cd p = hull[i], d = hull[(i + 1) % nv] - p;
    // |p + t d|^2 = r^2
    const double A2 = std::norm(d), B2 = 2.0 * (std::conj(p) * d).real(),
                 C2 = std::norm(p) - r_min * r_min;
    double cuts[4] = {0.0, 1.0, 0.0, 0.0};
    int nc = 2;
    const double disc = B2 * B2 - 4.0 * A2 * C2;
    if (disc > 0.0) {
      const double sq = std::sqrt(disc);
      const double t1 = (-B2 - sq) / (2.0 * A2), t2 = (-B2 + sq) / (2.0 * A2);
      if (t1 > 0.0 && t1 < 1.0) cuts[nc++] = t1;
      if (t2 > 0.0 && t2 < 1.0) cuts[nc++] = t2;
    }
    std::sort(cuts, cuts + nc);
    for (int c = 0; c + 1 < nc; ++c) {
      const cd a = p + cuts[c] * d, b = p + cuts[c + 1] * d;
      const cd mid = p + 0.5 * (cuts[c] + cuts[c + 1]) * d;
      if (std::abs(mid) >= r_min) {
        if (inside) {
          pcs.push_back({true, entry, a, 0.0, 0.0, 0.0});
          inside = false;
        }
        pcs.push_back({false, a, b, 0.0, 0.0, std::abs(b - a)});
      } else if (!inside) {
        inside = true;
        entry = a;
      }
    }
  }
  size_t first_seg = pcs.size();
  for (size_t i = 0; i < pcs.size(); ++i)
    if (!pcs[i].arc) {
      first_seg = i;
      break;
    }
  if (first_seg == pcs.size()) return DENSE_NOCONV;  // the hull lies within r_min of 0
  if (inside) pcs.push_back({true, entry, pcs[first_seg].a, 0.0, 0.0, 0.0});
  // arcs run clockwise about 0 (the region, outside the disk, on the left)
  const double two_pi = 2.0 * M_PI;
  for (Piece& pc : pcs) {
    if (!pc.arc) continue;
    const double a0 = std::atan2(pc.a.imag(), pc.a.real());
    const double a1 = std::atan2(pc.b.imag(), pc.b.real());
    double span = std::fmod(a0 - a1, two_pi);
    if (span < 0.0) span += two_pi;
    if (span > M_PI) span = 0.0;  // a zero-length arc, up to rounding
    pc.a0 = a0;
    pc.da = -span;
    pc.len = r_min * span;
  }
  double total = 0.0;
  for (const Piece& pc : pcs) total += pc.len;
  const long N = std::max(2L, (long)std::ceil(total / step));
  const double h = total / (double)N;
  out.reserve(symmetric ? 2 * N : N);
  double s0 = 0.0;
  long k = 0;
  for (const Piece& pc : pcs) {
    for (; k < N && (double)k * h < s0 + pc.len; ++k) {
      const double t = pc.len > 0.0 ? ((double)k * h - s0) / pc.len : 0.0;
      if (pc.arc) {
        const double ang = pc.a0 + t * pc.da;
        out.push_back(cd(r_min * std::cos(ang), r_min * std::sin(ang)));
      } else {
        out.push_back(pc.a + t * (pc.b - pc.a));
      }
    }
    s0 += pc.len;
  }
  if (symmetric) {
    const size_t m = out.size();
    for (size_t i = 0; i < m; ++i) out.push_back(std::conj(out[i]));
  }
  return DENSE_OK;
}

int ls_fit_invsqrt(const std::vector<cd>& z, int degree, bool real_op, std::vector<cd>& hls,
                   std::vector<cd>& alpha) {
  const size_t N = z.size();
  const int d = degree + 1;
  if ((size_t)d > N || degree < 1) return DENSE_NOCONV;
  // P (N x d) column-major: the values of p_0..p_{d-1} at the points
  std::vector<cd> P(N * (size_t)d);
  hls.assign((size_t)d * (d - 1), cd(0.0));
  auto col = [&](int j) { return P.data() + (size_t)j * N; };
  const double p0 = 1.0 / std::sqrt((double)N);
  for (size_t i = 0; i < N; ++i) col(0)[i] = p0;
  std::vector<cd> w(N), g(d);
  for (int j = 0; j + 1 < d; ++j) {
    for (size_t i = 0; i < N; ++i) w[i] = z[i] * col(j)[i];
    std::vector<cd> hj(j + 1, cd(0.0));
    for (int pass = 0; pass < 2; ++pass) {  // classical Gram-Schmidt, twice
      for (int c = 0; c <= j; ++c) {
        cd s = 0.0;
        const cd* pc = col(c);
        for (size_t i = 0; i < N; ++i) s += std::conj(pc[i]) * w[i];
        g[c] = s;
      }
      for (int c = 0; c <= j; ++c) {
        const cd* pc = col(c);
        for (size_t i = 0; i < N; ++i) w[i] -= g[c] * pc[i];
        hj[c] += g[c];
      }
    }
    double nn = 0.0;
    for (size_t i = 0; i < N; ++i) nn += std::norm(w[i]);
    nn = std::sqrt(nn);
    if (!(nn > 0.0)) return DENSE_NOCONV;
    for (int c = 0; c <= j; ++c) hls[(size_t)j * d + c] = hj[c];
    hls[(size_t)j * d + j + 1] = nn;
    cd* pn = col(j + 1);
    for (size_t i = 0; i < N; ++i) pn[i] = w[i] / nn;
  }
  alpha.assign(d, cd(0.0));
  for (int j = 0; j < d; ++j) {
    cd s = 0.0;
    const cd* pc = col(j);
    for (size_t i = 0; i < N; ++i) s += std::conj(pc[i]) / std::sqrt(z[i]);
    alpha[j] = s;
  }
  // Re q(z_i) > 0 at every contour point (Sec. 5.3)
  for (size_t i = 0; i < N; ++i) {
    cd q = 0.0;
    for (int j = 0; j < d; ++j) q += alpha[j] * col(j)[i];
    if (!(q.real() > 0.0)) return DENSE_BRANCH;
  }
  if (real_op) {  // a conjugate-symmetric point set: real up to rounding
    double scale = 0.0, im = 0.0;
    for (const cd& v : hls) scale = std::max(scale, std::abs(v)), im = std::max(im, std::fabs(v.imag()));
    for (const cd& v : alpha) scale = std::max(scale, std::abs(v)), im = std::max(im, std::fabs(v.imag()));
    if (im > 1e-10 * scale) return DENSE_NOCONV;
    for (cd& v : hls) v = cd(v.real(), 0.0);
    for (cd& v : alpha) v = cd(v.real(), 0.0);
  }
  return DENSE_OK;
}

}  // namespace fa
