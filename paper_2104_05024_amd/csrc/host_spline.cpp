// Closed 2D curves given by their nodes: the periodic cubic spline through them (Sec. 7, the
// 2D set-up represents the boundary by quasi-uniform nodes and periodic cubic splines), with
// the derivatives, normals, curvature and grid-line crossings the setup reads off it.
#include <algorithm>
#include <cmath>

#include "host_tables.h"

namespace kfbi {

void SplineCurve2::build(const double *pts, int64_t m_, int orient_) {
  m = m_;
  orient = orient_;
  // second derivatives M_j of the C2 periodic interpolant with unit knot spacing:
  // M_{j-1} + 4 M_j + M_{j+1} = 6 (P_{j+1} - 2 P_j + P_{j-1}), a cyclic tridiagonal system,
  // solved as a tridiagonal one plus a rank-one correction (Sherman-Morrison)
  const int64_t n = m;
  auto tridiag = [n](const std::vector<double> &diag, std::vector<double> r) {
    // sub- and super-diagonal entries are 1
    std::vector<double> cp(n), x(n);
    double b = diag[0];
    cp[0] = 1.0 / b;
    r[0] /= b;
    for (int64_t i = 1; i < n; ++i) {
      b = diag[i] - cp[i - 1];
      cp[i] = 1.0 / b;
      r[i] = (r[i] - r[i - 1]) / b;
    }
    x[n - 1] = r[n - 1];
    for (int64_t i = n - 2; i >= 0; --i) x[i] = r[i] - cp[i] * x[i + 1];
    return x;
  };
  const double gamma = -4.0;
  std::vector<double> diag(n, 4.0);
  diag[0] = 4.0 - gamma;
  diag[n - 1] = 4.0 - 1.0 / gamma;
  std::vector<double> u(n, 0.0);
  u[0] = gamma;
  u[n - 1] = 1.0;
  const std::vector<double> z = tridiag(diag, u);
  double area = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    const int64_t k = (j + 1) % n;
    area += pts[2 * j] * pts[2 * k + 1] - pts[2 * k] * pts[2 * j + 1];
  }
  sigma = (double)orient * (area > 0.0 ? 1.0 : -1.0);
  for (int c = 0; c < 2; ++c) {
    std::vector<double> r(n);
    for (int64_t j = 0; j < n; ++j) {
      const double pm = pts[2 * ((j + n - 1) % n) + c], p0 = pts[2 * j + c], pp = pts[2 * ((j + 1) % n) + c];
      r[j] = 6.0 * ((pp - p0) - (p0 - pm));
    }
    std::vector<double> x = tridiag(diag, r);
    const double fact = (x[0] + x[n - 1] / gamma) / (1.0 + z[0] + z[n - 1] / gamma);
    for (int64_t j = 0; j < n; ++j) x[j] -= fact * z[j];
    co[c].resize(4 * n);
    for (int64_t j = 0; j < n; ++j) {
      const int64_t k = (j + 1) % n;
      const double p0 = pts[2 * j + c], p1 = pts[2 * k + c];
      double *q = &co[c][4 * j];
      q[0] = p0;
      q[1] = (p1 - p0) - (2.0 * x[j] + x[k]) / 6.0;
      q[2] = 0.5 * x[j];
      q[3] = (x[k] - x[j]) / 6.0;
    }
  }
}

void SplineCurve2::eval(double t, double *X, double *X1, double *X2) const {
  double tt = std::fmod(t, (double)m);
  if (tt < 0) tt += (double)m;
  int64_t j = (int64_t)std::floor(tt);
  if (j > m - 1) j = m - 1;
  const double s = tt - (double)j;
  for (int c = 0; c < 2; ++c) {
    const double *q = &co[c][4 * j];
    if (X) X[c] = q[0] + s * (q[1] + s * (q[2] + s * q[3]));
    if (X1) X1[c] = q[1] + s * (2.0 * q[2] + s * 3.0 * q[3]);
    if (X2) X2[c] = 2.0 * q[2] + 6.0 * q[3] * s;
  }
}

void SplineCurve2::tangent(double t, double *tau, double &speed) const {
  double X1[2];
  eval(t, nullptr, X1, nullptr);
  speed = std::sqrt(X1[0] * X1[0] + X1[1] * X1[1]);
  tau[0] = X1[0] / speed;
  tau[1] = X1[1] / speed;
}

// n = sigma (y', -x') / |X'|; dn/ds = sigma k tau with the signed curvature
// k = (x' y'' - y' x'') / |X'|^3, so the shape operator is W = sigma k tau tau^T.
void SplineCurve2::normal_shape(double t, double *n, double *W) const {
  double X1[2], X2[2];
  eval(t, nullptr, X1, X2);
  const double sp = std::sqrt(X1[0] * X1[0] + X1[1] * X1[1]);
  const double tau[2] = {X1[0] / sp, X1[1] / sp};
  n[0] = sigma * X1[1] / sp;
  n[1] = -sigma * X1[0] / sp;
  const double k = (X1[0] * X2[1] - X1[1] * X2[0]) / (sp * sp * sp);
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) W[i * 2 + j] = sigma * k * tau[i] * tau[j];
}

namespace {

inline double cubic(const double *q, double s) { return q[0] + s * (q[1] + s * (q[2] + s * q[3])); }
inline double dcubic(const double *q, double s) { return q[1] + s * (2.0 * q[2] + s * 3.0 * q[3]); }

// Break points 0 < s < 1 where the derivative of the cubic vanishes, sorted, framed by 0 and 1.
int monotone_breaks(const double *q, double *b) {
  int nb = 0;
  b[nb++] = 0.0;
  const double A = 3.0 * q[3], B = 2.0 * q[2], C = q[1];
  double r[2];
  int nr = 0;
  if (A == 0.0) {
    if (B != 0.0) r[nr++] = -C / B;
  } else {
    const double disc = B * B - 4.0 * A * C;
    if (disc > 0.0) {
      const double sq = std::sqrt(disc);
      const double qq = -0.5 * (B + (B >= 0 ? sq : -sq));
      r[nr++] = qq / A;
      if (qq != 0.0) r[nr++] = C / qq;
    }
  }
  if (nr == 2 && r[1] < r[0]) std::swap(r[0], r[1]);
  for (int i = 0; i < nr; ++i)
    if (r[i] > 0.0 && r[i] < 1.0) b[nb++] = r[i];
  b[nb++] = 1.0;
  return nb;
}

// Root of f = cubic - v on [sa, sb], where f(sa) > 0 exactly when a_above and f(sb) > 0 exactly
// when not: safeguarded Newton that keeps a bracket [s_le, s_gt] with f(s_le) <= 0 < f(s_gt).
double bracketed_root(const double *q, double v, double sa, double sb, bool a_above) {
  double s_le = a_above ? sb : sa, s_gt = a_above ? sa : sb;
  const double f_le = cubic(q, s_le) - v;
  if (f_le == 0.0) return s_le;
  const double f_gt = cubic(q, s_gt) - v;
  double s = s_le - f_le * (s_gt - s_le) / (f_gt - f_le);
  if (!(s > std::min(s_le, s_gt) && s < std::max(s_le, s_gt))) s = 0.5 * (s_le + s_gt);
  for (int it = 0; it < 100; ++it) {
    const double f = cubic(q, s) - v;
    if (f == 0.0) return s;
    if (f < 0.0) s_le = s; else s_gt = s;
    const double df = dcubic(q, s);
    double sn = df != 0.0 ? s - f / df : 0.5 * (s_le + s_gt);
    const double lo = std::min(s_le, s_gt), hi = std::max(s_le, s_gt);
    if (!(sn > lo && sn < hi)) sn = 0.5 * (s_le + s_gt);
    if (sn == s || hi - lo <= 0.0) return s;
    s = sn;
    if (std::fabs(s_gt - s_le) <= 4e-16) break;
  }
  return s;
}

}  // namespace

void SplineCurve2::grid_line_roots(int coord, double lo, double h, int64_t nl,
                                   std::vector<std::vector<std::pair<double, double>>> &out) const {
  out.assign(nl, {});
  const int other = 1 - coord;
  for (int64_t j = 0; j < m; ++j) {
    const double *q = &co[coord][4 * j], *qo = &co[other][4 * j];
    double b[4];
    const int nb = monotone_breaks(q, b);
    for (int p = 0; p + 1 < nb; ++p) {
      const double sa = b[p], sb = b[p + 1];
      // the ends of a piece take the node values themselves, so that neighbouring pieces agree
      // exactly at their common node
      const double va = p == 0 ? q[0] : cubic(q, sa);
      const double vb = p + 2 == nb ? co[coord][4 * ((j + 1) % m)] : cubic(q, sb);
      const double vmin = std::min(va, vb), vmax = std::max(va, vb);
      int64_t k0 = (int64_t)std::floor((vmin - lo) / h) - 2, k1 = (int64_t)std::ceil((vmax - lo) / h);
      k0 = std::max<int64_t>(k0, 0);
      k1 = std::min<int64_t>(k1, nl - 1);
      for (int64_t k = k0; k <= k1; ++k) {
        const double v = lo + h * (double)(k + 1);
        if ((va > v) == (vb > v)) continue;
        const double s = bracketed_root(q, v, sa, sb, va > v);
        double tp = (double)j + s;
        if (tp >= (double)m) tp -= (double)m;        // the root at the end of the last piece is t = 0
        out[k].push_back({tp, cubic(qo, s)});
      }
    }
  }
}

}  // namespace kfbi
