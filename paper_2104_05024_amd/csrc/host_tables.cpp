// Host construction of the KFBI static tables (FP64, deterministic, built once per problem).
//
// What is built, following the implementation paragraph after Algorithm 1 (Sec. 6):
//  * quasi-uniform interface nodes with normals and shape operators,
//  * the side (tissue "+" / complement "-") of every interior grid node,
//  * every intersection of the boundary with a grid arm (Sec. 5.3: one crossing per arm),
//  * weights that carry the density psi and its surface gradient to intersections and
//    nodes (the paper's local coordinate systems, Sec. 5.3 Fig. 1 paragraph),
//  * per interface node the "nearest six / ten" grid nodes of the quadratic fit and the
//    gradient rows of the inverse h-scaled Vandermonde matrix (Sec. 5.4).
// Analytic shapes are star-shaped surfaces r = R(u) (see kfbi.h); their level set is
// phi = orient (|x| - R(x/|x|)), with analytic gradient and Hessian.  2D curves given by their
// nodes use the periodic cubic spline through them (host_spline.cpp): grid nodes take their
// side from the parity of the crossings on their grid row, crossings are the spline's roots on
// the grid lines, and the transfer runs in the spline parameter.  3D surfaces given as
// triangle meshes (host_mesh.cpp) take their sides from crossing parity on the grid lines and
// their crossings, normals and shape operators from the mesh's local quadratic coordinate
// systems.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <numeric>
#include <stdexcept>

#include "host_tables.h"

namespace kfbi {
namespace {

inline double ipow(double x, int k) {
  double r = 1.0;
  for (int i = 0; i < k; ++i) r *= x;
  return r;
}

// R(u) = E(u) (1 + P(u)) with its ambient gradient g and Hessian H (row-major d x d).
void radial(const kfbi_surface &s, int d, const double *u, double &G, double *g, double *H) {
  double a2[3], c[3], q = 0.0;
  for (int i = 0; i < d; ++i) {
    a2[i] = s.axes[i] * s.axes[i];
    c[i] = u[i] / a2[i];
    q += u[i] * u[i] / a2[i];
  }
  const double E = 1.0 / std::sqrt(q), E3 = E * E * E, E5 = E3 * E * E;
  double gE[3], HE[9], gP[3] = {0, 0, 0}, HP[9] = {0}, P = 0.0;
  for (int i = 0; i < d; ++i) {
    gE[i] = -E3 * c[i];
    for (int j = 0; j < d; ++j) HE[i * d + j] = 3.0 * E5 * c[i] * c[j] - (i == j ? E3 / a2[i] : 0.0);
  }
  for (int t = 0; t < s.n_terms; ++t) {
    const int *e = s.exps[t];
    const double cf = s.coef[t];
    double m = 1.0;
    for (int i = 0; i < d; ++i) m *= ipow(u[i], e[i]);
    P += cf * m;
    for (int j = 0; j < d; ++j) {
      if (e[j] == 0) continue;
      int ej[3] = {e[0], e[1], e[2]};
      ej[j] -= 1;
      double mj = 1.0;
      for (int i = 0; i < d; ++i) mj *= ipow(u[i], ej[i]);
      gP[j] += cf * e[j] * mj;
      for (int k = 0; k < d; ++k) {
        if (ej[k] == 0) continue;
        int ejk[3] = {ej[0], ej[1], ej[2]};
        ejk[k] -= 1;
        double mjk = 1.0;
        for (int i = 0; i < d; ++i) mjk *= ipow(u[i], ejk[i]);
        HP[j * d + k] += cf * e[j] * ej[k] * mjk;
      }
    }
  }
  G = E * (1.0 + P);
  for (int i = 0; i < d; ++i) {
    g[i] = (1.0 + P) * gE[i] + E * gP[i];
    for (int j = 0; j < d; ++j)
      H[i * d + j] = (1.0 + P) * HE[i * d + j] + gE[i] * gP[j] + gP[i] * gE[j] + E * HP[i * d + j];
  }
}

double phi_of(const kfbi_surface &s, int d, const double *x) {
  double r2 = 0.0;
  for (int i = 0; i < d; ++i) r2 += x[i] * x[i];
  const double r = std::sqrt(r2);
  double u[3] = {1.0, 0.0, 0.0};
  if (r != 0.0)
    for (int i = 0; i < d; ++i) u[i] = x[i] / r;
  double G, g[3], H[9];
  radial(s, d, u, G, g, H);
  return s.orient * (r - G);
}

// phi, grad phi and (if hess != nullptr) Hess phi.
// rho(x) = R(x/r): grad rho = P_u g / r, Hess rho = (P_u H P_u - s P_u - u g_t^T - g_t u^T)/r^2.
void levelset(const kfbi_surface &s, int d, const double *x, double &phi, double *grad, double *hess) {
  double r2 = 0.0;
  for (int i = 0; i < d; ++i) r2 += x[i] * x[i];
  const double r = std::sqrt(r2);
  double u[3];
  for (int i = 0; i < d; ++i) u[i] = x[i] / r;
  double G, g[3], H[9];
  radial(s, d, u, G, g, H);
  const double o = s.orient;
  phi = o * (r - G);
  double Pu[9], gt[3] = {0, 0, 0}, sdot = 0.0;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) Pu[i * d + j] = (i == j ? 1.0 : 0.0) - u[i] * u[j];
  for (int i = 0; i < d; ++i) {
    for (int j = 0; j < d; ++j) gt[i] += Pu[i * d + j] * g[j];
    sdot += u[i] * g[i];
  }
  for (int i = 0; i < d; ++i) grad[i] = o * (u[i] - gt[i] / r);
  if (!hess) return;
  double PH[9], PHP[9];
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      double acc = 0.0;
      for (int k = 0; k < d; ++k) acc += Pu[i * d + k] * H[k * d + j];
      PH[i * d + j] = acc;
    }
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      double acc = 0.0;
      for (int k = 0; k < d; ++k) acc += PH[i * d + k] * Pu[k * d + j];
      PHP[i * d + j] = acc;
    }
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      const double hr = (PHP[i * d + j] - sdot * Pu[i * d + j] - u[i] * gt[j] - gt[i] * u[j]) / r2;
      hess[i * d + j] = o * (Pu[i * d + j] / r - hr);
    }
}

// Unit normal out of the tissue and shape operator W = P_n Hess(phi) P_n / |grad phi|.
void normal_shape(const kfbi_surface &s, int d, const double *x, double *n, double *W) {
  double phi, grad[3], hess[9];
  levelset(s, d, x, phi, grad, hess);
  double gn = 0.0;
  for (int i = 0; i < d; ++i) gn += grad[i] * grad[i];
  gn = std::sqrt(gn);
  for (int i = 0; i < d; ++i) n[i] = grad[i] / gn;
  double Pn[9], T[9];
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) Pn[i * d + j] = (i == j ? 1.0 : 0.0) - n[i] * n[j];
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      double acc = 0.0;
      for (int k = 0; k < d; ++k) acc += Pn[i * d + k] * hess[k * d + j];
      T[i * d + j] = acc;
    }
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      double acc = 0.0;
      for (int k = 0; k < d; ++k) acc += T[i * d + k] * Pn[k * d + j];
      W[i * d + j] = acc / gn;
    }
}

void node_direction(int d, int64_t m, int64_t j, double *u) {
  if (d == 2) {
    const double t = 2.0 * M_PI * (double)j / (double)m;
    u[0] = std::cos(t);
    u[1] = std::sin(t);
    return;
  }
  const double z = 1.0 - (2.0 * (double)j + 1.0) / (double)m;
  const double az = (double)j * (M_PI * (3.0 - std::sqrt(5.0)));
  const double rho = std::sqrt(1.0 - z * z);
  u[0] = rho * std::cos(az);
  u[1] = rho * std::sin(az);
  u[2] = z;
}

// 2D: unit tangent (increasing t) and speed |X'(t)| of X(t) = R(u(t)) u(t).
void curve_tangent(const kfbi_surface &s, double t, double *tau, double &speed) {
  const double u[2] = {std::cos(t), std::sin(t)}, up[2] = {-std::sin(t), std::cos(t)};
  double G, g[3], H[9];
  radial(s, 2, u, G, g, H);
  const double dR = g[0] * up[0] + g[1] * up[1];
  const double Xp[2] = {dR * u[0] + G * up[0], dR * u[1] + G * up[1]};
  speed = std::sqrt(Xp[0] * Xp[0] + Xp[1] * Xp[1]);
  tau[0] = Xp[0] / speed;
  tau[1] = Xp[1] / speed;
}

// Householder least squares: rows 0..nrow-1 of pinv(A) for A (m x n, m >= n, full rank).
void pinv_rows(const double *A_in, int m, int n, int nrow, double *out /* nrow x m */) {
  std::vector<double> A(A_in, A_in + (size_t)m * n), Q((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) Q[(size_t)i * m + i] = 1.0;   // Q^T accumulated as rows
  for (int k = 0; k < n; ++k) {
    double nrm = 0.0;
    for (int i = k; i < m; ++i) nrm += A[(size_t)i * n + k] * A[(size_t)i * n + k];
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) continue;
    const double alpha = A[(size_t)k * n + k] > 0 ? -nrm : nrm;
    std::vector<double> v(m, 0.0);
    for (int i = k; i < m; ++i) v[i] = A[(size_t)i * n + k];
    v[k] -= alpha;
    double vv = 0.0;
    for (int i = k; i < m; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    for (int j = 0; j < n; ++j) {
      double dot = 0.0;
      for (int i = k; i < m; ++i) dot += v[i] * A[(size_t)i * n + j];
      const double f = 2.0 * dot / vv;
      for (int i = k; i < m; ++i) A[(size_t)i * n + j] -= f * v[i];
    }
    for (int j = 0; j < m; ++j) {   // apply to Q^T columns: Q^T <- H Q^T
      double dot = 0.0;
      for (int i = k; i < m; ++i) dot += v[i] * Q[(size_t)i * m + j];
      const double f = 2.0 * dot / vv;
      for (int i = k; i < m; ++i) Q[(size_t)i * m + j] -= f * v[i];
    }
  }
  // Solve R X = (Q^T)[0:n, :], X is n x m; keep rows 0..nrow-1.
  std::vector<double> X((size_t)n * m);
  for (int j = 0; j < m; ++j)
    for (int i = n - 1; i >= 0; --i) {
      double acc = Q[(size_t)i * m + j];
      for (int k = i + 1; k < n; ++k) acc -= A[(size_t)i * n + k] * X[(size_t)k * m + j];
      X[(size_t)i * m + j] = acc / A[(size_t)i * n + i];
    }
  std::memcpy(out, X.data(), sizeof(double) * nrow * m);
}

// Inverse of a small dense matrix by Gauss-Jordan with partial pivoting.
bool invert(std::vector<double> A, int n, std::vector<double> &inv) {
  inv.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[(size_t)r * n + c]) > std::fabs(A[(size_t)p * n + c])) p = r;
    if (A[(size_t)p * n + c] == 0.0) return false;
    if (p != c)
      for (int k = 0; k < n; ++k) {
        std::swap(A[(size_t)p * n + k], A[(size_t)c * n + k]);
        std::swap(inv[(size_t)p * n + k], inv[(size_t)c * n + k]);
      }
    const double piv = A[(size_t)c * n + c];
    for (int k = 0; k < n; ++k) {
      A[(size_t)c * n + k] /= piv;
      inv[(size_t)c * n + k] /= piv;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = A[(size_t)r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        A[(size_t)r * n + k] -= f * A[(size_t)c * n + k];
        inv[(size_t)r * n + k] -= f * inv[(size_t)c * n + k];
      }
    }
  }
  return true;
}

// Quadratic Taylor basis at scaled offset r: 1, r_a, r_a^2/2, r_a r_b.
void quad_basis(int d, const double *r, double *b) {
  if (d == 2) {
    const double x = r[0], y = r[1];
    b[0] = 1; b[1] = x; b[2] = y; b[3] = x * x / 2; b[4] = x * y; b[5] = y * y / 2;
    return;
  }
  const double x = r[0], y = r[1], z = r[2];
  b[0] = 1; b[1] = x; b[2] = y; b[3] = z;
  b[4] = x * x / 2; b[5] = y * y / 2; b[6] = z * z / 2;
  b[7] = x * y; b[8] = x * z; b[9] = y * z;
}

// Uniform-cell index over the nodes of one 3D surface for exact k-nearest queries.
struct NodeGrid {
  double lo[3], cell;
  int n[3];
  std::vector<int64_t> start, items;
  const double *X;
  int64_t first, count;

  NodeGrid(const double *Xall, int64_t first_, int64_t count_) : X(Xall), first(first_), count(count_) {
    double hi[3];
    for (int a = 0; a < 3; ++a) lo[a] = hi[a] = X[first * 3 + a];
    for (int64_t i = first; i < first + count; ++i)
      for (int a = 0; a < 3; ++a) {
        lo[a] = std::min(lo[a], X[i * 3 + a]);
        hi[a] = std::max(hi[a], X[i * 3 + a]);
      }
    double area = 0.0;  // crude surface-area scale -> ~4 nodes per cell
    const double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]});
    area = 3.2 * ext * ext;
    cell = std::max(1e-6, 2.0 * std::sqrt(area / (double)count));
    for (int a = 0; a < 3; ++a) {
      lo[a] -= 1e-9;
      n[a] = std::max(1, (int)std::ceil((hi[a] - lo[a]) / cell) + 1);
    }
    const int64_t nc = (int64_t)n[0] * n[1] * n[2];
    std::vector<int64_t> cnt(nc + 1, 0), key(count);
    for (int64_t i = 0; i < count; ++i) {
      key[i] = cell_of(&X[(first + i) * 3]);
      cnt[key[i] + 1]++;
    }
    for (int64_t c = 0; c < nc; ++c) cnt[c + 1] += cnt[c];
    start = cnt;
    items.resize(count);
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t i = 0; i < count; ++i) items[fill[key[i]]++] = first + i;
  }
  int clampi(int v, int a) const { return std::min(std::max(v, 0), n[a] - 1); }
  int64_t cell_of(const double *p) const {
    int c[3];
    for (int a = 0; a < 3; ++a) c[a] = clampi((int)std::floor((p[a] - lo[a]) / cell), a);
    return ((int64_t)c[2] * n[1] + c[1]) * n[0] + c[0];
  }
  // k nearest by (squared distance, node index); squared distance summed x, y, z in order.
  void knn(const double *p, int k, int64_t *out) const {
    int c[3];
    for (int a = 0; a < 3; ++a) c[a] = (int)std::floor((p[a] - lo[a]) / cell);
    std::vector<std::pair<double, int64_t>> cand;
    for (int rad = 1;; ++rad) {
      cand.clear();
      for (int dz = -rad; dz <= rad; ++dz)
        for (int dy = -rad; dy <= rad; ++dy)
          for (int dx = -rad; dx <= rad; ++dx) {
            const int ix = c[0] + dx, iy = c[1] + dy, iz = c[2] + dz;
            if (ix < 0 || iy < 0 || iz < 0 || ix >= n[0] || iy >= n[1] || iz >= n[2]) continue;
            const int64_t cc = ((int64_t)iz * n[1] + iy) * n[0] + ix;
            for (int64_t s = start[cc]; s < start[cc + 1]; ++s) {
              const int64_t j = items[s];
              const double dx0 = X[j * 3 + 0] - p[0], dy0 = X[j * 3 + 1] - p[1], dz0 = X[j * 3 + 2] - p[2];
              const double d2 = (dx0 * dx0 + dy0 * dy0) + dz0 * dz0;
              cand.push_back({d2, j});
            }
          }
      const bool all = (int64_t)cand.size() >= count;
      if ((int)cand.size() >= k) {
        std::partial_sort(cand.begin(), cand.begin() + k, cand.end());
        const double reach = rad * cell;
        if (all || cand[k - 1].first <= reach * reach) break;
      } else if (all) {
        throw GeometryError{"fewer interface nodes than the transfer stencil"};
      }
    }
    for (int i = 0; i < k; ++i) out[i] = cand[i].second;
  }
};

void tangent_frame(const double *n, double *t1, double *t2) {
  int m = 0;
  for (int a = 1; a < 3; ++a)
    if (std::fabs(n[a]) < std::fabs(n[m])) m = a;
  double e[3] = {0, 0, 0};
  e[m] = 1.0;
  t1[0] = e[1] * n[2] - e[2] * n[1];
  t1[1] = e[2] * n[0] - e[0] * n[2];
  t1[2] = e[0] * n[1] - e[1] * n[0];
  const double l = std::sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
  for (int a = 0; a < 3; ++a) t1[a] /= l;
  t2[0] = n[1] * t1[2] - n[2] * t1[1];
  t2[1] = n[2] * t1[0] - n[0] * t1[2];
  t2[2] = n[0] * t1[1] - n[1] * t1[0];
}

// LSQ quadratic fit over k nearest nodes in tangent coordinates / h: psi(p), grad_Gamma psi(p).
void lsq_transfer(const NodeGrid &ng, const double *X, const double *p, const double *n, double h, int k,
                  int64_t *idx, double *w0, double *wg) {
  ng.knn(p, k, idx);
  double t1[3], t2[3];
  tangent_frame(n, t1, t2);
  std::vector<double> V((size_t)k * 6), pinv((size_t)3 * k);
  for (int i = 0; i < k; ++i) {
    const double *x = &X[idx[i] * 3];
    const double df[3] = {x[0] - p[0], x[1] - p[1], x[2] - p[2]};
    const double xi = (df[0] * t1[0] + df[1] * t1[1] + df[2] * t1[2]) / h;
    const double eta = (df[0] * t2[0] + df[1] * t2[1] + df[2] * t2[2]) / h;
    double *row = &V[(size_t)i * 6];
    row[0] = 1; row[1] = xi; row[2] = eta; row[3] = xi * xi; row[4] = xi * eta; row[5] = eta * eta;
  }
  pinv_rows(V.data(), k, 6, 3, pinv.data());
  for (int i = 0; i < k; ++i) {
    w0[i] = pinv[i];
    for (int a = 0; a < 3; ++a) wg[i * 3 + a] = (pinv[k + i] * t1[a] + pinv[2 * k + i] * t2[a]) / h;
  }
}

// 2D: cubic Lagrange in the polar angle over nodes j-1..j+2, j = floor(t*/dt).
void lagrange_transfer(const kfbi_surface &s, int64_t off, int64_t m, const double *p, int64_t *idx,
                       double *w0, double *wg) {
  const double dt = 2.0 * M_PI / (double)m;
  double t = std::atan2(p[1], p[0]);
  t = std::fmod(t, 2.0 * M_PI);
  if (t < 0) t += 2.0 * M_PI;
  int64_t j = (int64_t)std::floor(t / dt);
  if (j > m - 1) j = m - 1;
  const double sl = (t - (double)j * dt) / dt;
  const double w[4] = {-sl * (sl - 1) * (sl - 2) / 6.0, (sl + 1) * (sl - 1) * (sl - 2) / 2.0,
                       -(sl + 1) * sl * (sl - 2) / 2.0, (sl + 1) * sl * (sl - 1) / 6.0};
  const double dw[4] = {-(3 * sl * sl - 6 * sl + 2) / 6.0, (3 * sl * sl - 4 * sl - 1) / 2.0,
                        -(3 * sl * sl - 2 * sl - 2) / 2.0, (3 * sl * sl - 1) / 6.0};
  double tau[2], speed;
  curve_tangent(s, t, tau, speed);
  for (int i = 0; i < 4; ++i) {
    idx[i] = off + (((j + i - 1) % m) + m) % m;
    w0[i] = w[i];
    const double c = dw[i] / (dt * speed);
    wg[i * 2 + 0] = c * tau[0];
    wg[i * 2 + 1] = c * tau[1];
  }
}

// Spline curves: the same cubic Lagrange fit in the spline parameter t* (nodes at t = j).
void spline_transfer(const SplineCurve2 &sc, int64_t off, double tp, int64_t *idx, double *w0, double *wg) {
  const int64_t m = sc.m;
  const int64_t j = (int64_t)std::floor(tp);
  const double sl = tp - (double)j;
  const double w[4] = {-sl * (sl - 1) * (sl - 2) / 6.0, (sl + 1) * (sl - 1) * (sl - 2) / 2.0,
                       -(sl + 1) * sl * (sl - 2) / 2.0, (sl + 1) * sl * (sl - 1) / 6.0};
  const double dw[4] = {-(3 * sl * sl - 6 * sl + 2) / 6.0, (3 * sl * sl - 4 * sl - 1) / 2.0,
                        -(3 * sl * sl - 2 * sl - 2) / 2.0, (3 * sl * sl - 1) / 6.0};
  double tau[2], speed;
  sc.tangent(tp, tau, speed);
  for (int i = 0; i < 4; ++i) {
    idx[i] = off + (((j + i - 1) % m) + m) % m;
    w0[i] = w[i];
    const double c = dw[i] / speed;
    wg[i * 2 + 0] = c * tau[0];
    wg[i * 2 + 1] = c * tau[1];
  }
}

int64_t lin_of(const int64_t *k, int d, int64_t N) {
  int64_t lin = 0;
  for (int a = d - 1; a >= 0; --a) lin = lin * N + k[a];
  return lin;
}

}  // namespace

void build_host_tables(const kfbi_interface &iface, const kfbi_grid &grid, const kfbi_coeffs &co,
                       HostTables &t) {
  const int d = iface.dim;
  if ((d != 2 && d != 3) || grid.dim != d) throw std::invalid_argument("dimension must be 2 or 3 and match");
  if (iface.n_surfaces < 1 || iface.n_surfaces > KFBI_MAX_SURFACES) throw std::invalid_argument("n_surfaces");
  if (grid.cells < 8 || !(grid.hi > grid.lo) || !std::isfinite(grid.lo) || !std::isfinite(grid.hi))
    throw std::invalid_argument("grid");
  if (co.ncomp != 1 && co.ncomp != 2) throw std::invalid_argument("ncomp");
  if (!(co.kappa >= 0) || !std::isfinite(co.kappa)) throw std::invalid_argument("kappa");
  for (int c = 0; c < co.ncomp; ++c)
    for (int a = 0; a < d; ++a)
      if (!(co.D[c][a] > 0) || !std::isfinite(co.D[c][a]))
        throw std::invalid_argument("D must be positive per component and axis");
  t.dim = d;
  t.ncomp = co.ncomp;
  t.cells = grid.cells;
  t.N = grid.cells - 1;
  t.lo = grid.lo;
  t.hi = grid.hi;
  t.h = (grid.hi - grid.lo) / grid.cells;
  t.kappa = co.kappa;
  std::memcpy(t.D, co.D, sizeof(t.D));
  t.surf.assign(iface.surf, iface.surf + iface.n_surfaces);
  t.offsets.assign(1, 0);
  std::vector<SplineCurve2> spl(t.surf.size());
  std::vector<TriMesh3> msh(t.surf.size());
  std::vector<char> is_spl(t.surf.size(), 0), is_msh(t.surf.size(), 0);
  for (size_t si = 0; si < t.surf.size(); ++si) {
    const auto &s = t.surf[si];
    if (s.n_nodes < 8 || (s.orient != 1 && s.orient != -1)) throw std::invalid_argument("surface descriptor");
    if (s.kind == KFBI_SURF_ANALYTIC) {
      if (s.n_terms < 0 || s.n_terms > KFBI_MAX_TERMS) throw std::invalid_argument("surface descriptor");
      for (int a = 0; a < d; ++a)
        if (!(s.axes[a] > 0)) throw std::invalid_argument("surface axes");
    } else if (s.kind == KFBI_SURF_SPLINE) {
      if (d != 2) throw std::invalid_argument("spline curves are two-dimensional");
      if (!s.points) throw std::invalid_argument("spline curve without points");
      for (int64_t j = 0; j < 2 * s.n_nodes; ++j)
        if (!std::isfinite(s.points[j])) throw std::invalid_argument("spline points must be finite");
      spl[si].build(s.points, s.n_nodes, s.orient);
      is_spl[si] = 1;
    } else if (s.kind == KFBI_SURF_MESH) {
      if (d != 3) throw std::invalid_argument("triangle meshes are three-dimensional");
      if (!s.points || !s.tris || s.n_tris < 4) throw std::invalid_argument("mesh without points or triangles");
      for (int64_t j = 0; j < 3 * s.n_nodes; ++j)
        if (!std::isfinite(s.points[j])) throw std::invalid_argument("mesh points must be finite");
      msh[si].build(s.points, s.n_nodes, s.tris, s.n_tris, s.orient);
      is_msh[si] = 1;
    } else {
      throw std::invalid_argument("surface kind");
    }
    t.offsets.push_back(t.offsets.back() + s.n_nodes);
  }
  t.M = t.offsets.back();
  const int64_t N = t.N, M = t.M;
  const double h = t.h, lo = t.lo;
  int64_t total = 1;
  for (int a = 0; a < d; ++a) total *= N;

  // -- clearance: the boundary stays >= 3h inside the box (stencils never reach it)
  for (size_t si = 0; si < t.surf.size(); ++si) {
    const auto &s = t.surf[si];
    if (is_spl[si]) {
      for (int64_t q = 0; q < 16 * s.n_nodes; ++q) {
        double x[2];
        spl[si].eval((double)q / 16.0, x, nullptr, nullptr);
        for (int a = 0; a < 2; ++a)
          if (x[a] > grid.hi - 3 * h || x[a] < grid.lo + 3 * h) throw GeometryError{"interface closer than 3h to the box"};
      }
      continue;
    }
    if (is_msh[si]) {
      for (int64_t j = 0; j < 3 * s.n_nodes; ++j)
        if (s.points[j] > grid.hi - 3 * h || s.points[j] < grid.lo + 3 * h)
          throw GeometryError{"interface closer than 3h to the box"};
      continue;
    }
    const int64_t m = std::max<int64_t>(s.n_nodes, d == 3 ? 4096 : 1024);
    for (int64_t j = 0; j < m; ++j) {
      double u[3], G, g[3], H[9];
      node_direction(d, m, j, u);
      radial(s, d, u, G, g, H);
      for (int a = 0; a < d; ++a) {
        const double x = G * u[a];
        if (x > grid.hi - 3 * h || x < grid.lo + 3 * h) throw GeometryError{"interface closer than 3h to the box"};
      }
    }
  }

  // -- interface nodes
  t.X.resize(M * d);
  t.nrm.resize(M * d);
  t.W.resize(M * d * d);
  for (size_t s = 0; s < t.surf.size(); ++s)
    for (int64_t j = 0; j < t.surf[s].n_nodes; ++j) {
      const int64_t i = t.offsets[s] + j;
      if (is_spl[s]) {
        for (int a = 0; a < 2; ++a) t.X[i * 2 + a] = t.surf[s].points[2 * j + a];
        spl[s].normal_shape((double)j, &t.nrm[i * 2], &t.W[i * 4]);
        continue;
      }
      if (is_msh[s]) {
        for (int a = 0; a < 3; ++a) t.X[i * 3 + a] = t.surf[s].points[3 * j + a];
        msh[s].vertex_geometry(j, &t.nrm[i * 3], &t.W[i * 9]);
        continue;
      }
      double u[3], G, g[3], H[9];
      node_direction(d, t.surf[s].n_nodes, j, u);
      radial(t.surf[s], d, u, G, g, H);
      for (int a = 0; a < d; ++a) t.X[i * d + a] = G * u[a];
      normal_shape(t.surf[s], d, &t.X[i * d], &t.nrm[i * d], &t.W[i * d * d]);
    }

  // -- sides of the grid nodes, per surface
  const int S_ = (int)t.surf.size();
  std::vector<std::vector<int8_t>> side(S_, std::vector<int8_t>(total));
  // spline curves: crossings of every grid row (y = const) and column (x = const), sorted by
  // the coordinate along the line; a node's side is the parity of the row crossings beyond it
  // A node within kSideTol of a crossing on its row or column lies on the curve: it counts as
  // tissue and is the crossing point of its arms that change side (on_t: its spline parameter).
  std::vector<std::vector<std::vector<std::pair<double, double>>>> rows(S_), cols(S_);
  std::vector<std::vector<double>> on_t(S_);
  for (int s = 0; s < S_; ++s) {
    if (!is_spl[s]) continue;
    on_t[s].assign(total, std::nan(""));
    spl[s].grid_line_roots(1, lo, h, N, rows[s]);
    spl[s].grid_line_roots(0, lo, h, N, cols[s]);
    for (auto *lines : {&rows[s], &cols[s]})
      for (auto &ln : *lines)
        std::sort(ln.begin(), ln.end(), [](const std::pair<double, double> &A, const std::pair<double, double> &B) {
          return A.second < B.second || (A.second == B.second && A.first < B.first);
        });
    for (int pass = 0; pass < 2; ++pass)           // rows (y = y_l), then columns (x = x_k)
      for (int64_t l = 0; l < N; ++l)
        for (const auto &r : pass == 0 ? rows[s][l] : cols[s][l]) {
          const int64_t k = (int64_t)std::llround((r.second - lo) / h) - 1;
          if (k < 0 || k >= N || std::fabs(r.second - (lo + h * (double)(k + 1))) > kSideTol) continue;
          const int64_t node = pass == 0 ? l * N + k : k * N + l;
          if (std::isnan(on_t[s][node])) on_t[s][node] = r.first;
        }
    for (int64_t l = 0; l < N; ++l) {
      const auto &ln = rows[s][l];
      for (int64_t k = 0; k < N; ++k) {
        const double x = lo + h * (double)(k + 1);
        size_t beyond = 0;
        for (const auto &r : ln)
          if (r.second > x) ++beyond;
        const bool interior = (beyond & 1) != 0;
        const bool on = !std::isnan(on_t[s][l * N + k]);
        side[s][l * N + k] = (on || interior == (t.surf[s].orient == 1)) ? 1 : 0;
      }
    }
  }
  // meshes: crossings of every grid line per axis; a node's side is the parity of the x-line
  // crossings beyond it, and a node within kSideTol of a crossing on any of its three lines
  // lies on the surface (tissue; the crossing point of its arms that change side)
  std::vector<std::array<std::vector<std::vector<std::pair<double, int64_t>>>, 3>> mlines(S_);
  for (int s = 0; s < S_; ++s) {
    if (!is_msh[s]) continue;
    for (int a = 0; a < 3; ++a) msh[s].grid_line_hits(a, lo, h, N, mlines[s][a]);
    std::vector<char> on(total, 0);
    for (int a = 0; a < 3; ++a) {
      const int bx = a == 0 ? 1 : 0, cx = a == 2 ? 1 : 2;
      for (int64_t ic = 0; ic < N; ++ic)
        for (int64_t ib = 0; ib < N; ++ib)
          for (const auto &hit : mlines[s][a][ic * N + ib]) {
            const int64_t k = (int64_t)std::llround((hit.first - lo) / h) - 1;
            if (k < 0 || k >= N || std::fabs(hit.first - (lo + h * (double)(k + 1))) > kSideTol) continue;
            int64_t idx[3];
            idx[a] = k;
            idx[bx] = ib;
            idx[cx] = ic;
            on[(idx[2] * N + idx[1]) * N + idx[0]] = 1;
          }
    }
    for (int64_t iz = 0; iz < N; ++iz)
      for (int64_t iy = 0; iy < N; ++iy) {
        const auto &ln = mlines[s][0][iz * N + iy];
        for (int64_t ix = 0; ix < N; ++ix) {
          const double x = lo + h * (double)(ix + 1);
          size_t beyond = 0;
          for (const auto &hit : ln)
            if (hit.first > x) ++beyond;
          const int64_t lin = (iz * N + iy) * N + ix;
          const bool interior = (beyond & 1) != 0;
          side[s][lin] = (on[lin] || interior == (t.surf[s].orient == 1)) ? 1 : 0;
        }
      }
  }
  for (int s = 0; s < S_; ++s) {
    if (is_spl[s] || is_msh[s]) continue;
#pragma omp parallel for schedule(static)
    for (int64_t lin = 0; lin < total; ++lin) {
      int64_t r = lin;
      double x[3];
      for (int a = 0; a < d; ++a) {
        x[a] = lo + h * (double)(r % N + 1);
        r /= N;
      }
      side[s][lin] = phi_of(t.surf[s], d, x) <= kSideTol ? 1 : 0;
    }
  }
  t.inside.assign(total, 1);
  for (int s = 0; s < S_; ++s)
    for (int64_t lin = 0; lin < total; ++lin) t.inside[lin] &= side[s][lin];

  // -- grid-arm intersections, ordered by (surface, axis, lower node)
  int64_t stride[3] = {1, N, N * N};
  std::vector<double> mesh_cn, mesh_cW;        // n, W of mesh crossings, in crossing order
  for (int s = 0; s < S_; ++s)
    for (int a = 0; a < d; ++a)
      for (int64_t lin = 0; lin < total; ++lin) {
        const int64_t ka = (lin / stride[a]) % N;
        if (ka == N - 1) continue;
        const int64_t lin1 = lin + stride[a];
        if (side[s][lin] == side[s][lin1]) continue;
        for (int o = 0; o < S_; ++o)
          if (o != s && !(side[o][lin] && side[o][lin1])) throw GeometryError{"grid arm crosses two surfaces"};
        double p[3];
        {
          int64_t r = lin;
          for (int b = 0; b < d; ++b) {
            p[b] = lo + h * (double)(r % N + 1);
            r /= N;
          }
        }
        const kfbi_surface &sf = t.surf[s];
        if (is_spl[s]) {
          // the one root of the spline on this arm: the arm's line is a row (x arms) or a column
          const int64_t kl = (lin / stride[1 - a]) % N;     // index of the line among rows / columns
          const auto &ln = a == 0 ? rows[s][kl] : cols[s][kl];
          const double x0 = p[a], x1 = lo + h * (double)(ka + 2);
          double tt, tp;
          if (!std::isnan(on_t[s][lin])) {            // an end on the curve is the crossing
            tt = 0.0;
            tp = on_t[s][lin];
          } else if (!std::isnan(on_t[s][lin1])) {
            tt = 1.0;
            tp = on_t[s][lin1];
          } else {
            int cnt = 0;
            double along = 0.0;
            tp = 0.0;
            for (const auto &r : ln)
              if (r.second >= x0 - kSideTol && r.second <= x1 + kSideTol) {
                ++cnt;
                along = r.second;
                tp = r.first;
              }
            if (cnt != 1) throw GeometryError{"grid arm crossed more than once"};
            tt = std::min(1.0, std::max(0.0, (along - x0) / h));
          }
          double z[3] = {p[0], p[1], p[2]};
          z[a] += tt * h;
          t.c_surf.push_back(s);
          t.c_axis.push_back(a);
          const bool in0 = side[s][lin] != 0;
          t.c_pin.push_back(in0 ? lin : lin1);
          t.c_pout.push_back(in0 ? lin1 : lin);
          for (int b = 0; b < d; ++b) t.c_z.push_back(z[b]);
          t.c_t.push_back(tp);
          continue;
        }
        if (is_msh[s]) {
          // the crossing on the flat triangle the arm passes through, moved onto that
          // triangle's six-point patch; an end point on the surface is the crossing itself
          const int bx = a == 0 ? 1 : 0, cx = a == 2 ? 1 : 2;
          int64_t kk[3];
          {
            int64_t r = lin;
            for (int b = 0; b < 3; ++b) {
              kk[b] = r % N;
              r /= N;
            }
          }
          const auto &ln = mlines[s][a][kk[cx] * N + kk[bx]];
          const double x0 = p[a], x1 = lo + h * (double)(ka + 2);
          double best = 0.0, cn[3], cW[9];
          int64_t tri = -1;
          bool at_end = false, at0 = false;
          for (const auto &hit : ln) {
            const double dd = std::min(std::fabs(hit.first - x0), std::fabs(hit.first - x1));
            if ((std::fabs(hit.first - x0) <= kSideTol || std::fabs(hit.first - x1) <= kSideTol) &&
                (!at_end || dd < best)) {
              at_end = true;
              best = dd;
              tri = hit.second;
              at0 = std::fabs(hit.first - x0) <= kSideTol;
            }
          }
          double z[3] = {p[0], p[1], p[2]};
          if (at_end) {
            if (!at0) z[a] = x1;
            msh[s].patch_geometry(tri, z, cn, cW);
          } else {
            int cnt = 0;
            double along = 0.0;
            for (const auto &hit : ln)
              if (hit.first >= x0 - kSideTol && hit.first <= x1 + kSideTol) {
                ++cnt;
                along = hit.first;
                tri = hit.second;
              }
            if (cnt != 1) throw GeometryError{"grid arm crossed more than once"};
            z[a] += msh[s].onto_patch(tri, p, a, along - x0, h, cn, cW);
          }
          t.c_surf.push_back(s);
          t.c_axis.push_back(a);
          const bool in0 = side[s][lin] != 0;
          t.c_pin.push_back(in0 ? lin : lin1);
          t.c_pout.push_back(in0 ? lin1 : lin);
          for (int b = 0; b < 3; ++b) t.c_z.push_back(z[b]);
          t.c_t.push_back((double)tri);                 // meshes: the triangle of the crossing
          for (int b = 0; b < 3; ++b) mesh_cn.push_back(cn[b]);
          for (int b = 0; b < 9; ++b) mesh_cW.push_back(cW[b]);
          continue;
        }
        auto f = [&](double tt, double &ft, double &dft) {
          double x[3] = {p[0], p[1], p[2]};
          x[a] += tt * h;
          double grad[3];
          levelset(sf, d, x, ft, grad, nullptr);
          dft = grad[a] * h;
        };
        double f0, f1, dd;
        f(0.0, f0, dd);
        f(1.0, f1, dd);
        double tt = std::fabs(f0) <= std::fabs(f1) ? 0.0 : 1.0;
        // a grid node on the boundary (|phi| <= kSideTol) is its own crossing point: along an arm
        // tangent to the boundary phi ~ t^2 there and the root would be ill-conditioned
        const bool on0 = std::fabs(f0) <= kSideTol, on1 = std::fabs(f1) <= kSideTol;
        if (on0) tt = 0.0;
        else if (on1) tt = 1.0;
        const bool bracket = f0 * f1 <= 0.0 && !on0 && !on1;
        double blo = f0 <= 0.0 ? 0.0 : 1.0, bhi = 1.0 - blo;
        if (bracket && f1 != f0) tt = std::min(1.0, std::max(0.0, -f0 / (f1 - f0)));
        if (bracket)
          for (int it = 0; it < 80; ++it) {
            double ft, dft;
            f(tt, ft, dft);
            if (ft == 0.0) break;
            if (ft < 0.0) blo = tt; else bhi = tt;
            double tn = dft != 0.0 ? tt - ft / dft : 0.0;
            const double A = std::min(blo, bhi), B = std::max(blo, bhi);
            if (dft == 0.0 || !(tn > A && tn < B)) tn = 0.5 * (blo + bhi);
            const bool done = std::fabs(tn - tt) <= 1e-15;
            tt = tn;
            if (done) break;
          }
        // an arm crossed more than once is outside the method's assumption
        int changes = 0;
        int prev = -1;
        for (int q = 0; q <= 8; ++q) {
          double x[3] = {p[0], p[1], p[2]};
          x[a] += (q / 8.0) * h;
          const int sd = phi_of(sf, d, x) <= kSideTol ? 1 : 0;
          if (prev >= 0 && sd != prev) ++changes;
          prev = sd;
        }
        if (changes != 1) throw GeometryError{"grid arm crossed more than once"};
        double z[3] = {p[0], p[1], p[2]};
        z[a] += tt * h;
        t.c_surf.push_back(s);
        t.c_axis.push_back(a);
        const bool in0 = side[s][lin] != 0;
        t.c_pin.push_back(in0 ? lin : lin1);
        t.c_pout.push_back(in0 ? lin1 : lin);
        for (int b = 0; b < d; ++b) t.c_z.push_back(z[b]);
        t.c_t.push_back(std::nan(""));
      }
  t.nc = (int64_t)t.c_surf.size();
  t.c_n.resize(t.nc * d);
  t.c_W.resize(t.nc * d * d);
  for (int64_t c = 0, mc = 0; c < t.nc; ++c) {
    if (is_msh[t.c_surf[c]]) {
      std::copy(&mesh_cn[3 * mc], &mesh_cn[3 * mc] + 3, &t.c_n[c * 3]);
      std::copy(&mesh_cW[9 * mc], &mesh_cW[9 * mc] + 9, &t.c_W[c * 9]);
      ++mc;
    } else if (is_spl[t.c_surf[c]])
      spl[t.c_surf[c]].normal_shape(t.c_t[c], &t.c_n[c * d], &t.c_W[c * d * d]);
    else
      normal_shape(t.surf[t.c_surf[c]], d, &t.c_z[c * d], &t.c_n[c * d], &t.c_W[c * d * d]);
  }

  // -- density transfer weights
  t.K = d == 2 ? 4 : kLsqNodes;
  t.Kn = d == 2 ? 5 : kLsqNodes;
  t.z_idx.resize(t.nc * t.K);
  t.z_w0.resize(t.nc * t.K);
  t.z_wg.resize(t.nc * t.K * d);
  t.q_idx.resize(M * t.Kn);
  t.q_wg.resize(M * t.Kn * d);
  for (int s = 0; s < S_; ++s) {
    const int64_t off = t.offsets[s], m = t.surf[s].n_nodes;
    if (is_msh[s]) {
      // the six-point system of the crossing's triangle (slots beyond six carry zero weight)
      // and the one-ring fit at each vertex
      for (int64_t c = 0; c < t.nc; ++c) {
        if (t.c_surf[c] != s) continue;
        int64_t idx[6];
        double w0[6], wg[18];
        msh[s].crossing_transfer((int64_t)t.c_t[c], &t.c_z[c * 3], idx, w0, wg);
        for (int k = 0; k < t.K; ++k) {
          t.z_idx[c * t.K + k] = off + (k < 6 ? idx[k] : idx[0]);
          t.z_w0[c * t.K + k] = k < 6 ? w0[k] : 0.0;
          for (int a = 0; a < 3; ++a) t.z_wg[(c * t.K + k) * 3 + a] = k < 6 ? wg[k * 3 + a] : 0.0;
        }
      }
      for (int64_t j = 0; j < m; ++j) {
        int64_t idx[10];
        double wg[30];
        const int k = msh[s].vertex_transfer(j, t.Kn, idx, wg);
        const int64_t q = off + j;
        for (int r = 0; r < t.Kn; ++r) {
          t.q_idx[q * t.Kn + r] = off + (r < k ? idx[r] : idx[0]);
          for (int a = 0; a < 3; ++a) t.q_wg[(q * t.Kn + r) * 3 + a] = r < k ? wg[r * 3 + a] : 0.0;
        }
      }
    } else if (is_spl[s]) {
      for (int64_t c = 0; c < t.nc; ++c)
        if (t.c_surf[c] == s) spline_transfer(spl[s], off, t.c_t[c], &t.z_idx[c * 4], &t.z_w0[c * 4], &t.z_wg[c * 8]);
      const double cw[5] = {1.0, -8.0, 0.0, 8.0, -1.0};
      for (int64_t j = 0; j < m; ++j) {
        double tau[2], speed;
        spl[s].tangent((double)j, tau, speed);
        for (int i = 0; i < 5; ++i) {
          const int64_t q = off + j;
          t.q_idx[q * 5 + i] = off + (((j + i - 2) % m) + m) % m;
          const double c = cw[i] / 12.0 / speed;
          t.q_wg[(q * 5 + i) * 2 + 0] = c * tau[0];
          t.q_wg[(q * 5 + i) * 2 + 1] = c * tau[1];
        }
      }
    } else if (d == 2) {
      for (int64_t c = 0; c < t.nc; ++c)
        if (t.c_surf[c] == s)
          lagrange_transfer(t.surf[s], off, m, &t.c_z[c * 2], &t.z_idx[c * 4], &t.z_w0[c * 4], &t.z_wg[c * 8]);
      const double dt = 2.0 * M_PI / (double)m;
      const double cw[5] = {1.0, -8.0, 0.0, 8.0, -1.0};
      for (int64_t j = 0; j < m; ++j) {
        const double tj = 2.0 * M_PI * (double)j / (double)m;
        double tau[2], speed;
        curve_tangent(t.surf[s], tj, tau, speed);
        for (int i = 0; i < 5; ++i) {
          const int64_t q = off + j;
          t.q_idx[q * 5 + i] = off + (((j + i - 2) % m) + m) % m;
          const double c = cw[i] / (12.0 * dt) / speed;
          t.q_wg[(q * 5 + i) * 2 + 0] = c * tau[0];
          t.q_wg[(q * 5 + i) * 2 + 1] = c * tau[1];
        }
      }
    } else {
      NodeGrid ng(t.X.data(), off, m);
#pragma omp parallel for schedule(dynamic, 256)
      for (int64_t c = 0; c < t.nc; ++c)
        if (t.c_surf[c] == s)
          lsq_transfer(ng, t.X.data(), &t.c_z[c * 3], &t.c_n[c * 3], h, t.K, &t.z_idx[c * t.K],
                       &t.z_w0[c * t.K], &t.z_wg[c * t.K * 3]);
#pragma omp parallel for schedule(dynamic, 256)
      for (int64_t j = 0; j < m; ++j) {
        const int64_t q = off + j;
        std::vector<double> w0(t.Kn);
        lsq_transfer(ng, t.X.data(), &t.X[q * 3], &t.nrm[q * 3], h, t.Kn, &t.q_idx[q * t.Kn], w0.data(),
                     &t.q_wg[q * t.Kn * 3]);
      }
    }
  }

  // -- extrapolation stencils: ranked candidates, greedy rank-raising selection
  t.S = d == 2 ? 6 : 10;
  const int S = t.S;
  t.st_lin.resize(M * S);
  t.st_r.resize(M * S * d);
  t.st_wgrad.resize(M * S * d);
  t.st_chi.resize(M * S);
  std::vector<std::string> errors(1);
  bool fail = false;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t qi = 0; qi < M; ++qi) {
    if (fail) continue;
    const double *q = &t.X[qi * d];
    int64_t kc[3];
    for (int a = 0; a < d; ++a) kc[a] = (int64_t)std::floor((q[a] - lo) / h);
    const int nc = d == 2 ? 16 : 64;
    struct Cand { double d2; int64_t lin; double r[3]; };
    std::vector<Cand> cand(nc);
    bool bad = false;
    for (int ci = 0; ci < nc; ++ci) {
      int64_t k[3];
      int rem = ci;
      // candidate order does not matter: ranking below is total
      for (int a = d - 1; a >= 0; --a) {
        k[a] = kc[a] - 1 + rem % 4;
        rem /= 4;
      }
      Cand &cd = cand[ci];
      cd.d2 = 0.0;
      int64_t k0[3];
      for (int a = 0; a < d; ++a) {
        if (k[a] < 1 || k[a] > grid.cells - 1) bad = true;
        const double x = lo + (double)k[a] * h;
        cd.r[a] = (x - q[a]) / h;
        k0[a] = k[a] - 1;
      }
      for (int a = 0; a < d; ++a) cd.d2 += cd.r[a] * cd.r[a];
      cd.lin = lin_of(k0, d, N);
    }
    if (bad) {
      fail = true;
      continue;
    }
    std::sort(cand.begin(), cand.end(), [](const Cand &A, const Cand &B) {
      return A.d2 < B.d2 || (A.d2 == B.d2 && A.lin < B.lin);
    });
    std::vector<Cand> ranked;
    size_t g0 = 0;
    for (size_t i = 1; i <= cand.size(); ++i)
      if (i == cand.size() || cand[i].d2 - cand[g0].d2 > kTieTol) {
        std::vector<Cand> grp(cand.begin() + g0, cand.begin() + i);
        std::sort(grp.begin(), grp.end(), [](const Cand &A, const Cand &B) { return A.lin < B.lin; });
        ranked.insert(ranked.end(), grp.begin(), grp.end());
        g0 = i;
      }
    std::vector<std::vector<double>> Q;
    std::vector<int> acc;
    for (size_t i = 0; i < ranked.size() && (int)acc.size() < S; ++i) {
      std::vector<double> v(S), w(S);
      quad_basis(d, ranked[i].r, v.data());
      w = v;
      for (int pass = 0; pass < 2; ++pass)
        for (const auto &qv : Q) {
          double dot = 0.0;
          for (int k = 0; k < S; ++k) dot += qv[k] * w[k];
          for (int k = 0; k < S; ++k) w[k] -= dot * qv[k];
        }
      double nw = 0.0, nv = 0.0;
      for (int k = 0; k < S; ++k) {
        nw += w[k] * w[k];
        nv += v[k] * v[k];
      }
      nw = std::sqrt(nw);
      nv = std::sqrt(nv);
      if (nw > kRankTol * nv) {
        for (int k = 0; k < S; ++k) w[k] /= nw;
        Q.push_back(w);
        acc.push_back((int)i);
      }
    }
    if ((int)acc.size() < S) {
      fail = true;
      continue;
    }
    std::vector<double> V((size_t)S * S), Vinv;
    for (int j = 0; j < S; ++j) quad_basis(d, ranked[acc[j]].r, &V[(size_t)j * S]);
    if (!invert(V, S, Vinv)) {
      fail = true;
      continue;
    }
    for (int j = 0; j < S; ++j) {
      const Cand &cd = ranked[acc[j]];
      t.st_lin[qi * S + j] = cd.lin;
      t.st_chi[qi * S + j] = t.inside[cd.lin] ? 0 : 1;
      for (int a = 0; a < d; ++a) {
        t.st_r[(qi * S + j) * d + a] = cd.r[a] * h;
        t.st_wgrad[(qi * S + j) * d + a] = Vinv[(size_t)(1 + a) * S + j] / h;
      }
    }
  }
  if (fail) throw GeometryError{"extrapolation stencil reaches the box or is rank-deficient"};

  // -- irregular nodes
  t.irregular.clear();
  t.irregular.insert(t.irregular.end(), t.c_pin.begin(), t.c_pin.end());
  t.irregular.insert(t.irregular.end(), t.c_pout.begin(), t.c_pout.end());
  std::sort(t.irregular.begin(), t.irregular.end());
  t.irregular.erase(std::unique(t.irregular.begin(), t.irregular.end()), t.irregular.end());
  // the caller's point / triangle arrays are only valid during setup
  for (auto &s : t.surf) {
    s.points = nullptr;
    s.tris = nullptr;
  }
}

}  // namespace kfbi
