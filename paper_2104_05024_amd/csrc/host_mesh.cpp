// Closed 3D surfaces given as triangle meshes.  The paper builds local coordinate systems on
// the boundary's triangle grid for normals, tangents and curvatures (Sec. 6, 3D jumps, the
// six boundary points of a triangle; Sec. 7, Example 4).  Nodes are the vertices.
//
// For a graph zeta = w(xi, eta) over a frame (t1, t2, n0) with the tissue below it, the level
// set phi = zeta - w has n = (-w_xi, -w_eta, 1)/q, q = |grad phi|, and the shape operator
// W = P_n Hess(phi) P_n / q with Hess(phi) = -Hess(w) in the tangent block.
#include <algorithm>
#include <cmath>
#include <unordered_map>

#include "host_tables.h"

namespace kfbi {
namespace {

void cross3(const double *a, const double *b, double *c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

double norm3(const double *a) { return std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]); }

// n, W of the graph zeta = c0 + c1 xi + c2 eta + c3 xi^2 + c4 xi eta + c5 eta^2 in the frame R
// (row-major 3x3 whose columns are t1, t2, n0) at (xi, eta).
void graph_geometry(const double *R, const double *c, double xi, double eta, double *n, double *W) {
  const double wx = c[1] + 2 * c[3] * xi + c[4] * eta;
  const double wy = c[2] + c[4] * xi + 2 * c[5] * eta;
  const double g[3] = {-wx, -wy, 1.0};
  const double q = norm3(g);
  const double nf[3] = {g[0] / q, g[1] / q, g[2] / q};
  const double Hf[9] = {-2 * c[3], -c[4], 0.0, -c[4], -2 * c[5], 0.0, 0.0, 0.0, 0.0};
  double P[9], T[9], Wf[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) P[i * 3 + j] = (i == j ? 1.0 : 0.0) - nf[i] * nf[j];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += P[i * 3 + k] * Hf[k * 3 + j];
      T[i * 3 + j] = acc;
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += T[i * 3 + k] * P[k * 3 + j];
      Wf[i * 3 + j] = acc / q;
    }
  for (int i = 0; i < 3; ++i) {
    double acc = 0.0;
    for (int k = 0; k < 3; ++k) acc += R[i * 3 + k] * nf[k];
    n[i] = acc;
  }
  double RW[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += R[i * 3 + k] * Wf[k * 3 + j];
      RW[i * 3 + j] = acc;
    }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc += RW[i * 3 + k] * R[j * 3 + k];
      W[i * 3 + j] = acc;
    }
}

// Least squares min |A x - b| (A: rows x cols, rows >= cols) by Householder QR; false if
// rank-deficient.
bool lsq(std::vector<double> A, int rows, int cols, std::vector<double> b, double *x) {
  for (int k = 0; k < cols; ++k) {
    double nrm = 0.0;
    for (int i = k; i < rows; ++i) nrm += A[i * cols + k] * A[i * cols + k];
    nrm = std::sqrt(nrm);
    if (nrm == 0.0) return false;
    const double alpha = A[k * cols + k] > 0 ? -nrm : nrm;
    std::vector<double> v(rows, 0.0);
    for (int i = k; i < rows; ++i) v[i] = A[i * cols + k];
    v[k] -= alpha;
    double vv = 0.0;
    for (int i = k; i < rows; ++i) vv += v[i] * v[i];
    if (vv == 0.0) continue;
    for (int j = k; j < cols; ++j) {
      double d = 0.0;
      for (int i = k; i < rows; ++i) d += v[i] * A[i * cols + j];
      const double f = 2.0 * d / vv;
      for (int i = k; i < rows; ++i) A[i * cols + j] -= f * v[i];
    }
    double d = 0.0;
    for (int i = k; i < rows; ++i) d += v[i] * b[i];
    const double f = 2.0 * d / vv;
    for (int i = k; i < rows; ++i) b[i] -= f * v[i];
  }
  double amax = 0.0;
  for (int k = 0; k < cols; ++k) amax = std::max(amax, std::fabs(A[k * cols + k]));
  for (int k = cols - 1; k >= 0; --k) {
    if (std::fabs(A[k * cols + k]) <= 1e-12 * amax) return false;
    double acc = b[k];
    for (int j = k + 1; j < cols; ++j) acc -= A[k * cols + j] * x[j];
    x[k] = acc / A[k * cols + k];
  }
  return true;
}

// Weights of grad_Gamma psi on the graph zeta = w(xi, eta) (frame R, coefficients c) at
// (xi, eta) from the weights wx, wy of psi_xi, psi_eta: [X_xi X_eta] g^-1 (psi_xi, psi_eta)
// with the tangents X_xi = t1 + w_xi n0, X_eta = t2 + w_eta n0 and their metric g.
void grad_weights(const double *R, const double *c, double xi, double eta, const double *wx, const double *wy,
                  int k, double *wg) {
  const double wxi = c[1] + 2 * c[3] * xi + c[4] * eta, weta = c[2] + c[4] * xi + 2 * c[5] * eta;
  double Xx[3], Xy[3];
  for (int a = 0; a < 3; ++a) {
    Xx[a] = R[a * 3 + 0] + wxi * R[a * 3 + 2];
    Xy[a] = R[a * 3 + 1] + weta * R[a * 3 + 2];
  }
  const double g00 = Xx[0] * Xx[0] + Xx[1] * Xx[1] + Xx[2] * Xx[2];
  const double g01 = Xx[0] * Xy[0] + Xx[1] * Xy[1] + Xx[2] * Xy[2];
  const double g11 = Xy[0] * Xy[0] + Xy[1] * Xy[1] + Xy[2] * Xy[2];
  const double det = g00 * g11 - g01 * g01;
  const double i00 = g11 / det, i01 = -g01 / det, i11 = g00 / det;
  for (int j = 0; j < k; ++j) {
    const double ax = i00 * wx[j] + i01 * wy[j], ay = i01 * wx[j] + i11 * wy[j];
    for (int a = 0; a < 3; ++a) wg[j * 3 + a] = ax * Xx[a] + ay * Xy[a];
  }
}

}  // namespace

void TriMesh3::crossing_transfer(int64_t t, const double *z, int64_t *idx, double *w0, double *wg) const {
  const Patch &P = patch[t];
  const int64_t id[6] = {F[3 * t], F[3 * t + 1], F[3 * t + 2], opp[3 * t], opp[3 * t + 1], opp[3 * t + 2]};
  double L = 0.0, d[6][3];
  for (int k = 0; k < 6; ++k)
    for (int a = 0; a < 3; ++a) d[k][a] = V[3 * id[k] + a] - P.o[a];
  for (int k = 0; k < 3; ++k) L = std::max(L, norm3(d[k]));
  // A (rows: [1, x, y, x^2, xy, y^2] at the six points, scaled coordinates); the weights of
  // psi and its derivatives at z solve A^T w = basis(z)
  std::vector<double> At(36);
  for (int k = 0; k < 6; ++k) {
    const double x = (d[k][0] * P.R[0] + d[k][1] * P.R[3] + d[k][2] * P.R[6]) / L;
    const double y = (d[k][0] * P.R[1] + d[k][1] * P.R[4] + d[k][2] * P.R[7]) / L;
    const double row[6] = {1.0, x, y, x * x, x * y, y * y};
    for (int j = 0; j < 6; ++j) At[j * 6 + k] = row[j];
  }
  double q[3];
  for (int k = 0; k < 3; ++k) {
    double acc = 0.0;
    for (int a = 0; a < 3; ++a) acc += P.R[a * 3 + k] * (z[a] - P.o[a]);
    q[k] = acc;
  }
  const double x = q[0] / L, y = q[1] / L;
  const std::vector<double> b = {1.0, x, y, x * x, x * y, y * y};
  const std::vector<double> bx = {0.0, 1.0 / L, 0.0, 2 * x / L, y / L, 0.0};
  const std::vector<double> by = {0.0, 0.0, 1.0 / L, 0.0, x / L, 2 * y / L};
  double wx[6], wy[6];
  if (!lsq(At, 6, 6, b, w0) || !lsq(At, 6, 6, bx, wx) || !lsq(At, 6, 6, by, wy))
    throw GeometryError{"degenerate six-point local coordinate system"};
  grad_weights(P.R, P.c, q[0], q[1], wx, wy, 6, wg);
  for (int k = 0; k < 6; ++k) idx[k] = id[k];
}

int TriMesh3::vertex_transfer(int64_t i, int kmax, int64_t *idx, double *wg) const {
  const double *acc = &vacc[3 * i];
  const double an = norm3(acc);
  const double n0[3] = {acc[0] / an, acc[1] / an, acc[2] / an};
  int mi = 0;
  for (int a = 1; a < 3; ++a)
    if (std::fabs(n0[a]) < std::fabs(n0[mi])) mi = a;
  double e[3] = {0, 0, 0}, t1[3], t2[3];
  e[mi] = 1.0;
  cross3(e, n0, t1);
  const double l1 = norm3(t1);
  for (double &v : t1) v /= l1;
  cross3(n0, t1, t2);
  double R[9];
  for (int a = 0; a < 3; ++a) {
    R[a * 3 + 0] = t1[a];
    R[a * 3 + 1] = t2[a];
    R[a * 3 + 2] = n0[a];
  }
  // nearest one-ring neighbours (squared distance, then index)
  std::vector<std::pair<double, int64_t>> nb;
  for (int64_t s = nbr_ptr[i]; s < nbr_ptr[i + 1]; ++s) {
    const int64_t j = nbr[s];
    const double dx = V[3 * j] - V[3 * i], dy = V[3 * j + 1] - V[3 * i + 1], dz = V[3 * j + 2] - V[3 * i + 2];
    nb.push_back({(dx * dx + dy * dy) + dz * dz, j});
  }
  std::sort(nb.begin(), nb.end());
  if ((int)nb.size() > kmax - 1) nb.resize(kmax - 1);
  const int kn = (int)nb.size(), k = kn + 1;
  // graph coefficients over the selected neighbours
  std::vector<double> G((size_t)kn * 5), zeta(kn);
  for (int r = 0; r < kn; ++r) {
    const int64_t j = nb[r].second;
    const double d[3] = {V[3 * j] - V[3 * i], V[3 * j + 1] - V[3 * i + 1], V[3 * j + 2] - V[3 * i + 2]};
    const double xi = d[0] * t1[0] + d[1] * t1[1] + d[2] * t1[2];
    const double eta = d[0] * t2[0] + d[1] * t2[1] + d[2] * t2[2];
    zeta[r] = d[0] * n0[0] + d[1] * n0[1] + d[2] * n0[2];
    const double row[5] = {xi, eta, xi * xi, xi * eta, eta * eta};
    for (int c5 = 0; c5 < 5; ++c5) G[(size_t)r * 5 + c5] = row[c5];
  }
  double c[6] = {0, 0, 0, 0, 0, 0};
  if (!lsq(G, kn, 5, zeta, c + 1)) throw GeometryError{"degenerate vertex neighbourhood in the mesh"};
  // psi fit [1, x, y, x^2, xy, y^2] over the vertex and the neighbours (scaled coordinates);
  // column j of pinv(A) is the least-squares solution for the unit vector e_j
  idx[0] = i;
  for (int r = 0; r < kn; ++r) idx[r + 1] = nb[r].second;
  double L = 0.0, xy[10][2];
  for (int r = 0; r < k; ++r) {
    const int64_t j = idx[r];
    const double d[3] = {V[3 * j] - V[3 * i], V[3 * j + 1] - V[3 * i + 1], V[3 * j + 2] - V[3 * i + 2]};
    L = std::max(L, norm3(d));
    xy[r][0] = d[0] * t1[0] + d[1] * t1[1] + d[2] * t1[2];
    xy[r][1] = d[0] * t2[0] + d[1] * t2[1] + d[2] * t2[2];
  }
  std::vector<double> A((size_t)k * 6);
  for (int r = 0; r < k; ++r) {
    const double x = xy[r][0] / L, y = xy[r][1] / L;
    const double row[6] = {1.0, x, y, x * x, x * y, y * y};
    for (int j = 0; j < 6; ++j) A[(size_t)r * 6 + j] = row[j];
  }
  double wx[10], wy[10];
  for (int r = 0; r < k; ++r) {
    std::vector<double> ej(k, 0.0);
    ej[r] = 1.0;
    double col[6];
    if (!lsq(A, k, 6, ej, col)) throw GeometryError{"degenerate vertex neighbourhood in the mesh"};
    wx[r] = col[1] / L;
    wy[r] = col[2] / L;
  }
  grad_weights(R, c, 0.0, 0.0, wx, wy, k, wg);
  return k;
}

void TriMesh3::build(const double *pts, int64_t m_, const int32_t *tris, int64_t nt_, int orient) {
  m = m_;
  nt = nt_;
  V.assign(pts, pts + 3 * m);
  F.resize(3 * nt);
  for (int64_t i = 0; i < 3 * nt; ++i) {
    if (tris[i] < 0 || tris[i] >= m) throw GeometryError{"mesh triangle index out of range"};
    F[i] = tris[i];
  }
  // directed edges: each must appear once, and its reverse once (closed, consistently oriented)
  std::unordered_map<int64_t, int64_t> half;   // p * m + q -> 3 t + e
  half.reserve(6 * nt);
  for (int64_t t = 0; t < nt; ++t)
    for (int e = 0; e < 3; ++e) {
      const int64_t p = F[3 * t + e], q = F[3 * t + (e + 1) % 3];
      if (!half.emplace(p * m + q, 3 * t + e).second) throw GeometryError{"mesh is not consistently oriented"};
    }
  opp.resize(3 * nt);
  for (int64_t t = 0; t < nt; ++t)
    for (int e = 0; e < 3; ++e) {
      const int64_t p = F[3 * t + e], q = F[3 * t + (e + 1) % 3];
      const auto it = half.find(q * m + p);
      if (it == half.end()) throw GeometryError{"mesh is not closed"};
      const int64_t t2 = it->second / 3, e2 = it->second % 3;
      opp[3 * t + e] = F[3 * t2 + (e2 + 2) % 3];
    }
  cr.resize(3 * nt);
  double vol = 0.0;
  for (int64_t t = 0; t < nt; ++t) {
    const double *a = &V[3 * F[3 * t]], *b = &V[3 * F[3 * t + 1]], *c = &V[3 * F[3 * t + 2]];
    const double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, w[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    cross3(u, w, &cr[3 * t]);
    vol += a[0] * cr[3 * t] + a[1] * cr[3 * t + 1] + a[2] * cr[3 * t + 2];
  }
  sigma = (double)orient * (vol > 0.0 ? 1.0 : -1.0);
  for (auto &v : cr) v *= sigma;
  vacc.assign(3 * m, 0.0);
  for (int k = 0; k < 3; ++k)          // corner by corner, triangles in order
    for (int64_t t = 0; t < nt; ++t)
      for (int a = 0; a < 3; ++a) vacc[3 * F[3 * t + k] + a] += cr[3 * t + a];
  // one-rings
  std::vector<std::vector<int64_t>> ring(m);
  for (int64_t t = 0; t < nt; ++t)
    for (int e = 0; e < 3; ++e) {
      ring[F[3 * t + e]].push_back(F[3 * t + (e + 1) % 3]);
      ring[F[3 * t + e]].push_back(F[3 * t + (e + 2) % 3]);
    }
  nbr_ptr.assign(m + 1, 0);
  nbr.clear();
  for (int64_t i = 0; i < m; ++i) {
    auto &r = ring[i];
    std::sort(r.begin(), r.end());
    r.erase(std::unique(r.begin(), r.end()), r.end());
    if (r.size() < 5) throw GeometryError{"mesh vertex with fewer than five neighbours"};
    nbr.insert(nbr.end(), r.begin(), r.end());
    nbr_ptr[i + 1] = (int64_t)nbr.size();
  }
  // six-point patches
  patch.resize(nt);
  for (int64_t t = 0; t < nt; ++t) {
    Patch &P = patch[t];
    const int64_t idx[6] = {F[3 * t], F[3 * t + 1], F[3 * t + 2], opp[3 * t], opp[3 * t + 1], opp[3 * t + 2]};
    for (int a = 0; a < 3; ++a) P.o[a] = (V[3 * idx[0] + a] + V[3 * idx[1] + a] + V[3 * idx[2] + a]) / 3.0;
    const double cn = norm3(&cr[3 * t]);
    const double n0[3] = {cr[3 * t] / cn, cr[3 * t + 1] / cn, cr[3 * t + 2] / cn};
    double t1[3] = {V[3 * idx[1]] - V[3 * idx[0]], V[3 * idx[1] + 1] - V[3 * idx[0] + 1],
                    V[3 * idx[1] + 2] - V[3 * idx[0] + 2]};
    const double l1 = norm3(t1);
    for (double &v : t1) v /= l1;
    double t2[3];
    cross3(n0, t1, t2);
    for (int a = 0; a < 3; ++a) {
      P.R[a * 3 + 0] = t1[a];
      P.R[a * 3 + 1] = t2[a];
      P.R[a * 3 + 2] = n0[a];
    }
    double L = 0.0, d[6][3];
    for (int k = 0; k < 6; ++k)
      for (int a = 0; a < 3; ++a) d[k][a] = V[3 * idx[k] + a] - P.o[a];
    for (int k = 0; k < 3; ++k) L = std::max(L, norm3(d[k]));
    std::vector<double> A(36), b(6);
    for (int k = 0; k < 6; ++k) {
      const double xi = (d[k][0] * t1[0] + d[k][1] * t1[1] + d[k][2] * t1[2]) / L;
      const double eta = (d[k][0] * t2[0] + d[k][1] * t2[1] + d[k][2] * t2[2]) / L;
      b[k] = d[k][0] * n0[0] + d[k][1] * n0[1] + d[k][2] * n0[2];
      const double row[6] = {1.0, xi, eta, xi * xi, xi * eta, eta * eta};
      for (int j = 0; j < 6; ++j) A[k * 6 + j] = row[j];
    }
    if (!lsq(A, 6, 6, b, P.c)) throw GeometryError{"degenerate six-point local coordinate system"};
    P.c[1] /= L;
    P.c[2] /= L;
    P.c[3] /= L * L;
    P.c[4] /= L * L;
    P.c[5] /= L * L;
  }
}

void TriMesh3::vertex_geometry(int64_t i, double *n, double *W) const {
  const double *acc = &vacc[3 * i];   // area-weighted normal of the incident triangles
  const double an = norm3(acc);
  const double n0[3] = {acc[0] / an, acc[1] / an, acc[2] / an};
  int mi = 0;
  for (int a = 1; a < 3; ++a)
    if (std::fabs(n0[a]) < std::fabs(n0[mi])) mi = a;
  double e[3] = {0, 0, 0}, t1[3], t2[3];
  e[mi] = 1.0;
  cross3(e, n0, t1);
  const double l1 = norm3(t1);
  for (double &v : t1) v /= l1;
  cross3(n0, t1, t2);
  double R[9];
  for (int a = 0; a < 3; ++a) {
    R[a * 3 + 0] = t1[a];
    R[a * 3 + 1] = t2[a];
    R[a * 3 + 2] = n0[a];
  }
  const int k = (int)(nbr_ptr[i + 1] - nbr_ptr[i]);
  std::vector<double> A((size_t)k * 5), b(k);
  for (int r = 0; r < k; ++r) {
    const int64_t j = nbr[nbr_ptr[i] + r];
    const double d[3] = {V[3 * j] - V[3 * i], V[3 * j + 1] - V[3 * i + 1], V[3 * j + 2] - V[3 * i + 2]};
    const double xi = d[0] * t1[0] + d[1] * t1[1] + d[2] * t1[2];
    const double eta = d[0] * t2[0] + d[1] * t2[1] + d[2] * t2[2];
    b[r] = d[0] * n0[0] + d[1] * n0[1] + d[2] * n0[2];
    const double row[5] = {xi, eta, xi * xi, xi * eta, eta * eta};
    for (int j2 = 0; j2 < 5; ++j2) A[(size_t)r * 5 + j2] = row[j2];
  }
  double c[6] = {0, 0, 0, 0, 0, 0};
  if (!lsq(A, k, 5, b, c + 1)) throw GeometryError{"degenerate vertex neighbourhood in the mesh"};
  graph_geometry(R, c, 0.0, 0.0, n, W);
}

void TriMesh3::patch_geometry(int64_t t, const double *z, double *n, double *W) const {
  const Patch &P = patch[t];
  double q[3];
  for (int k = 0; k < 3; ++k) {
    double acc = 0.0;
    for (int a = 0; a < 3; ++a) acc += P.R[a * 3 + k] * (z[a] - P.o[a]);
    q[k] = acc;
  }
  graph_geometry(P.R, P.c, q[0], q[1], n, W);
}

double TriMesh3::onto_patch(int64_t t, const double *p, int axis, double s_flat, double h, double *n,
                            double *W) const {
  const Patch &P = patch[t];
  const double *c = P.c;
  double q0[3], dq[3];
  for (int k = 0; k < 3; ++k) {
    double acc = 0.0;
    for (int a = 0; a < 3; ++a) acc += P.R[a * 3 + k] * (p[a] - P.o[a]);
    q0[k] = acc;
    dq[k] = P.R[axis * 3 + k];
  }
  const double x0 = q0[0], y0 = q0[1], z0 = q0[2], dx = dq[0], dy = dq[1], dz = dq[2];
  // zeta(s) - w(xi(s), eta(s)) = A2 s^2 + A1 s + A0 along the line
  const double A2 = -(c[3] * dx * dx + c[4] * dx * dy + c[5] * dy * dy);
  const double A1 = dz - (c[1] * dx + c[2] * dy + 2 * c[3] * x0 * dx + c[4] * (x0 * dy + y0 * dx) + 2 * c[5] * y0 * dy);
  const double A0 = z0 - (c[0] + c[1] * x0 + c[2] * y0 + c[3] * x0 * x0 + c[4] * x0 * y0 + c[5] * y0 * y0);
  double roots[2];
  int nr = 0;
  if (A2 != 0.0) {
    const double disc = A1 * A1 - 4.0 * A2 * A0;
    if (disc >= 0.0) {
      const double qq = -0.5 * (A1 + (A1 >= 0 ? std::sqrt(disc) : -std::sqrt(disc)));
      roots[nr++] = qq / A2;
      if (qq != 0.0) roots[nr++] = A0 / qq;
    }
  } else if (A1 != 0.0) {
    roots[nr++] = -A0 / A1;
  }
  double s = s_flat;
  if (nr > 0) {
    s = roots[0];
    if (nr == 2 && std::fabs(roots[1] - s_flat) < std::fabs(roots[0] - s_flat)) s = roots[1];
  }
  s = std::min(h, std::max(0.0, s));
  double z[3] = {p[0], p[1], p[2]};
  z[axis] += s;
  patch_geometry(t, z, n, W);
  return s;
}

void TriMesh3::grid_line_hits(int axis, double lo, double h, int64_t N,
                              std::vector<std::vector<std::pair<double, int64_t>>> &out) const {
  out.assign((size_t)N * N, {});
  const int bx = axis == 0 ? 1 : 0, cx = axis == 2 ? 1 : 2;
  for (int64_t t = 0; t < nt; ++t) {
    double P[3][3];   // projected (b, c) and the coordinate along the axis
    for (int k = 0; k < 3; ++k) {
      const double *v = &V[3 * F[3 * t + k]];
      P[k][0] = v[bx];
      P[k][1] = v[cx];
      P[k][2] = v[axis];
    }
    double s2 = (P[1][0] - P[0][0]) * (P[2][1] - P[0][1]) - (P[1][1] - P[0][1]) * (P[2][0] - P[0][0]);
    if (s2 == 0.0) continue;
    if (s2 < 0) {
      for (int a = 0; a < 3; ++a) std::swap(P[1][a], P[2][a]);
      s2 = -s2;
    }
    const double lb = std::min({P[0][0], P[1][0], P[2][0]}), hb = std::max({P[0][0], P[1][0], P[2][0]});
    const double lc = std::min({P[0][1], P[1][1], P[2][1]}), hc = std::max({P[0][1], P[1][1], P[2][1]});
    const int64_t kb0 = std::max<int64_t>(0, (int64_t)std::floor((lb - lo) / h) - 2);
    const int64_t kb1 = std::min<int64_t>(N - 1, (int64_t)std::ceil((hb - lo) / h));
    const int64_t kc0 = std::max<int64_t>(0, (int64_t)std::floor((lc - lo) / h) - 2);
    const int64_t kc1 = std::min<int64_t>(N - 1, (int64_t)std::ceil((hc - lo) / h));
    for (int64_t ic = kc0; ic <= kc1; ++ic) {
      const double yc = lo + h * (double)(ic + 1);
      if (yc < lc || yc > hc) continue;
      for (int64_t ib = kb0; ib <= kb1; ++ib) {
        const double yb = lo + h * (double)(ib + 1);
        if (yb < lb || yb > hb) continue;
        double lam[3];
        bool in = true;
        for (int e = 0; e < 3 && in; ++e) {
          const double *A = P[(e + 1) % 3], *B = P[(e + 2) % 3];
          const double eb = B[0] - A[0], ec = B[1] - A[1];
          const double E = eb * (yc - A[1]) - ec * (yb - A[0]);
          // a point on an edge belongs to the triangle for which the edge points down (or +b)
          if (E < 0 || (E == 0 && !(ec < 0 || (ec == 0 && eb > 0)))) in = false;
          lam[e] = E;
        }
        if (!in) continue;
        const double x = (lam[0] * P[0][2] + lam[1] * P[1][2] + lam[2] * P[2][2]) / s2;
        out[(size_t)ic * N + ib].push_back({x, t});
      }
    }
  }
  for (auto &ln : out) std::sort(ln.begin(), ln.end());
}

}  // namespace kfbi
