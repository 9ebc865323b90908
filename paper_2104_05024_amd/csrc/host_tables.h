// Host-side static tables of one KFBI problem (FP64).  Built once by kfbi_setup.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/kfbi.h"

namespace kfbi {

constexpr double kSideTol = 1e-12;   // grid nodes with phi <= kSideTol lie in the tissue
constexpr double kTieTol = 1e-9;     // squared-distance ties (units of h^2) in stencil ranking
constexpr double kRankTol = 1e-6;    // relative residual for accepting a stencil node
constexpr int kLsqNodes = 10;        // nodes of the 3D least-squares density fit

struct GeometryError {
  std::string what;
};

struct HostTables {
  int dim = 0, ncomp = 1, cells = 0;
  int64_t N = 0, M = 0;
  double lo = 0, hi = 0, h = 0, kappa = 0;
  double D[2][3] = {{0}};
  std::vector<kfbi_surface> surf;          // descriptors (points / tris pointers cleared after setup)
  std::vector<int64_t> offsets;            // first node of each surface (+ total)

  std::vector<double> X, nrm, W;           // nodes: M*d, M*d, M*d*d
  std::vector<int8_t> inside;              // N^d, 1 = tissue

  int64_t nc = 0;                          // grid-line intersections
  std::vector<int64_t> c_surf, c_axis, c_pin, c_pout;
  std::vector<double> c_z, c_n, c_W;       // nc*d, nc*d, nc*d*d
  std::vector<double> c_t;                 // nc: spline parameter (spline curves), NaN otherwise

  int K = 0, Kn = 0;                       // transfer stencil sizes (crossings / nodes)
  std::vector<int64_t> z_idx, q_idx;       // nc*K, M*Kn
  std::vector<double> z_w0, z_wg, q_wg;    // nc*K, nc*K*d, M*Kn*d

  int S = 0;                               // extrapolation stencil size (6 / 10)
  std::vector<int64_t> st_lin;             // M*S linear interior index
  std::vector<double> st_r, st_wgrad;      // M*S*d (physical offsets p_j - q), gradient weights
  std::vector<int8_t> st_chi;              // M*S, 1 = stencil node outside the tissue

  std::vector<int64_t> irregular;          // sorted linear indices
};

// Closed 2D curve through m ordered nodes: the periodic cubic spline in the node index
// (t_j = j), one cubic per piece and coordinate, a + b s + c s^2 + d s^3 for s = t - j in [0, 1].
struct SplineCurve2 {
  int64_t m = 0;
  std::vector<double> co[2];   // [coord][piece][4]
  double sigma = 1;            // n = sigma (y', -x') / |X'| points out of the tissue
  int orient = 1;

  void build(const double *pts, int64_t m, int orient);
  // position, first and second derivatives at parameter t (taken modulo m)
  void eval(double t, double *X, double *X1, double *X2) const;
  void normal_shape(double t, double *n, double *W) const;
  void tangent(double t, double *tau, double &speed) const;
  // Crossings of the grid lines {coordinate `coord` = lo + (k+1) h}, k = 0..nl-1, as
  // (parameter t, other coordinate) per line: one root per change of the predicate
  // "coordinate > line value" along each monotone part of a piece, so a curve that only
  // touches a line contributes an even number of roots.
  void grid_line_roots(int coord, double lo, double h, int64_t nl,
                       std::vector<std::vector<std::pair<double, double>>> &out) const;
};

// Closed, consistently oriented triangle mesh in 3D with the local coordinate systems of the
// method: a quadratic height function fitted over each vertex's one-ring (normals and shape
// operators at the nodes) and, per triangle, the quadratic height function through its six
// boundary points (its vertices and the three vertices across its edges) over its plane.
struct TriMesh3 {
  int64_t m = 0, nt = 0;
  std::vector<double> V;             // m*3
  std::vector<int64_t> F, opp;       // nt*3 vertices; vertex across edge e = (F[e], F[e+1])
  std::vector<double> cr;            // nt*3 area-weighted normals out of the tissue
  std::vector<double> vacc;          // m*3 sum of cr over each vertex's triangles
  std::vector<int64_t> nbr_ptr, nbr; // one-ring of each vertex (CSR, ascending)
  double sigma = 1;                  // orient * sign(enclosed volume)
  struct Patch {
    double o[3], R[9], c[6];         // origin, frame columns (t1, t2, n), height coefficients
  };
  std::vector<Patch> patch;

  // Throws GeometryError for an open, inconsistently oriented or degenerate mesh.
  void build(const double *pts, int64_t m, const int32_t *tris, int64_t nt, int orient);
  void vertex_geometry(int64_t i, double *n, double *W) const;
  void patch_geometry(int64_t t, const double *z, double *n, double *W) const;
  // Crossing of the line p + s e_axis with triangle t (flat crossing at s_flat) moved onto the
  // triangle's patch, s clamped to [0, h]; returns s and n, W there.
  double onto_patch(int64_t t, const double *p, int axis, double s_flat, double h, double *n, double *W) const;
  // psi and grad_Gamma psi at z on triangle t's patch from its six nodal values: indices (6),
  // value weights w0 (6), gradient weights wg (6 x 3).
  void crossing_transfer(int64_t t, const double *z, int64_t *idx, double *w0, double *wg) const;
  // grad_Gamma psi at vertex i from a least-squares quadratic over the vertex and its nearest
  // kmax - 1 one-ring neighbours: indices and weights (3 per index); returns the count.
  int vertex_transfer(int64_t i, int kmax, int64_t *idx, double *wg) const;
  // Crossings of the grid lines parallel to `axis` as (coordinate along the axis, triangle),
  // per line (ic * N + ib over the other two axes b < c), sorted by coordinate.
  void grid_line_hits(int axis, double lo, double h, int64_t N,
                      std::vector<std::vector<std::pair<double, int64_t>>> &out) const;
};

// Throws GeometryError on geometric failure, std::invalid_argument on bad input.
void build_host_tables(const kfbi_interface &iface, const kfbi_grid &grid, const kfbi_coeffs &co,
                       HostTables &t);

}  // namespace kfbi
