// Batched two-dimensional Neumann problems: size groups, work lists, lockstep GMRES.
#pragma once
#include <memory>
#include <vector>

#include "../../include/kfbi.h"
#include "device.h"

namespace kfbi {

// one problem's fields inside the group buffers, for packing caller arrays
struct PackItem {
  double *fpad, *work;
  int64_t N, P;
};

struct Group {
  int Mfft = 0, N = 0;
  int64_t cs = 0;              // padded field size of one problem (N rows of pitch Mfft)
  std::vector<int> members;    // problem indices, in slot order
  double *rhs64 = nullptr, *fpad64 = nullptr, *work64 = nullptr;
  float *rhs32 = nullptr, *fpad32 = nullptr, *work32 = nullptr;
  ModeParams *msv = nullptr;   // per-slot mode parameters (device)
  int tile_w[2][3] = {{1, 1, 1}, {1, 1, 1}};   // autotuned tile widths [FP64 / FP32][x, -, last]
  template <typename T>
  T *rhs() const;
  template <typename T>
  T *work() const;
};
template <>
inline double *Group::rhs<double>() const { return rhs64; }
template <>
inline float *Group::rhs<float>() const { return rhs32; }
template <>
inline double *Group::work<double>() const { return work64; }
template <>
inline float *Group::work<float>() const { return work32; }

struct Batch {
  static constexpr int kMaxRestart = 64;
  int np = 0;
  std::vector<std::unique_ptr<DevProblem>> probs;
  std::vector<Group> groups;
  std::vector<int> group_of, slot_of;
  std::vector<int64_t> off, goff;      // prefix sums of M_p (interface) and N_p^2 (grid)
  int64_t L = 0;                       // total interface nodes
  int16_t *pid = nullptr;              // problem of every concatenated interface entry
  int64_t *off_dev = nullptr, *goff_dev = nullptr, *cum_nc = nullptr, *cum_irr = nullptr;
  BatchCounts counts;
  BatchItem<double> *items64 = nullptr;
  BatchItem<float> *items32 = nullptr;
  PackItem *packs = nullptr;
  double *V = nullptr, *vin = nullptr, *w = nullptr, *r = nullptr, *d = nullptr, *t = nullptr, *gp = nullptr;
  double *x = nullptr, *dx = nullptr;
  double *hcols = nullptr, *hhost = nullptr, *ydev = nullptr, *sdev = nullptr, *nrm = nullptr;
  int *jdev = nullptr, *jhost = nullptr;
  int *seqdev = nullptr, *seqhost = nullptr;   // step counter polled by the host (as the solver's)
  int seq_next = 0;
  void host_wait(hipStream_t st);
  bool use_graph = true;
  // box solves of all size groups as one launch per pass (box_solve_multi) when every group's
  // size is 64..1024; otherwise, or when switched off, one launch per group and pass
  bool merged = true;
  bool mergeable() const;
  template <typename T>
  void box_all(bool from_fpad, hipStream_t st);   // every group: src (rhs, or fpad if from_fpad) -> work
  void drop_graphs();                              // the captured steps are captured again when next used
  hipStream_t cap = nullptr;           // capture stream (the caller's stream may be the null stream)
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  int graph_m[2] = {0, 0};

  void init(int n, const kfbi_interface *ifaces, const kfbi_grid *grids, const kfbi_coeffs *coeffs);
  void release();
  template <typename T>
  BatchItem<T> *items() const;
  // A psi for every problem with the grid side (correction, box solve) in T; the density side
  // (jumps, extrapolation fits) is FP64 in both, and so are the vectors
  template <typename T>
  void matvec(const double *in, double *out, hipStream_t st);
  void apply_vec(int prec, const double *in, double *out, hipStream_t st);
  // FP32 vectors at the boundary (converted to and from FP64 around the FP32 product)
  void apply_f32(const float *in, float *out, hipStream_t st);
  void seg_norms(const double *v, std::vector<double> &out, hipStream_t st);
  void arnoldi_step(int prec, int m, hipStream_t st);
  void run_step(int prec, int m, hipStream_t st);
  void gmres(int prec, const double *b, double *x, bool x_zero, const std::vector<double> &tol, int restart,
             int maxit, std::vector<int> &its, int &matvecs, std::vector<double> &res, hipStream_t st);
  void pack(const double *plain, int which, bool to_padded, hipStream_t st);
  int solve(const double *g, const double *f, double *u, double *psi, const kfbi_solve_opts &o,
            kfbi_solve_info *info, hipStream_t st);
};
template <>
inline BatchItem<double> *Batch::items<double>() const { return items64; }
template <>
inline BatchItem<float> *Batch::items<float>() const { return items32; }

}  // namespace kfbi
