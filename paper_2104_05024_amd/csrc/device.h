// Device-side state and kernel launchers of the KFBI library (HIP, gfx950).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "host_tables.h"

namespace kfbi {

struct HipError {
  hipError_t code;
  std::string where;
};

#define KFBI_HIP(call)                                                        \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess) throw ::kfbi::HipError{e_, #call};                  \
  } while (0)

// Grid fields inside the library use a padded layout: [comp][z][y][x] with row pitch
// P = N + 1 (a power of two), so that every row starts on a 2 KB (FP64) boundary.
// Caller-visible fields use the unpadded layout (pitch N).

template <typename T>
struct PrecTables {          // per-precision device copies of the numeric tables
  // density-side tables, FP64 only (null in the FP32 set): every product takes its jumps and its
  // extrapolation fits in FP64
  T *z_A = nullptr, *z_B = nullptr;      // crossing jumps [comp][K][nc]: [u_a] = sum A psi, [u_aa] = sum B psi
  T *q_wg = nullptr;                     // node surface-gradient weights [Kn][d][M]
  T *q_c = nullptr, *q_G = nullptr;      // node jumps [comp][d + NH][M] on psi_q, [comp][d + NH][d][M] on g
  T *st_nw = nullptr, *st_r = nullptr;   // gather weights n.D_c grad [comp][S][M]; offsets [S][d][M]
  // grid-side tables, one copy per precision
  T *arm_d = nullptr, *arm_s = nullptr;  // arm offsets [narm]; s D_{c,a} / h^2 [comp][narm]
  T *tw = nullptr, *sp = nullptr;        // DST twiddles exp(-2 pi i m/M) (complex) and sin(pi n/M)
  T *rhs = nullptr, *work = nullptr;     // matvec right-hand side (zero off irregular nodes), work field
  T *xbuf = nullptr;                     // sparse matvec: x-forward output, zero outside the rhs rows
  T *ybuf = nullptr;                     // sparse matvec: y-forward output, zero in planes without rhs rows
  T *gbuf = nullptr;                     // coupled 3D FP64: x-y transform of kappa V1 (one component),
                                         // kept from a step's volume solve for its final solve
  T *jz = nullptr;                       // jumps at crossings [comp][2][nc] (written in this precision)
  T *jq = nullptr;                       // jumps at nodes [comp][d+nh][M] (FP64 set only)
};

// Per-kernel-class launch timer: HIP events recorded around each launch on the launch
// stream, without synchronising; durations are harvested when queried or when the pool fills.
struct Timer {
  static constexpr int kPairs = 2048;
  std::vector<hipEvent_t> ev;
  int used = 0;
  double total_ms = 0;
  int64_t n = 0;
  void create() {
    ev.resize(2 * kPairs);
    for (auto &e : ev) KFBI_HIP(hipEventCreate(&e));
  }
  void destroy() {
    for (auto &e : ev) (void)hipEventDestroy(e);
    ev.clear();
    used = 0;
  }
  void harvest() {
    for (int i = 0; i < used; ++i) {
      KFBI_HIP(hipEventSynchronize(ev[2 * i + 1]));
      float ms = 0;
      KFBI_HIP(hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]));
      total_ms += ms;
      ++n;
    }
    used = 0;
  }
  void tic(bool on, hipStream_t st) {
    if (!on) return;
    if (used == kPairs) harvest();
    KFBI_HIP(hipEventRecord(ev[2 * used], st));
  }
  void toc(bool on, hipStream_t st) {
    if (!on) return;
    KFBI_HIP(hipEventRecord(ev[2 * used + 1], st));
    ++used;
  }
  void reset() {
    harvest();
    total_ms = 0;
    n = 0;
  }
};

// A set of z planes as bits (plane z = bit z % 64 of word z / 64; up to 1024 planes), passed to
// kernels by value so that testing a plane needs no memory access.
struct PlaneBits {
  uint64_t w[16] = {};
};

struct DevProblem {
  HostTables ht;
  bool on_device = false;
  int dev = 0;
  int dim = 0, ncomp = 1, Mfft = 0;
  int64_t N = 0, M = 0, P = 0, nc = 0, nirr = 0, narm = 0;
  int64_t comp_stride = 0;     // padded elements per component
  int K = 0, Kn = 0, S = 0;
  double h = 0, kappa = 0, D[2][3] = {{1, 1, 1}, {1, 1, 1}};   // diagonal conductivity per component
  double lam_scale = 1;        // (2/M)^d normalisation of the inverse transforms

  // integer tables
  int32_t *z_idx = nullptr, *z_axis = nullptr, *q_idx = nullptr;
  int32_t *irr_pos = nullptr, *irr_ptr = nullptr, *arm_cross = nullptr;
  int32_t *st_pos = nullptr;   // padded index, negative (-pos-1) for stencil nodes outside the tissue
  int8_t *inside_pad = nullptr;  // padded-layout tissue mask
  // sparse matvec box solve (3D): rows of the flattened [comp][z][y] row list that carry
  // irregular nodes (in) / extrapolation-stencil nodes (out), and their [z][y] byte masks
  bool sparse = true;
  int32_t *rows_in = nullptr, *rows_out = nullptr;
  int64_t n_rows_in = 0, n_rows_out = 0;
  uint64_t *mask_in = nullptr, *mask_out = nullptr;     // [z][16] bit rows: y rows with rhs / stencil nodes
  uint8_t *planes_in = nullptr, *planes_out = nullptr;   // [z]: plane holds any rhs / stencil row
  PlaneBits planes_in_bits, planes_out_bits;             // the same sets as bits
  double *lam = nullptr;       // (4/h^2) sin^2(k pi / 2M), k = 1..N

  PrecTables<double> f64;
  PrecTables<float> f32;

  // reductions / scratch
  double *red = nullptr;       // small device scratch for dot products
  double *host_red = nullptr;  // pinned host mirror

  // tile width multiplier (1 or 2) per precision (0: FP64, 1: FP32) and pass (x, y, last axis)
  int tile_w[2][3] = {{1, 1, 1}, {1, 1, 1}};

  bool profile = false;
  Timer t_dst_x, t_dst_y, t_dst_last, t_correct, t_gather, t_jumps, t_dst_x_rows, t_dst_y_sparse, t_dst_last_sparse,
      t_dst_last_out, t_dst_x_fhn, t_dst_x_fe1, t_dst_y1, t_dst_last_anti, t_dst_last_diff, t_dst_x_be1,
      t_dst_last_comb;
  hipStream_t stream = nullptr;

  template <typename T>
  PrecTables<T> &tab();
};

template <>
inline PrecTables<double> &DevProblem::tab<double>() { return f64; }
template <>
inline PrecTables<float> &DevProblem::tab<float>() { return f32; }

// Mode solve parameters of one problem: eigenvalues (4/h^2) sin^2(k pi / 2M), k = 1..N,
// diagonal conductivities of the (one or two) components per axis, kappa, and the (2/M)^d
// factor; the mode sum of component c is sum_a D_{c,a} lambda_{k_a}.
struct ModeParams {
  const double *lam;
  double D0[3], D1[3], kappa, norm;   // conductivity per axis of component 0 and 1
};

// One two-dimensional, one-component problem of a batch as the batched interface kernels see
// it: its tables, its fields inside the size-group buffers, and its offset in the
// concatenated interface vectors.
// The density-side tables and node jumps are FP64 for both precisions (as in PrecTables).
template <typename T>
struct BatchItem {
  const int32_t *z_idx;
  const double *z_A, *z_B;
  const int32_t *irr_pos, *irr_ptr, *arm_cross;
  const T *arm_d, *arm_s;
  int64_t narm;
  const int32_t *q_idx;
  const double *q_wg, *q_c, *q_G;
  const int32_t *st_pos;
  const double *st_nw, *st_r;
  T *jz;
  double *jq;
  T *rhs, *fpad, *work;        // padded fields inside the group buffers
  int64_t M, nc, nirr, ioff;
};

// Prefix sums over the problems of a batch (device arrays of n + 1 entries) and totals.
struct BatchCounts {
  const int64_t *cum_nc = nullptr, *cum_M = nullptr, *cum_nirr = nullptr;
  int n = 0;
  int64_t tot_nc = 0, tot_M = 0, tot_nirr = 0;
};

// ---- launchers (defined in dst.hip / kfbi_kernels.hip)
// Box solve: dst = S(src). Layout flags: true = caller (unpadded) layout, false = padded.
template <typename T>
void box_solve(DevProblem &p, const T *src, bool src_plain, T *dst, bool dst_plain, hipStream_t st);

// Box solve of the matrix-vector product: rhs (padded, sparse) -> work (padded); only the
// extrapolation-stencil values of work are meaningful afterwards.
template <typename T>
void box_solve_matvec(DevProblem &p, hipStream_t st);

// Box solve of src (padded) into work when only the extrapolation-stencil values of the result
// are read afterwards (identical there to box_solve).
template <typename T>
void box_solve_stencils(DevProblem &p, const T *src, hipStream_t st);

// 1/x from the hardware reciprocal estimate refined by Newton steps (two in FP64, one in FP32):
// within an ulp or two of the IEEE quotient at a fraction of the cost of a full division.
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
__device__ __forceinline__ float recip(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// Waits until the step counter *seq_host (pinned host memory, stored by a one-thread kernel with
// a system-scope release after the work it follows) reaches expect: polls it for up to 20 ms,
// then synchronises the stream, which also reports any error.  Returns the counter's value.
int poll_step_counter(const int *seq_host, int expect, hipStream_t st);

// FitzHugh-Nagumo reaction (Sec. 7) and its two half steps in the Strang splitting (Sec. 3):
// forward Euler, and backward Euler with q eliminated and Newton on V.  inv_cm = 1 / C_m and
// inv_den = 1 / (1 + dth zeta) for the half step dth, so that no node divides by constants.
struct FhnCoef {
  double Cm, H, theta, alpha, zeta, tol;
  int maxit;
  double inv_cm, inv_den;
};

// Forward Euler over dth: (v, g) <- (v - dth I_ion(v, g) / C_m, g + dth (alpha v - zeta g)).
__device__ __forceinline__ void fhn_fe(double &v, double &g, double dth, const FhnCoef &m) {
  const double I = m.H * (g - v * (v - m.theta) * (1.0 - v));
  const double v1 = v + dth * (-I * m.inv_cm);
  const double q1 = g + dth * (m.alpha * v - m.zeta * g);
  v = v1;
  g = q1;
}

// Backward Euler over dth from (vb, g): q' = (g + dth alpha V') / (1 + dth zeta) is eliminated
// and Newton solves for V'; it stops once |F| <= tol and takes one more step.
__device__ __forceinline__ void fhn_be(double vb, double g, double dth, const FhnCoef &m, double &V, double &q) {
  const double a = dth * m.alpha * m.inv_den;
  const double qb = g * m.inv_den;
  const double c = dth * m.H * m.inv_cm;
  double x = vb;
  for (int it = 0; it < m.maxit; ++it) {
    const double cub = x * (x - m.theta) * (1.0 - x);
    const double F = x - vb + c * (qb + a * x - cub);
    const double dcub = -3.0 * x * x + 2.0 * (1.0 + m.theta) * x - m.theta;
    const double dF = 1.0 + c * (a - dcub);
    const bool ok = fabs(F) <= m.tol;
    x = x - F * recip(dF);
    if (ok) break;
  }
  V = x;
  q = qb + a * x;
}

// Pointwise state of a coupled bidomain step (caller layout, pitch N) handed to the box
// solves that carry the reaction half steps in their x passes.
struct FhnArgs {
  double *V, *q;
  const double *stim;         // I_stim or null
  double dth, kappa, beta;
  FhnCoef m;
};

// Box solves of a coupled (two-component, FP64) bidomain step whose x passes pair row r of
// component 0 with row r of component 1, so that both potentials of a node share one complex
// value and the pointwise work of the splitting rides in those passes:
//   bidomain_volume_solve: S f for f = (kappa V1, -kappa V1 + beta I), (V1, q1) the forward
//     Euler half step of (V, q), into work (extrapolation-stencil values, as
//     box_solve_stencils); V and q are left unchanged.  Without I (3D, M >= 64) the source is
//     antisymmetric and the forward x and y passes run over the one field kappa V1;
//   bidomain_final_solve: S(f + C psi) with C psi taken from rhs (launch_correct), into work;
//     with fuse_be the inverse x pass instead finishes the step: V <- 2 (u_i - u_e) - V1 and the
//     backward Euler half step from q1 into V and q, and work is left holding the y-inverse
//     output (3D, M >= 64: of u_i - u_e alone, in component 0, the only field the update
//     needs).  Each pass recomputes (V1, q1) from the unchanged (V, q).
void bidomain_volume_solve(DevProblem &p, const FhnArgs &a, hipStream_t st);
void bidomain_final_solve(DevProblem &p, const FhnArgs &a, bool fuse_be, hipStream_t st);

// Jumps from the FP64 density (FP64 weights and arithmetic); the crossing jumps are stored in T
// for the correction of a T product, the node jumps in FP64.
template <typename T>
void launch_jumps(DevProblem &p, const double *psi, hipStream_t st);
template <typename T>
void launch_correct(DevProblem &p, hipStream_t st);
// n.D grad u+ at the nodes from the T grid values u: FP64 fit weights, jumps and sums, FP64 out.
template <typename T>
void launch_gather(DevProblem &p, const T *u, bool with_jumps, double *out, hipStream_t st);
template <typename T>
void launch_add_correction(DevProblem &p, T *field_padded, hipStream_t st);

// Batched 2D launches: jumps of every problem (crossings and nodes) in one launch; the
// correction into rhs (overwrite, target 0) or fpad (accumulate, target 1); the gather from work.
template <typename T>
void launch_batch_jumps(const BatchItem<T> *items, const BatchCounts &c, const double *psi, hipStream_t st);
template <typename T>
void launch_batch_correct(const BatchItem<T> *items, const BatchCounts &c, int target, hipStream_t st);
template <typename T>
void launch_batch_gather(const BatchItem<T> *items, const BatchCounts &c, bool with_jumps, double *out,
                         hipStream_t st);
// Grouped 2D box solve of G equal-size problems (padded layout, stride cs, msv on the device).
// w: tile widths of the x and last-axis passes (w[0], w[2]).
template <typename T>
void box_solve_group(int Mfft, int G, const T *src, T *dst, int64_t cs, const ModeParams *msv, const T *tw,
                     const T *sp, const int *w, hipStream_t st);
// Merged 2D box solve of several such groups (each with its own size): one launch per pass for
// all groups together, so the tiles of small grids run beside those of large ones instead of in
// launches of their own that cannot fill the GPU.  Sizes 64..1024, tile width 1; the groups are
// those of one precision, src -> dst per group as in box_solve_group.  Results are identical to
// box_solve_group's.
struct MultiGroupDesc {
  int Mfft = 0, G = 0;
  int64_t cs = 0;
  const void *src = nullptr;
  void *dst = nullptr;
  const ModeParams *msv = nullptr;
  const void *tw = nullptr, *sp = nullptr;
};
constexpr int kMaxMultiGroups = 8;
template <typename T>
void box_solve_multi(const MultiGroupDesc *groups, int ngroups, hipStream_t st);
// Autotuner: time each dense pass at both tile widths and keep the faster (cached per process
// by dimension, grid size, components and precision); clears the work buffers afterwards.
void autotune_tiles(DevProblem &p, hipStream_t st);
template <typename T>
void autotune_group(int Mfft, int G, T *a, int64_t cs, const ModeParams *msv, const T *tw, const T *sp, int *w,
                    hipStream_t st);

void upload_tables(DevProblem &p);
void free_tables(DevProblem &p);

}  // namespace kfbi
