// Iterative solver and bidomain driver state (device vectors, FP64 Krylov workspace).
#pragma once
#include "device.h"

namespace kfbi {

struct Mlp;   // learned warm start (mlp.hip)

struct Solver {
  static constexpr int kMaxRestart = 64;
  int64_t L = 0;               // ncomp * M
  int nb = 0;                  // reduction blocks per dot product
  double *V = nullptr;         // (kMaxRestart + 1) * L Krylov basis
  double *r = nullptr, *w = nullptr, *t = nullptr, *gp = nullptr, *d = nullptr;
  double *fpad = nullptr;      // padded FP64 field: source + correction of the final solve
  double *partials = nullptr;  // [vector][block] partial sums
  double *npart = nullptr;     // [block] partials of ||w||^2 from the last Gram-Schmidt pass
  double *hdev = nullptr;      // device dot results (3 * (kMaxRestart + 2))
  double *hhost = nullptr;     // pinned host mirror
  double *ydev = nullptr;      // least-squares coefficients uploaded for the update
  double *ypin = nullptr;      // pinned staging of those coefficients [2][kMaxRestart + 2]
  int64_t n_inside = 0;
  int8_t *inside_plain = nullptr;
  // captured Arnoldi step (per precision of the product), replayed every GMRES iteration
  bool use_graph = true;
  double *vin = nullptr, *wv = nullptr;
  int *jdev = nullptr, *jhost = nullptr;
  // step counter: each replayed step ends by storing its number in pinned host memory, which
  // the host polls instead of sleeping in a stream synchronisation between steps
  int *seqdev = nullptr, *seqhost = nullptr;
  int seq_next = 0;
  void wait_step(hipStream_t st);
  // waits until the stream has run all work enqueued so far (a step counter stored by a tiny
  // kernel, polled; errors are reported through the stream synchronisation it falls back to)
  void host_wait(hipStream_t st);
  hipStream_t cap = nullptr;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  int graph_m[2] = {0, 0};
  void arnoldi_step(DevProblem &p, int prec, int m, hipStream_t st);
  void run_step(DevProblem &p, int prec, int m, hipStream_t st);

  void init(DevProblem &p);
  void release();

  // out = A psi with FP64 vectors; T is the precision of the grid side (correction and box solve),
  // the density side (jumps, extrapolation fits) is FP64 in both
  template <typename T>
  void apply(DevProblem &p, const double *psi, double *out, hipStream_t st);
  // y = A x; prec 1 runs the grid side in FP32
  void apply_vec(DevProblem &p, int prec, const double *x, double *y, hipStream_t st);
  // FP32 vectors at the boundary, converted to and from FP64 around the FP32 product
  void apply_f32(DevProblem &p, const float *psi, float *out, hipStream_t st);

  double dot(const double *a, const double *b, hipStream_t st);
  double residual_norm(const double *b, const double *Ax, hipStream_t st);   // ||b - Ax||_2 (uses d)
  // GMRES(m) with FP64 Arnoldi (CGS2) and Givens rotations on A x = b (stops at ||b - A x|| <= tol_abs);
  // the update is added to x, so x_zero (r = b without a product) requires x to hold zeros.
  // Products in precision a.prec, or with a.relax FP32 once the current residual is <= a.sw_abs and
  // FP64 before: the computed residual of such a solve is then checked by an FP64 product of the
  // result (counted in certs), and the iteration continues from that residual if it misses.
  // a.r0: b - A x already known (no first product).  On return r = b - A x: from the Arnoldi
  // relation (exact to rounding when every product was FP64; the FP32 operator's residual for
  // a.prec = 1), or the FP64 certificate product of a relaxed solve.
  struct GmresArgs {
    int prec = 0;
    bool relax = false;
    double sw_abs = 0;
    const double *r0 = nullptr;
  };
  struct GmresStats {
    int its = 0, mv64 = 0, mv32 = 0, certs = 0;
    double resid = 0, beta0 = 0;
  };
  int gmres(DevProblem &p, const double *b, double bnorm, double *x, bool x_zero, double tol_abs, int restart,
            int maxit, const GmresArgs &a, GmresStats &s, hipStream_t st);
  // the simple iteration; nz (unit, optional): residuals measured without their component along it
  int richardson(DevProblem &p, const double *b, double bnorm, double *x, double gamma, double tol_abs, int maxit,
                 int &its, int &matvecs, double &resid, hipStream_t st, double *r0 = nullptr,
                 const double *nz = nullptr);
  double norm_without(const double *v, const double *nz, hipStream_t st);
  // g' = g - n.D grad (S f)+, with f already in fpad (padded). g may be null.
  // fa: bidomain step (source from V after the forward Euler half step it performs; fpad unused)
  void bie_rhs(DevProblem &p, const double *g, hipStream_t st, const FhnArgs *fa = nullptr);
  // psi solve of A psi = gp with the options; psi holds the start if x0 = 1; r0 (optional) is
  // its residual gp - A psi if already known, unless *r0_bad (pinned host memory, valid after the
  // first wait of the solve) is set, when the residual is computed with an FP64 product.
  // Afterwards last_resid holds gp - A64 psi.
  int solve_density(DevProblem &p, double *psi, const kfbi_solve_opts &o, bool x0, kfbi_solve_info &info,
                    hipStream_t st, const double *r0 = nullptr, const int *r0_bad = nullptr);
  const double *last_resid = nullptr;
  // The coupled pair's null density (insulated tissue: both potentials fixed up to one common
  // constant, so the BIE operator of the pair is singular): the unit eigenvector of A of smallest
  // |eigenvalue|, found once by inverse iteration (null_init, FP64 GMRES solves; it uses the
  // Krylov workspace, so it runs before a solve forms any of its vectors).  The potentials are
  // reconstructed from the density without its component along it: in Omega that changes them
  // by a constant pair (which the gauge removes); outside Omega, where V is evolved too, it
  // removes the field of a component that the near-zero eigenvalue makes large and
  // step-dependent, and that would otherwise feed back through the extended source.
  double *nullz = nullptr, *nully = nullptr, *nullp = nullptr, *nullc = nullptr;
  bool null_ready = false;
  void null_init(DevProblem &p, hipStream_t st);
  // u = S(fpad + C psi) into the padded work buffer (fpad gets the correction added); for the
  // coupled pair psi without its null component (null_init must have run)
  // fa: bidomain step (source from V); fuse_be: the inverse x pass also finishes the step
  // (midpoint update and backward Euler half step), leaving no potentials in work
  void reconstruct(DevProblem &p, const double *psi, hipStream_t st, const FhnArgs *fa = nullptr,
                   bool fuse_be = false);
  double gauge_mean(DevProblem &p, hipStream_t st);   // mean over tissue nodes of comp 1 of work
  int solve_neumann(DevProblem &p, const double *g, const double *f, double *u, double *psi,
                    const kfbi_solve_opts &o, kfbi_solve_info &info, hipStream_t st);
};

}  // namespace kfbi

struct bidomain_s {
  kfbi::DevProblem *prob = nullptr;
  kfbi::Solver *solver = nullptr;
  bidomain_params params{};
  kfbi::Mlp *mlp = nullptr;
  double *psi0 = nullptr;      // start density of the solve
  double *r0v = nullptr;       // its residual, recycled from the previous solve
  double *gp_prev = nullptr;   // BIE right-hand side of the previous step
  double *d_prev = nullptr;    // final FP64 residual g'^{n-1} - A psi^{n-1} of the previous solve
  // the recycled residual belongs to the density of the previous solve: the context keeps its own
  // copy (psi_last) and the history array it was given (hist_last); a step whose psi^{n-1}
  // differs from it at any node (flag set on the device, read by the host) takes the starting
  // residual with an FP64 product instead
  double *psi_last = nullptr;
  const double *hist_last = nullptr;
  double *zdir = nullptr;      // warm_start 4: predicted correction of the start (minimal-residual step)
  int *r0_bad_dev = nullptr, *r0_bad_host = nullptr;
  bool have_prev = false;
  void reset();                // forget the recycled residual, the projection history and the counts
  // projection start: the last kProj solutions psi_j and their images b_j = A psi_j (known
  // without a product: g'_j minus the final residual), with Gram matrix G = B^T B
  static constexpr int kProj = 8;
  double *proj_psi = nullptr, *proj_b = nullptr;   // [kProj][L] rings
  int proj_n = 0, proj_head = 0;
  double proj_G[kProj][kProj] = {};
  void proj_start(double *out_psi, double *out_r, hipStream_t st);
  void proj_record(const double *psi, hipStream_t st);
  int64_t steps_done = 0;
  void init();
  void release();
  int step(bidomain_state &s, double dt, kfbi_solve_info &info, hipStream_t st);
  void mlp_init(int capacity, uint64_t seed);
  double mlp_train(int epochs, double lr, hipStream_t st);
  int mlp_params(float *dst, int64_t *count);
};
